// api.hip -- host side of the C ABI declared in include/atabu.h.
//
// Every call validates its scalar arguments on the host, copies a small
// descriptor table into the caller's device workspace, runs the prepare kernel
// (device-side checks of the instance arrays and the compact travel block),
// reads back the per-instance status, then launches the search.  Nothing is
// allocated except by the server (at_server_*), which owns its memory.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "atabu.h"
#include "atabu_internal.h"

namespace at {

static thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(AT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// Host-side check of one instance's scalars and one parameter set.
int check_scalars(const at_instance *in, const at_params *pr)
{
    if (!in || !pr) return fail(AT_EINVAL, "null instance or params");
    if (in->n_locs < 1 || in->n_locs > kMaxLocs)
        return fail(AT_EINVAL, "n_locs %d outside [1, %d]", in->n_locs, kMaxLocs);
    if (in->n_missions < 0 || in->n_missions > kMaxMissions)
        return fail(AT_EINVAL, "n_missions %d outside [0, %d]", in->n_missions, kMaxMissions);
    if (in->n_vehicles < 1 || in->n_vehicles > kMaxVehicles)
        return fail(AT_EINVAL, "n_vehicles %d outside [1, %d]", in->n_vehicles, kMaxVehicles);
    if (!in->travel || !in->vehicle_loc || (in->n_missions > 0 && (!in->pickup || !in->delivery)))
        return fail(AT_EINVAL, "null instance array");
    if (n_slots(in->n_missions, in->n_vehicles) >= (int64_t(1) << 32))
        return fail(AT_ERANGE, "%lld move slots do not fit 32-bit indices",
                    (long long)n_slots(in->n_missions, in->n_vehicles));
    if (pr->variant != AT_TABU && pr->variant != AT_NS) return fail(AT_EINVAL, "bad variant %d", pr->variant);
    if (pr->tenure < 0) return fail(AT_EINVAL, "negative tenure");
    if (pr->max_iters < 0) return fail(AT_EINVAL, "negative max_iters");
    if ((int64_t)pr->max_iters + pr->tenure + 1 > INT32_MAX) return fail(AT_EINVAL, "max_iters + tenure too large");
    if (pr->block != 0 && pr->block != 256 && pr->block != 512 && pr->block != 1024)
        return fail(AT_EINVAL, "block must be 0, 256, 512 or 1024");
    if (pr->chunk != 0 && (pr->chunk != 8 && pr->chunk != 16 && pr->chunk != 32 && pr->chunk != 64))
        return fail(AT_EINVAL, "chunk must be 0, 8, 16, 32 or 64");
    if (pr->schedule < AT_SCHED_AUTO || pr->schedule > AT_SCHED_GLOBAL) return fail(AT_EINVAL, "bad schedule");
    if (pr->n_groups < 0) return fail(AT_EINVAL, "negative n_groups");
    return AT_OK;
}

// ---------------------------------------------------------------------------
// workspace carving
// ---------------------------------------------------------------------------
struct InstPlan {
    size_t exit_loc, enter_loc, mrow, mcol, vrow, vcol, tc;
    int64_t tc_cap;
};

struct WsPlan {
    size_t xchg, insts, jobs, scal, states, end;
    std::vector<InstPlan> ip;
    std::vector<size_t> st_arrays;   // per job: base of seq|off|tabu
};

static int64_t tc_capacity(const at_instance &in)
{
    const int64_t B = compact_bound(in.n_locs, in.n_missions, in.n_vehicles);
    return B * (B + 4) * 4;
}

static WsPlan plan_ws(int32_t n_inst, const at_instance *insts, int32_t n_jobs, bool with_state)
{
    WsPlan p;
    size_t o = 0;
    p.xchg = o; o = al256(o + sizeof(Xchg));
    p.insts = o; o = al256(o + sizeof(InstDev) * (size_t)n_inst);
    p.ip.resize((size_t)n_inst);
    for (int32_t i = 0; i < n_inst; ++i) {
        const at_instance &in = insts[i];
        InstPlan &q = p.ip[(size_t)i];
        q.exit_loc = o; o = al256(o + 4 * (size_t)in.n_locs);
        q.enter_loc = o; o = al256(o + 4 * (size_t)in.n_locs);
        q.mrow = o; o = al256(o + 4 * (size_t)in.n_missions);
        q.mcol = o; o = al256(o + 4 * (size_t)in.n_missions);
        q.vrow = o; o = al256(o + 4 * (size_t)in.n_vehicles);
        q.vcol = o; o = al256(o + 4 * (size_t)in.n_vehicles);
        q.tc_cap = tc_capacity(in);
        q.tc = o; o = al256(o + (size_t)q.tc_cap);
    }
    p.jobs = o; o = al256(o + sizeof(JobDev) * (size_t)n_jobs);
    p.scal = o; o = al256(o + sizeof(JobScal) * (size_t)n_jobs);
    p.states = o;
    if (with_state) o = al256(o + sizeof(SolveState) * (size_t)n_jobs);
    p.st_arrays.assign((size_t)n_jobs, 0);
    p.end = o;
    return p;
}

static size_t state_bytes(const at_instance &in)
{
    const size_t M = (size_t)in.n_missions, V = (size_t)in.n_vehicles;
    return al256(4 * M) + al256(4 * (V + 1)) + al256(4 * M * V);
}

// ---------------------------------------------------------------------------
// prepare: upload descriptors, run the checks, read back per-instance results
// ---------------------------------------------------------------------------
static int prepare(int32_t n_inst, const at_instance *insts, char *ws, const WsPlan &p,
                   hipStream_t s, std::vector<InstDev> &host)
{
    host.assign((size_t)n_inst, InstDev{});
    for (int32_t i = 0; i < n_inst; ++i) {
        const at_instance &in = insts[i];
        const InstPlan &q = p.ip[(size_t)i];
        InstDev &d = host[(size_t)i];
        d.L = in.n_locs; d.M = in.n_missions; d.V = in.n_vehicles;
        d.T = in.travel; d.p = in.pickup; d.d = in.delivery; d.b = in.vehicle_loc;
        d.exit_loc = (int32_t *)(ws + q.exit_loc);
        d.enter_loc = (int32_t *)(ws + q.enter_loc);
        d.mrow = (int32_t *)(ws + q.mrow);
        d.mcol = (int32_t *)(ws + q.mcol);
        d.vrow = (int32_t *)(ws + q.vrow);
        d.vcol = (int32_t *)(ws + q.vcol);
        d.tc = (void *)(ws + q.tc);
        d.tc_cap = q.tc_cap;
        d.status = AT_EDEVICE;
    }
    InstDev *dev = (InstDev *)(ws + p.insts);
    hipError_t e = hipMemcpyAsync(dev, host.data(), sizeof(InstDev) * (size_t)n_inst,
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "upload instances");
    if ((e = launch_prepare(dev, n_inst, s)) != hipSuccess) return hip_fail(e, "prepare launch");
    if ((e = hipMemcpyAsync(host.data(), dev, sizeof(InstDev) * (size_t)n_inst,
                            hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "read back instances");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "prepare");
    for (int32_t i = 0; i < n_inst; ++i) {
        const InstDev &d = host[(size_t)i];
        if (d.status == AT_EINVAL)
            return fail(AT_EINVAL, "instance %d: mission or vehicle location out of range, or pickup == delivery", i);
        if (d.status == AT_ERANGE)
            return fail(AT_ERANGE, "instance %d: travel time outside [0, 2^27)", i);
        if (d.status != AT_OK) return fail(AT_EDEVICE, "instance %d: prepare status %d", i, d.status);
    }
    return AT_OK;
}

// ---------------------------------------------------------------------------
// schedule
// ---------------------------------------------------------------------------
struct JobHost {
    int inst;
    at_params pr;
    uint64_t seed;
    at_result *out;
    int64_t slots;
    uint32_t lds;
    int tb16, esz16, block, chunk;
};

static int pick_chunk(const at_params &pr, int64_t M)
{
    if (pr.chunk) return pr.chunk;
    return M >= 256 ? 32 : 16;
}

static int pick_block(const at_params &pr, int64_t slots)
{
    if (pr.block) return pr.block;
    if (slots >= 60000) return 1024;
    if (slots >= 8000) return 512;
    return 256;
}

static int fill_job(JobDev &j, const JobHost &h, const InstDev *dev_inst, JobScal *scal)
{
    std::memset(&j, 0, sizeof(j));
    j.inst = dev_inst;
    j.variant = h.pr.variant;
    j.tenure = h.pr.tenure;
    j.max_iters = h.pr.max_iters;
    j.aspiration = h.pr.aspiration ? 1 : 0;
    j.trace = h.pr.trace ? 1 : 0;
    j.t_begin = 0;
    j.t_end = h.pr.max_iters;
    j.tb16 = h.tb16;
    j.chunk = h.chunk;
    j.seed = h.seed;
    j.out_off = h.out->route_off;
    j.out_seq = h.out->route_seq;
    j.out_of = h.out->route_of;
    if (j.trace) {
        j.tr_move = h.out->tr_move;
        j.tr_delta = h.out->tr_delta;
        j.tr_obj = h.out->tr_obj;
        j.tr_flags = h.out->tr_flags;
        if (h.pr.max_iters > 0 && (!j.tr_move || !j.tr_delta || !j.tr_obj || !j.tr_flags))
            return fail(AT_EINVAL, "trace requested but a trace array is null");
    }
    j.scal = scal;
    j.st = nullptr;
    return AT_OK;
}

static int run_jobs(std::vector<JobHost> &jobs, const std::vector<InstDev> &ih, char *ws,
                    const WsPlan &p, hipStream_t s)
{
    const uint32_t lds_max = max_lds_bytes() - 64;
    const InstDev *dev_insts = (const InstDev *)(ws + p.insts);
    JobDev *dj = (JobDev *)(ws + p.jobs);
    JobScal *ds = (JobScal *)(ws + p.scal);
    Xchg *xs = (Xchg *)(ws + p.xchg);
    const int n = (int)jobs.size();
    for (auto &h : jobs) {
        const InstDev &d = ih[(size_t)h.inst];
        h.slots = n_slots(d.M, d.V);
        h.tb16 = ((int64_t)h.pr.max_iters + h.pr.tenure + 1 <= 65535) ? 1 : 0;
        h.esz16 = d.esz == 2 ? 1 : 0;
        h.lds = lds_layout(d.M, d.V, d.R, d.Cs, d.esz, h.tb16 ? 2 : 4).total;
        h.block = pick_block(h.pr, h.slots);
        h.chunk = pick_chunk(h.pr, d.M);
        if (h.lds > lds_max)
            return fail(AT_ENOMEM, "instance %d needs %u bytes of LDS (limit %u); larger instances "
                        "need the HBM-resident schedule", h.inst, h.lds, lds_max);
        if (h.pr.schedule == AT_SCHED_GLOBAL)
            return fail(AT_EINVAL, "the HBM-resident schedule is not available");
    }
    // order: by kernel class (entry width, tabu width), then largest first; the
    // queue of each class hands its jobs out in this order
    std::vector<int> order((size_t)n);
    for (int k = 0; k < n; ++k) order[(size_t)k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const JobHost &x = jobs[(size_t)a], &y = jobs[(size_t)b];
        const int cx = x.esz16 * 2 + x.tb16, cy = y.esz16 * 2 + y.tb16;
        if (cx != cy) return cx < cy;
        return x.slots > y.slots;
    });
    std::vector<JobDev> hj((size_t)n);
    for (int k = 0; k < n; ++k) {
        const JobHost &h = jobs[(size_t)order[(size_t)k]];
        int rc = fill_job(hj[(size_t)k], h, dev_insts + h.inst, ds + order[(size_t)k]);
        if (rc) return rc;
    }
    hipError_t e = hipMemcpyAsync(dj, hj.data(), sizeof(JobDev) * (size_t)n, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "upload jobs");
    if ((e = fill_u32((uint32_t *)ds, 0u, sizeof(JobScal) * (size_t)n / 4, s)) != hipSuccess)
        return hip_fail(e, "clear results");

    const JobHost &h0 = jobs[(size_t)order[0]];
    bool multi = false;
    int groups = 1;
    if (n == 1) {
        if (h0.pr.schedule == AT_SCHED_MULTI) multi = true;
        if (h0.pr.schedule == AT_SCHED_AUTO && h0.slots >= 20000) multi = true;
        if (multi) {
            const int cap = max_groups_multi(h0.block, h0.lds, h0.tb16, h0.esz16);
            groups = h0.pr.n_groups ? h0.pr.n_groups
                                    : (int)std::max<int64_t>(1, std::min<int64_t>(64, h0.slots / 4096));
            groups = std::min(groups, std::min(cap, num_cus()));
            if (groups < 1) return fail(AT_EDEVICE, "cannot co-schedule the multi-workgroup search");
        }
    }
    if (multi) {
        if ((e = fill_u64(xs->key, kKeyNone, 3, s)) != hipSuccess) return hip_fail(e, "reset exchange");
        if ((e = fill_u32(&xs->cnt, 0u, 5, s)) != hipSuccess) return hip_fail(e, "reset exchange");
        if ((e = launch_search_multi(dj, xs, groups, h0.block, h0.lds, h0.tb16, h0.esz16, s)) != hipSuccess)
            return hip_fail(e, "multi-workgroup search launch");
    } else {
        // one launch per kernel class, LDS sized for its largest job
        int k = 0;
        while (k < n) {
            const JobHost &hf = jobs[(size_t)order[(size_t)k]];
            int k1 = k, block = 256;
            uint32_t lds = 0;
            while (k1 < n) {
                const JobHost &h = jobs[(size_t)order[(size_t)k1]];
                if (h.esz16 != hf.esz16 || h.tb16 != hf.tb16) break;
                lds = std::max(lds, h.lds);
                block = std::max(block, h.block);
                ++k1;
            }
            const int count = k1 - k;
            if ((e = fill_u32(&xs->queue, 0u, 1, s)) != hipSuccess) return hip_fail(e, "reset queue");
            const int per_cu = std::max(1, (int)((160 * 1024) / std::max<uint32_t>(lds, 1)));
            const int grid = std::max(1, std::min(count, num_cus() * std::min(per_cu, 8)));
            if ((e = launch_search_wg(dj + k, count, xs, grid, block, lds, hf.tb16, hf.esz16, s)) != hipSuccess)
                return hip_fail(e, "search launch");
            k = k1;
        }
    }
    std::vector<JobScal> hs((size_t)n);
    if ((e = hipMemcpyAsync(hs.data(), ds, sizeof(JobScal) * (size_t)n, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "read back results");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "search");
    int rc = AT_OK;
    for (int k = 0; k < n; ++k) {
        at_result *o = jobs[(size_t)k].out;
        o->best_obj = hs[(size_t)k].best_obj;
        o->final_obj = hs[(size_t)k].final_obj;
        o->iters_done = hs[(size_t)k].iters_done;
        o->best_iter = hs[(size_t)k].best_iter;
        o->status = hs[(size_t)k].status;
        if (o->status != AT_OK && rc == AT_OK) rc = fail(AT_EDEVICE, "solve %d failed on the device (status %d)", k, o->status);
    }
    return rc;
}

}  // namespace at

using namespace at;

extern "C" {

const char *at_last_error(void) { return g_err.c_str(); }

int at_build_travel(int32_t n, const double *lat_deg, const double *lon_deg, double speed_kmh,
                    int32_t *travel, void *stream)
{
    if (n < 1 || n > kMaxLocs) return fail(AT_EINVAL, "n %d outside [1, %d]", n, kMaxLocs);
    if (!(speed_kmh > 0.0) || !std::isfinite(speed_kmh)) return fail(AT_EINVAL, "speed must be positive");
    if (!lat_deg || !lon_deg || !travel) return fail(AT_EINVAL, "null pointer");
    hipError_t e = launch_travel(n, lat_deg, lon_deg, speed_kmh, travel, (hipStream_t)stream);
    return e == hipSuccess ? AT_OK : hip_fail(e, "travel launch");
}

size_t at_workspace_size(int32_t n_inst, const at_instance *insts, const at_params *params,
                         int32_t n_restarts)
{
    if (n_inst < 1 || !insts || !params || n_restarts < 1) return 0;
    for (int32_t i = 0; i < n_inst; ++i)
        if (check_scalars(&insts[i], &params[i]) != AT_OK) return 0;
    const int64_t jobs = (int64_t)n_inst * n_restarts;
    if (jobs > INT32_MAX) return 0;
    WsPlan p = plan_ws(n_inst, insts, (int32_t)jobs, false);
    return p.end;
}

int at_solve_batch(int32_t n_inst, const at_instance *insts, const at_params *params,
                   int32_t n_restarts, void *ws, size_t ws_bytes, void *stream, at_result *out)
{
    if (n_inst < 1 || !insts || !params || !out || n_restarts < 1)
        return fail(AT_EINVAL, "bad batch arguments");
    if (!ws) return fail(AT_EINVAL, "null workspace");
    for (int32_t i = 0; i < n_inst; ++i) {
        int rc = check_scalars(&insts[i], &params[i]);
        if (rc) return rc;
    }
    const int64_t nj = (int64_t)n_inst * n_restarts;
    if (nj > INT32_MAX) return fail(AT_EINVAL, "too many solves");
    WsPlan p = plan_ws(n_inst, insts, (int32_t)nj, false);
    if (ws_bytes < p.end) return fail(AT_ENOMEM, "workspace %zu bytes, need %zu", ws_bytes, p.end);
    for (int64_t k = 0; k < nj; ++k)
        if (!out[k].route_off || (insts[k / n_restarts].n_missions > 0 && !out[k].route_seq))
            return fail(AT_EINVAL, "solve %lld: null route output", (long long)k);
    hipStream_t s = (hipStream_t)stream;
    std::vector<InstDev> ih;
    int rc = prepare(n_inst, insts, (char *)ws, p, s, ih);
    if (rc) return rc;
    std::vector<JobHost> jobs((size_t)nj);
    for (int64_t k = 0; k < nj; ++k) {
        const int i = (int)(k / n_restarts), r = (int)(k % n_restarts);
        JobHost &h = jobs[(size_t)k];
        h.inst = i;
        h.pr = params[i];
        h.seed = r == 0 ? 0 : params[i].restart_seed + (uint64_t)r;
        h.out = &out[k];
    }
    if (nj > 1)
        for (auto &h : jobs) if (h.pr.schedule == AT_SCHED_MULTI) h.pr.schedule = AT_SCHED_AUTO;
    return run_jobs(jobs, ih, (char *)ws, p, s);
}

int at_solve(const at_instance *inst, const at_params *params, void *ws, size_t ws_bytes,
             void *stream, at_result *out)
{
    if (!inst || !params || !out) return fail(AT_EINVAL, "null argument");
    int rc = check_scalars(inst, params);
    if (rc) return rc;
    if (!ws) return fail(AT_EINVAL, "null workspace");
    if (!out->route_off || (inst->n_missions > 0 && !out->route_seq)) return fail(AT_EINVAL, "null route output");
    WsPlan p = plan_ws(1, inst, 1, false);
    if (ws_bytes < p.end) return fail(AT_ENOMEM, "workspace %zu bytes, need %zu", ws_bytes, p.end);
    hipStream_t s = (hipStream_t)stream;
    std::vector<InstDev> ih;
    rc = prepare(1, inst, (char *)ws, p, s, ih);
    if (rc) return rc;
    std::vector<JobHost> jobs(1);
    jobs[0].inst = 0;
    jobs[0].pr = *params;
    jobs[0].seed = params->restart_seed;
    jobs[0].out = out;
    return run_jobs(jobs, ih, (char *)ws, p, s);
}

int at_debug_eval_moves(const at_instance *inst, const at_params *params, const int32_t *route_off,
                        const int32_t *route_seq, const int32_t *tabu_until, int32_t t, int64_t cur,
                        int64_t best, uint64_t *keys_out, void *ws, size_t ws_bytes, void *stream)
{
    if (!inst || !params) return fail(AT_EINVAL, "null argument");
    int rc = check_scalars(inst, params);
    if (rc) return rc;
    if (!route_off || !tabu_until || !keys_out || !ws) return fail(AT_EINVAL, "null pointer");
    if (inst->n_missions < 1) return AT_OK;
    WsPlan p = plan_ws(1, inst, 1, false);
    if (ws_bytes < p.end) return fail(AT_ENOMEM, "workspace %zu bytes, need %zu", ws_bytes, p.end);
    hipStream_t s = (hipStream_t)stream;
    std::vector<InstDev> ih;
    rc = prepare(1, inst, (char *)ws, p, s, ih);
    if (rc) return rc;
    const InstDev &d = ih[0];
    const uint32_t lds = lds_layout(d.M, d.V, d.R, d.Cs, d.esz, 4).total;
    if (lds > max_lds_bytes() - 64) return fail(AT_ENOMEM, "instance too large for the LDS-resident key dump");
    JobHost h;
    h.inst = 0;
    h.pr = *params;
    h.seed = 0;
    at_result dummy;
    std::memset(&dummy, 0, sizeof(dummy));
    dummy.route_off = (int32_t *)route_off;
    dummy.route_seq = (int32_t *)route_seq;
    h.out = &dummy;
    h.pr.trace = 0;
    h.slots = n_slots(d.M, d.V);
    h.chunk = pick_chunk(*params, d.M);
    JobDev j;
    rc = fill_job(j, h, (const InstDev *)((char *)ws + p.insts), (JobScal *)((char *)ws + p.scal));
    if (rc) return rc;
    JobDev *dj = (JobDev *)((char *)ws + p.jobs);
    hipError_t e = hipMemcpyAsync(dj, &j, sizeof(JobDev), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "upload job");
    const int block = params->block ? params->block : 256;
    if ((e = launch_debug_keys(dj, route_off, route_seq, tabu_until, t, cur, best, keys_out, block,
                               lds, d.esz == 2, s)) != hipSuccess)
        return hip_fail(e, "key dump launch");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "key dump");
    return AT_OK;
}

}  // extern "C"
