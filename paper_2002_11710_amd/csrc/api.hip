// api.hip -- host side of the C ABI declared in include/atabu.h (solve, batch,
// travel matrix, key dump).  The serving calls live in server.hip and share
// the engine functions declared in engine.h.
//
// Every call validates its scalar arguments on the host, copies a small
// descriptor table into the caller's device workspace, runs the prepare kernel
// (device-side checks of the instance arrays and the compact travel block),
// reads back the per-instance status, picks a schedule per solve and launches.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <queue>
#include <string>
#include <vector>

#include "atabu.h"
#include "atabu_internal.h"
#include "engine.h"
#include "tuned_table.h"

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

const char *last_error() { return g_err.c_str(); }

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
    if (pr->chunk != 0 && pr->chunk != 4 && pr->chunk != 8 && pr->chunk != 16 && pr->chunk != 32 && pr->chunk != 64)
        return fail(AT_EINVAL, "chunk must be 0, 4, 8, 16, 32 or 64");
    if (pr->schedule < AT_SCHED_AUTO || pr->schedule > AT_SCHED_WAVE) return fail(AT_EINVAL, "bad schedule");
    if (pr->n_groups < 0 || pr->n_groups > 4096) return fail(AT_EINVAL, "n_groups outside [0, 4096]");
    if (pr->form != AT_FORM_BEST && pr->form != AT_FORM_SWEEP) return fail(AT_EINVAL, "bad form %d", pr->form);
    const bool cons = in->travel_plane || in->vehicle_type || in->deadline || in->heli_only || in->flight_limit > 0;
    if (cons || pr->form == AT_FORM_SWEEP || pr->schedule == AT_SCHED_WAVE) {
        if (pr->schedule != AT_SCHED_AUTO && pr->schedule != AT_SCHED_WAVE)
            return fail(AT_EINVAL, "the constrained model and the sweep form run on the wave schedule only");
        if (in->n_missions > kWaveMaxMissions || in->n_vehicles > kWaveMaxVehicles)
            return fail(AT_EINVAL, "the wave schedule takes at most %d missions and %d vehicles",
                        kWaveMaxMissions, kWaveMaxVehicles);
    }
    if (in->deadline && (in->horizon <= 0 || in->horizon > (1 << 29)))
        return fail(AT_EINVAL, "horizon %d outside (0, 2^29]", in->horizon);
    if (in->vehicle_type && !in->travel_plane)
        return fail(AT_EINVAL, "vehicle types need the plane travel matrix");
    return AT_OK;
}

// ---------------------------------------------------------------------------
// sizes
// ---------------------------------------------------------------------------
static int64_t tc_capacity(int L, int M, int V)
{
    const int64_t B = compact_bound(L, M, V);
    return B * (B + 4) * 4;
}

int tabu_bytes(const at_params &pr) { return ((int64_t)pr.max_iters + pr.tenure + 1 <= 65535) ? 2 : 4; }

int ring_slots(const at_params &pr)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)pr.tenure + 1, pr.max_iters));
}

bool may_need_global(const at_instance &in, const at_params &pr)
{
    if (pr.schedule == AT_SCHED_GLOBAL) return true;
    if (in.n_missions >= (1 << 15) || in.n_missions + in.n_vehicles >= (1 << 16)) return true;   // move keys
    const int64_t B = compact_bound(in.n_locs, in.n_missions, in.n_vehicles);
    const uint32_t worst = lds_layout(in.n_missions, in.n_vehicles, (int)B, compact_stride((int)B, 4), 4,
                                      tabu_bytes(pr)).total;
    return worst > kLdsLimit;
}

size_t inst_bytes(const at_instance &in, bool with_t)
{
    size_t o = 0;
    o += al256(4 * (size_t)in.n_locs) * 2;
    o += al256(4 * (size_t)in.n_missions) * 2;
    o += al256(4 * (size_t)in.n_vehicles) * 2;
    o += al256((size_t)tc_capacity(in.n_locs, in.n_missions, in.n_vehicles)) * (with_t ? 3 : 1);
    return o;
}

size_t gstate_bytes(const at_instance &in, const at_params &pr)
{
    return al256(sizeof(GlobalBufs)) + al256(global_state_bytes(in.n_missions, in.n_vehicles, ring_slots(pr)));
}

void carve_inst(InstDev &d, const at_instance &in, char *base, bool with_t)
{
    size_t o = 0;
    d.L = in.n_locs; d.M = in.n_missions; d.V = in.n_vehicles;
    d.T = in.travel; d.p = in.pickup; d.d = in.delivery; d.b = in.vehicle_loc;
    d.exit_loc = (int32_t *)(base + o); o += al256(4 * (size_t)in.n_locs);
    d.enter_loc = (int32_t *)(base + o); o += al256(4 * (size_t)in.n_locs);
    d.mrow = (int32_t *)(base + o); o += al256(4 * (size_t)in.n_missions);
    d.mcol = (int32_t *)(base + o); o += al256(4 * (size_t)in.n_missions);
    d.vrow = (int32_t *)(base + o); o += al256(4 * (size_t)in.n_vehicles);
    d.vcol = (int32_t *)(base + o); o += al256(4 * (size_t)in.n_vehicles);
    d.tc = (void *)(base + o);
    d.tc_cap = tc_capacity(in.n_locs, in.n_missions, in.n_vehicles);
    o += al256((size_t)d.tc_cap);
    d.tct = with_t ? (void *)(base + o) : nullptr;
    d.tcr = with_t ? (void *)(base + o + al256((size_t)d.tc_cap)) : nullptr;
    d.status = AT_EDEVICE;
    d.T2 = in.travel_plane;
    d.vtype = in.vehicle_type;
    d.w = in.deadline;
    d.heli = in.heli_only;
    d.flimit = in.flight_limit > 0 ? in.flight_limit : 0;
    d.horizon = in.deadline ? in.horizon : 0;
}

void carve_gstate(GlobalBufs &g, int M, int V, int n_ring, char *base)
{
    auto a = [](uint64_t x) { return (size_t)((x + 255u) & ~(uint64_t)255u); };
    const uint64_t uM = (uint64_t)M, uV = (uint64_t)V;
    size_t o = al256(sizeof(GlobalBufs));
    for (int k = 0; k < 2; ++k) {
        g.seq[k] = (uint16_t *)(base + o); o += a(2 * uM);
        g.rt[k] = (uint16_t *)(base + o); o += a(2 * uM);
        g.pof[k] = (uint16_t *)(base + o); o += a(2 * uM);
        g.rof[k] = (uint16_t *)(base + o); o += a(2 * uM);
        g.off[k] = (int32_t *)(base + o); o += a(4 * (uV + 1));
    }
    for (int k = 0; k < 2; ++k) {
        g.posA[k] = (int4 *)(base + o); o += a(16 * uM);
        g.posB[k] = (int4 *)(base + o); o += a(16 * uM);
        g.gap[k] = (int4 *)(base + o); o += a(16 * (uM + uV));
        g.posC[k] = (int2 *)(base + o); o += a(8 * uM);
    }
    g.ring = (int4 *)(base + o);
    o += a(32 * (uint64_t)n_ring);
    g.slots = (uint64_t *)(base + o);   // set by the reset before every launch
    g.ring_slots = n_ring;
    g.cur = 0;
    g.abort = 0;
    g.pad2 = 0;
    g.init_obj = 0;
}

struct WsPlan {
    size_t xchg, insts, jobs, scal, states, end;
    std::vector<size_t> inst_off;
    std::vector<size_t> gstate_off;   // per job, 0 = none reserved
};

static WsPlan plan_ws(int32_t n_inst, const at_instance *insts, const at_params *params,
                      int32_t n_restarts)
{
    WsPlan p;
    const int32_t n_jobs = n_inst * n_restarts;
    size_t o = 0;
    p.xchg = o; o = al256(o + sizeof(Xchg));
    p.insts = o; o = al256(o + sizeof(InstDev) * (size_t)n_inst);
    p.inst_off.resize((size_t)n_inst);
    for (int32_t i = 0; i < n_inst; ++i) {
        p.inst_off[(size_t)i] = o;
        o += inst_bytes(insts[i], may_need_global(insts[i], params[i]));
    }
    p.jobs = o; o = al256(o + sizeof(JobDev) * (size_t)n_jobs);
    p.scal = o; o = al256(o + sizeof(JobScal) * (size_t)n_jobs);
    p.states = o; o = al256(o + sizeof(SolveState) * (size_t)n_jobs);
    p.gstate_off.assign((size_t)n_jobs, 0);
    for (int32_t k = 0; k < n_jobs; ++k) {
        const int32_t i = k / n_restarts;
        if (may_need_global(insts[i], params[i])) {
            p.gstate_off[(size_t)k] = o;
            o += gstate_bytes(insts[i], params[i]);
        }
    }
    p.end = o;
    return p;
}

// ---------------------------------------------------------------------------
// prepare: upload descriptors, run the checks, read back per-instance results
// ---------------------------------------------------------------------------
// Enqueue the prepare launches of n_inst instances (device table `dev`, host
// copies `host`, which must stay valid until the stream has passed the
// read-back enqueued here).
int prepare_enqueue(int32_t n_inst, InstDev *dev, InstDev *host, hipStream_t s)
{
    int64_t sc = 0, fc = 0;
    for (int32_t i = 0; i < n_inst; ++i) {
        InstDev &h = host[i];
        int64_t f = 0;
        const int64_t c = prepare_chunks(h, &f);
        h.scan0 = (int32_t)sc;
        h.fill0 = (int32_t)fc;
        sc += c;
        fc += f;
        h.maxT = 0;
        h.scan_bad = 0;
        h.status = AT_EDEVICE;
        if (sc > INT32_MAX || fc > INT32_MAX) return fail(AT_ENOMEM, "too many travel entries in one call");
    }
    hipError_t e = hipMemcpyAsync(dev, host, sizeof(InstDev) * (size_t)n_inst, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "upload instances");
    if ((e = launch_prepare(dev, n_inst, sc, fc, s)) != hipSuccess) return hip_fail(e, "prepare launch");
    if ((e = hipMemcpyAsync(host, dev, sizeof(InstDev) * (size_t)n_inst, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "read back instances");
    return AT_OK;
}

// Status of prepared instances (after the stream has passed prepare_enqueue's read-back).
int prepare_check(int32_t n_inst, const InstDev *host)
{
    for (int32_t i = 0; i < n_inst; ++i) {
        const InstDev &d = host[i];
        if (d.status == AT_EINVAL)
            return fail(AT_EINVAL, "instance %d: mission or vehicle location out of range, or pickup == delivery", i);
        if (d.status == AT_ERANGE)
            return fail(AT_ERANGE, "instance %d: travel time outside [0, 2^23)", i);
        if (d.status != AT_OK) return fail(AT_EDEVICE, "instance %d: prepare status %d", i, d.status);
    }
    return AT_OK;
}

int prepare_instances(int32_t n_inst, InstDev *dev, std::vector<InstDev> &host, hipStream_t s)
{
    int rc = prepare_enqueue(n_inst, dev, host.data(), s);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "prepare");
    return prepare_check(n_inst, host.data());
}

// ---------------------------------------------------------------------------
// schedule
// ---------------------------------------------------------------------------
// Default block size and column chunk by move slots per iteration, from the
// table the autotuner writes (paper_2002_11710_amd/autotune.py).
static int pick_block(const at_params &pr, int64_t slots)
{
    if (pr.block) return pr.block;
    for (const TunedRow &r : kTuned)
        if (slots < r.max_slots) return r.block;
    return 1024;
}

// Whether the tuned table gives solves of this many move slots to the wave
// schedule.
static bool pick_wave(int64_t slots)
{
    for (const TunedRow &r : kTuned)
        if (slots < r.max_slots) return r.wave != 0;
    return false;
}

static int pick_chunk(const at_params &pr, int64_t slots)
{
    if (pr.chunk) return pr.chunk;
    for (const TunedRow &r : kTuned)
        if (slots < r.max_slots) return r.chunk;
    return 32;
}

// Missions per block of a global-schedule job for its group count: one block
// per workgroup where LDS allows, else the LDS limit.
void set_block_size(JobHost &h)
{
    // as few rounds of blocks as LDS allows, then the smallest blocks with that many rounds
    const int64_t g = std::max(1, h.groups);
    const int64_t rounds = std::max<int64_t>(1, (h.dM + g * h.gkmax - 1) / (g * h.gkmax));
    const int per = (int)((h.dM + rounds * g - 1) / (rounds * g));
    h.gk = std::max(1, std::min(h.gkmax, per));
    h.lds = global_lds_bytes(h.gk, h.dR, h.dC, h.dM, h.dV, h.desz, h.tb16 ? 2 : 4);
}

// Wave schedule: one wavefront per solve (the constrained model, the sweep
// form, or a small unconstrained solve the tuned table gives to it).
static int plan_wave(JobHost &h, const InstDev &d)
{
    const bool two = d.T2 != nullptr;
    const int esz = constrained(d) ? 4 : d.esz;
    h.kind = AT_SCHED_WAVE;
    h.wtile = !constrained(d) && h.pr.form == AT_FORM_BEST;
    if (h.wtile) {
        // the unconstrained best form: the one-workgroup schedule's code on one wavefront
        if (d.M >= (1 << 15) || d.M + d.V >= (1 << 16))
            return fail(AT_ENOMEM, "instance too large for the wave schedule (%d missions, %d vehicles)", d.M, d.V);
        h.tb16 = tabu_bytes(h.pr) == 2 ? 1 : 0;
        h.esz16 = d.esz == 2 ? 1 : 0;
        h.lds = lds_layout(d.M, d.V, d.R, d.Cs, d.esz, h.tb16 ? 2 : 4).total;
        h.chunk = pick_chunk(h.pr, h.slots);
        h.rchunk = std::min(64, 2 * h.chunk);
        h.groups = 1;
        h.block = kWave;
        if (h.lds > kLdsLimit)
            return fail(AT_ENOMEM, "instance too large for the wave schedule (%u bytes of LDS per solve)", h.lds);
        return AT_OK;
    }
    h.esz16 = esz == 2 ? 1 : 0;
    h.tb16 = 0;
    h.lds = wave_lds_bytes(d.M, d.V, d.R, d.Cs, esz, two);
    h.groups = 1;
    h.block = kWave;
    if (h.lds > kLdsLimit)
        return fail(AT_ENOMEM, "instance too large for the wave schedule (%u bytes of LDS per solve)", h.lds);
    return AT_OK;
}

int plan_job(JobHost &h, const InstDev &d, bool alone)
{
    h.slots = n_slots(d.M, d.V);
    if (constrained(d) || h.pr.form == AT_FORM_SWEEP || h.pr.schedule == AT_SCHED_WAVE) {
        if (h.chunked) return fail(AT_EINVAL, "served requests run the best form on the unconstrained model");
        return plan_wave(h, d);
    }
    h.tb16 = tabu_bytes(h.pr) == 2 ? 1 : 0;
    h.esz16 = d.esz == 2 ? 1 : 0;
    h.lds = lds_layout(d.M, d.V, d.R, d.Cs, d.esz, h.tb16 ? 2 : 4).total;
    h.block = pick_block(h.pr, h.slots);
    h.chunk = pick_chunk(h.pr, h.slots);
    // relocate units twice as wide as swap units: a swap column costs about twice a
    // relocate column (measured on gfx950: 5% more batch throughput than equal widths)
    h.rchunk = std::min(64, 2 * h.chunk);
    h.groups = 1;
    // the LDS-resident schedules pack a move as mission << 16 | gap (M < 2^15,
    // M + V < 2^16); LDS itself runs out long before
    const bool lds_keys = d.M < (1 << 15) && d.M + d.V < (1 << 16);
    if (h.pr.schedule == AT_SCHED_GLOBAL || h.lds > kLdsLimit || !lds_keys) {
        if (!h.gstate) return fail(AT_ENOMEM, "solve needs the HBM-resident schedule but no state was reserved");
        h.kind = AT_SCHED_GLOBAL;
        // a requested block size above the schedule's limit applies to the other schedules only
        h.block = h.pr.block ? std::min(h.pr.block, kGlobalBlock) : kGlobalBlock;
        if (!d.tct) return fail(AT_ENOMEM, "solve needs the HBM-resident schedule but its transposed block was not reserved");
        const int g = h.pr.n_groups ? h.pr.n_groups
                                    : (int)std::max<int64_t>(1, std::min<int64_t>(num_cus(), h.slots / 16384));
        h.dM = d.M; h.dV = d.V; h.dR = d.R; h.dC = d.C; h.desz = d.esz;
        // the most missions per block that LDS holds (the block size itself is set
        // with the final group count: one block per workgroup where LDS allows)
        h.gkmax = 0;
        for (int K = kGlobalKMax; K >= 1; --K)
            if (global_lds_bytes(K, d.R, d.C, d.M, d.V, d.esz, h.tb16 ? 2 : 4) <= kLdsLimit) { h.gkmax = K; break; }
        if (!h.gkmax) return fail(AT_ENOMEM, "instance too large: %d exit and %d entry locations do not fit the staged search", d.R, d.C);
        h.lds = global_lds_bytes(h.gkmax, d.R, d.C, d.M, d.V, d.esz, h.tb16 ? 2 : 4);
        const int cap = max_groups_global(h.block, h.lds, h.tb16, h.esz16);
        if (cap < 1) return fail(AT_EDEVICE, "cannot co-schedule the HBM-resident search");
        h.groups = std::max(1, std::min(g, cap));
        set_block_size(h);
        return AT_OK;
    }
    h.kind = AT_SCHED_WG;
    if (!h.chunked && h.pr.schedule == AT_SCHED_AUTO && pick_wave(h.slots) &&
        lds_layout(d.M, d.V, d.R, d.Cs, d.esz, tabu_bytes(h.pr)).total <= kLdsLimit / 2)
        return plan_wave(h, d);
    if (alone && multi_eligible(h)) return plan_multi(h, d);
    return AT_OK;
}

// Whether a solve planned on one workgroup may run on the multi-workgroup
// schedule instead: asked for it, or large enough under AUTO.
bool multi_eligible(const JobHost &h)
{
    return h.kind == AT_SCHED_WG && !h.wtile &&
           (h.pr.schedule == AT_SCHED_MULTI || (h.pr.schedule == AT_SCHED_AUTO && h.slots >= kMultiMinSlots));
}

// The multi-workgroup plan of a solve whose state fits one workgroup's LDS:
// measured on gfx950 (16 x 400 missions): 512 threads, 8-column swap units
// (16-column relocate units), one wavefront per work unit (the iteration waits
// for the wavefront with the most work), up to 96 workgroups (more slots to poll
// cost more than the eval saves).  One solve alone: workgroups [0, groups),
// slot set 0.
int plan_multi(JobHost &h, const InstDev &d, bool small_units)
{
    if (!h.pr.block) h.block = 512;
    const int cap = max_groups_multi(h.block, h.lds, h.tb16, h.esz16);
    const int64_t waves = std::max(1, h.block / kWave);
    auto units_of = [&](int ch) {
        const int rch = std::min(64, 2 * ch);
        int64_t u = 0;
        for (int64_t jb = 0; jb < d.M; jb += kWave)
            u += (d.M + d.V + rch - 1) / rch + (d.M - jb + ch - 1) / ch;
        return u;
    };
    // the iteration waits for the slowest unit: half-width units (4 partners, 8
    // gaps) while they still leave every wavefront at most one unit at the group
    // limit, else 8-partner units
    if (!h.pr.chunk)
        h.chunk = (small_units && units_of(4) <= (int64_t)kMultiMaxGroups * waves) ? 4 : 8;
    h.rchunk = std::min(64, 2 * h.chunk);
    const int64_t units = units_of(h.chunk);
    int g = h.pr.n_groups ? h.pr.n_groups
                          : (int)std::max<int64_t>(1, std::min<int64_t>(kMultiMaxGroups, (units + waves - 1) / waves));
    g = std::min(g, std::min(std::min(cap, num_cus()), kMaxGroups));
    if (g < 1) return fail(AT_EDEVICE, "cannot co-schedule the multi-workgroup search");
    h.kind = AT_SCHED_MULTI;
    h.groups = g;
    h.g0 = 0;
    h.mx = 0;
    h.launch = 0;
    return AT_OK;
}

// A batch of at most kMaxMultiJobs solves, each large and fitting one
// workgroup's LDS (all of one entry and tabu width): one cooperative launch of
// the multi-workgroup schedule runs them side by side, each on its own range of
// workgroups and its own slot set; a workgroup per solve would leave most of the
// GPU idle.  Each asks for what it would take alone; when the sum exceeds what
// the GPU holds, the shares shrink in proportion (at least one each).  Leaves
// the jobs as they are when the batch does not qualify.
int plan_multi_batch(std::vector<JobHost> &jobs, const std::vector<InstDev> &ih)
{
    const int n = (int)jobs.size();
    if (n < 2 || n > kMaxMultiJobs) return AT_OK;
    for (const JobHost &h : jobs)
        if (!multi_eligible(h) || h.tb16 != jobs[0].tb16 || h.esz16 != jobs[0].esz16) return AT_OK;
    std::vector<JobHost> m;
    uint32_t lds = 0;
    int64_t want = 0;
    int cap = 0;
    // half-width units only while every solve keeps the groups it asks for
    for (const bool small_units : {true, false}) {
        m = jobs;
        lds = 0;
        want = 0;
        for (JobHost &h : m) {
            int rc = plan_multi(h, ih[(size_t)h.inst], small_units);
            if (rc) return rc;
            if (h.block != m[0].block) return AT_OK;
            lds = std::max(lds, h.lds);
            want += h.groups;
        }
        cap = max_groups_multi(m[0].block, lds, m[0].tb16, m[0].esz16);
        if (want <= cap) break;
    }
    if (cap < n) return AT_OK;
    if (want > cap) {
        // scale to the co-resident limit; the floor of 1 can overshoot it by a few groups,
        // which come off the largest jobs (cap >= n, so every job keeps one)
        int64_t sum = 0;
        for (JobHost &h : m) {
            h.groups = std::max(1, (int)((int64_t)h.groups * cap / want));
            sum += h.groups;
        }
        while (sum > cap) {
            JobHost *big = &m[0];
            for (JobHost &h : m)
                if (h.groups > big->groups) big = &h;
            --big->groups;
            --sum;
        }
    }
    int g0 = 0;
    for (int k = 0; k < n; ++k) {
        JobHost &h = m[(size_t)k];
        h.g0 = g0;
        h.mx = k;
        g0 += h.groups;
    }
    jobs.swap(m);
    return AT_OK;
}

int fill_job(JobDev &j, const JobHost &h, const InstDev *dev_inst, JobScal *scal)
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
    j.rchunk = h.rchunk;
    j.seed = h.seed;
    j.out_off = h.out.route_off;
    j.out_seq = h.out.route_seq;
    j.out_of = h.out.route_of;
    j.fin_off = h.out.final_off;
    j.fin_seq = h.out.final_off ? h.out.final_seq : nullptr;
    if (j.trace) {
        j.tr_move = h.out.tr_move;
        j.tr_delta = h.out.tr_delta;
        j.tr_obj = h.out.tr_obj;
        j.tr_flags = h.out.tr_flags;
        if (h.pr.max_iters > 0 && (!j.tr_move || !j.tr_delta || !j.tr_obj || !j.tr_flags))
            return fail(AT_EINVAL, "trace requested but a trace array is null");
    }
    j.scal = scal;
    j.st = nullptr;
    j.gb = h.gstate;
    j.form = h.pr.form;
    j.gk = h.gk;
    j.g0 = h.g0;
    j.ng = h.groups;
    j.sched = h.kind;
    j.mx = h.mx;
    return AT_OK;
}

// Upload GlobalBufs pointer tables for the jobs on the global schedule.
int upload_gstates(const std::vector<JobHost> &jobs, const std::vector<InstDev> &ih, hipStream_t s)
{
    // the host copies are the copy sources: they live until the synchronisation below
    std::vector<GlobalBufs> host;
    host.reserve(jobs.size());
    for (const auto &h : jobs) {
        if (h.kind != AT_SCHED_GLOBAL) continue;
        host.emplace_back();
        carve_gstate(host.back(), ih[(size_t)h.inst].M, ih[(size_t)h.inst].V, ring_slots(h.pr), (char *)h.gstate);
        hipError_t e = hipMemcpyAsync(h.gstate, &host.back(), sizeof(GlobalBufs), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "upload state tables");
    }
    if (host.empty()) return AT_OK;
    hipError_t e = hipStreamSynchronize(s);
    return e == hipSuccess ? AT_OK : hip_fail(e, "upload state tables");
}

// Internal streams on which the one-workgroup-per-job launches of different
// size classes run concurrently (forked from and joined back to the caller's
// stream with events).  Default priority, created once.
static hipStream_t g_class_pool[kMaxClasses] = {};

static hipStream_t class_stream(int k)
{
    if (!g_class_pool[k] && hipStreamCreateWithFlags(&g_class_pool[k], hipStreamNonBlocking) != hipSuccess) {
        g_class_pool[k] = nullptr;
        return nullptr;
    }
    return g_class_pool[k];
}

// Destroy the class streams (at_shutdown): each is synchronised first.
int release_class_streams()
{
    int rc = AT_OK;
    for (int k = 0; k < kMaxClasses; ++k) {
        if (!g_class_pool[k]) continue;
        hipError_t e = hipStreamSynchronize(g_class_pool[k]);
        if (e == hipSuccess) e = hipStreamDestroy(g_class_pool[k]);
        if (e != hipSuccess && rc == AT_OK) rc = hip_fail(e, "class stream release");
        g_class_pool[k] = nullptr;
    }
    return rc;
}

// Launch every job of `dj` (device table in the order of `order`).  Jobs of
// the one-workgroup schedule share one persistent launch per class (entry
// width, tabu width, block size); the classes run concurrently on internal
// streams.  Then, in order on the caller's stream: one cooperative launch per
// group of HBM-resident jobs that assign_groups put together (each job on its
// own range of the grid), and one cooperative launch per multi-workgroup job.
int launch_jobs(const std::vector<JobHost> &jobs, const std::vector<int> &order, JobDev *dj,
                Xchg *xs, hipStream_t s)
{
    hipError_t e;
    const int n = (int)order.size();
    struct Cls { int k0, k1, kind, block, tb16, esz16; bool wtile; uint32_t lds; };
    std::vector<Cls> cls;
    int k = 0;
    auto one_per_solve = [](int kind) { return kind == AT_SCHED_WG || kind == AT_SCHED_WAVE; };
    while (k < n && one_per_solve(jobs[(size_t)order[(size_t)k]].kind)) {
        const JobHost &hf = jobs[(size_t)order[(size_t)k]];
        Cls c{k, k, hf.kind, hf.block, hf.tb16, hf.esz16, hf.wtile, 0};
        while (c.k1 < n) {
            const JobHost &h = jobs[(size_t)order[(size_t)c.k1]];
            if (h.kind != hf.kind || h.esz16 != hf.esz16 || h.tb16 != hf.tb16 || h.block != hf.block ||
                h.wtile != hf.wtile)
                break;
            c.lds = std::max(c.lds, h.lds);
            ++c.k1;
        }
        cls.push_back(c);
        k = c.k1;
    }
    if ((int)cls.size() > kMaxClasses) return fail(AT_EINVAL, "too many launch classes");
    // the HBM-resident launches of the global jobs that assign_groups put together,
    // in order on stream `st`
    auto launch_globals = [&](int k0, hipStream_t st) -> int {
        for (int q = k0; q < n;) {
            const JobHost &hf = jobs[(size_t)order[(size_t)q]];
            if (hf.kind != AT_SCHED_GLOBAL) return fail(AT_EINVAL, "job order: a global job after the others expected");
            int e1 = q, groups = 0;
            uint32_t lds = 0;
            while (e1 < n && jobs[(size_t)order[(size_t)e1]].kind == AT_SCHED_GLOBAL &&
                   jobs[(size_t)order[(size_t)e1]].launch == hf.launch) {
                const JobHost &h = jobs[(size_t)order[(size_t)e1]];
                groups = std::max(groups, h.g0 + h.groups);
                lds = std::max(lds, h.lds);
                ++e1;
            }
            hipError_t e2 = launch_search_global(dj + q, e1 - q, groups, hf.block, lds, hf.tb16, hf.esz16, st);
            if (e2 != hipSuccess) return hip_fail(e2, "search launch (HBM-resident schedule)");
            q = e1;
        }
        return AT_OK;
    };
    if (!cls.empty()) {
        if ((e = fill_u32(xs->queues, 0u, kMaxClasses, s)) != hipSuccess) return hip_fail(e, "reset queues");
        hipEvent_t fork = nullptr;
        std::vector<hipEvent_t> joins(cls.size(), nullptr);
        const bool split = cls.size() > 1;
        int rc = AT_OK;
        if (split) {
            if ((e = hipEventCreateWithFlags(&fork, hipEventDisableTiming)) != hipSuccess ||
                (e = hipEventRecord(fork, s)) != hipSuccess)
                rc = hip_fail(e, "event");
        }
        for (size_t c = 0; c < cls.size() && rc == AT_OK; ++c) {
            const Cls &q = cls[c];
            hipStream_t st = s;
            if (split) {
                st = class_stream((int)c);
                if (!st) { rc = fail(AT_EDEVICE, "cannot create a class stream"); break; }
            }
            if (split && (e = hipStreamWaitEvent(st, fork, 0)) != hipSuccess) { rc = hip_fail(e, "fork"); break; }
            const int count = q.k1 - q.k0;
            if (q.kind == AT_SCHED_WAVE) {
                // up to four solves (wavefronts) per workgroup, as many workgroups per CU as
                // LDS holds
                const uint32_t per = std::max<uint32_t>(q.lds, 16);
                const int wpg = (int)std::max<uint32_t>(1, std::min<uint32_t>(4, kLdsLimit / per));
                const int by_lds = std::max(1, (int)((kLdsLimit + 64) / (per * (uint32_t)wpg)));
                const int per_cu = std::min(by_lds, 16 / wpg);
                const int grid = std::max(1, std::min((count + wpg - 1) / wpg, num_cus() * per_cu));
                e = q.wtile ? launch_search_wg_wave(dj + q.k0, count, &xs->queues[c], grid, wpg, per, q.tb16,
                                                    q.esz16, st)
                            : launch_search_wave(dj + q.k0, count, &xs->queues[c], grid, wpg, per, q.esz16, st);
            } else {
                const int by_lds = std::max(1, (int)((kLdsLimit + 64) / std::max<uint32_t>(q.lds, 1)));
                const int by_waves = std::max(1, 16 * kWave / q.block);
                const int per_cu = std::min(by_lds, by_waves);
                const int grid = std::max(1, std::min(count, num_cus() * per_cu));
                e = launch_search_wg(dj + q.k0, count, &xs->queues[c], grid, q.block, q.lds, q.tb16, q.esz16, st);
            }
            if (e != hipSuccess) {
                rc = hip_fail(e, "search launch");
                break;
            }
            if (split) {
                if ((e = hipEventCreateWithFlags(&joins[c], hipEventDisableTiming)) != hipSuccess ||
                    (e = hipEventRecord(joins[c], st)) != hipSuccess ||
                    (e = hipStreamWaitEvent(s, joins[c], 0)) != hipSuccess) {
                    rc = hip_fail(e, "join");
                    break;
                }
            }
        }
        if (fork) (void)hipEventDestroy(fork);
        for (hipEvent_t ev : joins) if (ev) (void)hipEventDestroy(ev);
        if (rc) return rc;
    }
    while (k < n) {
        const JobHost &hf = jobs[(size_t)order[(size_t)k]];
        if (hf.kind == AT_SCHED_GLOBAL) {
            // the global jobs, which come last: one cooperative launch per group of them
            return launch_globals(k, s);
        }
        // the multi-workgroup solves planned into one launch (consecutive, slot sets 0..)
        int e1 = k, groups = 0;
        uint32_t lds = 0;
        while (e1 < n && e1 - k < kMaxMultiJobs && jobs[(size_t)order[(size_t)e1]].kind == AT_SCHED_MULTI &&
               jobs[(size_t)order[(size_t)e1]].launch == hf.launch && jobs[(size_t)order[(size_t)e1]].mx == e1 - k) {
            const JobHost &h = jobs[(size_t)order[(size_t)e1]];
            groups = std::max(groups, h.g0 + h.groups);
            lds = std::max(lds, h.lds);
            ++e1;
        }
        if ((e = fill_u64(&xs->slots[0][0][0], 1ull << 63, (size_t)(e1 - k) * 2 * kMaxGroups * kSlotStride, s)) !=
            hipSuccess)
            return hip_fail(e, "reset exchange");
        e = launch_search_multi(dj + k, e1 - k, xs, groups, hf.block, lds, hf.tb16, hf.esz16, s);
        if (e != hipSuccess) return hip_fail(e, "cooperative search launch");
        k = e1;
    }
    return AT_OK;
}

// Order jobs: one-workgroup jobs grouped by launch class (entry width, tabu
// width, block), largest first inside a class (its queue hands jobs out in
// this order), then the cooperative ones.
std::vector<int> order_jobs(const std::vector<JobHost> &jobs)
{
    const int n = (int)jobs.size();
    std::vector<int> order((size_t)n);
    for (int k = 0; k < n; ++k) order[(size_t)k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const JobHost &x = jobs[(size_t)a], &y = jobs[(size_t)b];
        // one-solve-per-group kinds first (wave, then workgroup), then the cooperative ones
        auto grp = [](int kind) { return kind == AT_SCHED_WAVE ? 0 : kind == AT_SCHED_WG ? 1 : kind; };
        const int cx = grp(x.kind), cy = grp(y.kind);
        if (cx != cy) return cx < cy;
        // multi-workgroup solves of one launch in the order of their workgroup ranges
        // (the kernel finds a workgroup's solve by binary search over them)
        if (x.kind == AT_SCHED_MULTI) return x.g0 < y.g0;
        if (x.kind == AT_SCHED_WG || x.kind == AT_SCHED_GLOBAL || x.kind == AT_SCHED_WAVE) {
            const int kx = ((x.wtile * 2 + x.esz16) * 2 + x.tb16) * 4096 + x.block;
            const int ky = ((y.wtile * 2 + y.esz16) * 2 + y.tb16) * 4096 + y.block;
            if (kx != ky) return kx > ky;
        }
        return x.slots > y.slots;
    });
    return order;
}

// Split the global-schedule jobs (consecutive in `order`, grouped by class)
// into cooperative launches and give each job a range of its launch's
// workgroups: as many as it asked for when they all fit the co-resident
// limit, else shares proportional to the request (at least one each).
int assign_groups(std::vector<JobHost> &jobs, const std::vector<int> &order)
{
    const int n = (int)order.size();
    int k = 0, launch = 0;
    while (k < n && jobs[(size_t)order[(size_t)k]].kind != AT_SCHED_GLOBAL) ++k;
    while (k < n && jobs[(size_t)order[(size_t)k]].kind == AT_SCHED_GLOBAL) {
        const JobHost &hf = jobs[(size_t)order[(size_t)k]];
        int e = k;
        uint32_t lds = 0;
        while (e < n) {
            const JobHost &h = jobs[(size_t)order[(size_t)e]];
            if (h.kind != AT_SCHED_GLOBAL || h.esz16 != hf.esz16 || h.tb16 != hf.tb16 || h.block != hf.block) break;
            lds = std::max(lds, h.lds);
            ++e;
        }
        const int cap = max_groups_global(hf.block, lds, hf.tb16, hf.esz16);
        if (cap < 1) return fail(AT_EDEVICE, "cannot co-schedule the HBM-resident search");
        for (int a = k; a < e; a += cap, ++launch) {
            const int b = std::min(e, a + cap);
            int64_t want = 0;
            for (int q = a; q < b; ++q) want += jobs[(size_t)order[(size_t)q]].groups;
            if (want > cap) {
                // A job's launch time is about iters x (slots / groups + c): the move slots
                // its groups share plus a per-iteration cost (apply, prep and two barriers)
                // worth about c move slots of one workgroup, measured on gfx950.  Starting
                // from one group each, every further group goes to the job that would
                // finish last, up to what the job asked for; this minimises the launch's
                // longest job, where shares proportional to work lose most to rounding
                // when a job's share is a few groups.
                constexpr double kIterSlots = 12288.0;
                const int nq = b - a;
                std::vector<int> give((size_t)nq, 1);
                auto span = [&](int i) {
                    const JobHost &h = jobs[(size_t)order[(size_t)(a + i)]];
                    const double it = (double)std::max<int64_t>(1, h.iters);
                    return it * ((double)h.slots / (double)give[(size_t)i] + kIterSlots);
                };
                std::priority_queue<std::pair<double, int>> pq;
                for (int i = 0; i < nq; ++i)
                    if (jobs[(size_t)order[(size_t)(a + i)]].groups > 1) pq.push({span(i), i});
                for (int left = cap - nq; left > 0 && !pq.empty(); --left) {
                    const int i = pq.top().second;
                    pq.pop();
                    ++give[(size_t)i];
                    if (give[(size_t)i] < jobs[(size_t)order[(size_t)(a + i)]].groups) pq.push({span(i), i});
                }
                for (int i = 0; i < nq; ++i) jobs[(size_t)order[(size_t)(a + i)]].groups = give[(size_t)i];
            }
            int g0 = 0;
            for (int q = a; q < b; ++q) {
                JobHost &h = jobs[(size_t)order[(size_t)q]];
                int g = std::min(h.groups, cap - g0 - (b - q - 1));   // leave one for each later job
                h.groups = std::max(1, g);
                h.g0 = g0;
                h.launch = launch;
                g0 += h.groups;
                set_block_size(h);
            }
        }
        k = e;
    }
    return AT_OK;
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t create()
    {
        hipError_t e = hipEventCreate(&a);
        return e != hipSuccess ? e : hipEventCreate(&b);
    }
    ~EventPair()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

static int run_jobs(std::vector<JobHost> &jobs, const std::vector<InstDev> &ih, char *ws,
                    const WsPlan &p, hipStream_t s, at_result *const *outs, bool timed)
{
    const InstDev *dev_insts = (const InstDev *)(ws + p.insts);
    JobDev *dj = (JobDev *)(ws + p.jobs);
    JobScal *ds = (JobScal *)(ws + p.scal);
    Xchg *xs = (Xchg *)(ws + p.xchg);
    const int n = (int)jobs.size();
    for (auto &h : jobs) {
        int rc = plan_job(h, ih[(size_t)h.inst], n == 1);
        if (rc) return rc;
        h.iters = h.pr.max_iters;
    }
    int rc = plan_multi_batch(jobs, ih);
    if (rc) return rc;
    rc = upload_gstates(jobs, ih, s);
    if (rc) return rc;
    const std::vector<int> order = order_jobs(jobs);
    if ((rc = assign_groups(jobs, order)) != AT_OK) return rc;
    std::vector<JobDev> hj((size_t)n);
    for (int k = 0; k < n; ++k) {
        const JobHost &h = jobs[(size_t)order[(size_t)k]];
        rc = fill_job(hj[(size_t)k], h, dev_insts + h.inst, ds + order[(size_t)k]);
        if (rc) return rc;
    }
    hipError_t e = hipMemcpyAsync(dj, hj.data(), sizeof(JobDev) * (size_t)n, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "upload jobs");
    if ((e = fill_u32((uint32_t *)ds, 0u, sizeof(JobScal) * (size_t)n / 4, s)) != hipSuccess)
        return hip_fail(e, "clear results");
    EventPair ev;
    if (timed) {
        if ((e = ev.create()) != hipSuccess) return hip_fail(e, "event create");
        if ((e = hipEventRecord(ev.a, s)) != hipSuccess) return hip_fail(e, "event record");
    }
    rc = launch_jobs(jobs, order, dj, xs, s);
    if (rc) return rc;
    if (timed && (e = hipEventRecord(ev.b, s)) != hipSuccess) return hip_fail(e, "event record");
    std::vector<JobScal> hs((size_t)n);
    if ((e = hipMemcpyAsync(hs.data(), ds, sizeof(JobScal) * (size_t)n, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "read back results");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "search");
    float ms = 0.f;
    if (timed && (e = hipEventElapsedTime(&ms, ev.a, ev.b)) != hipSuccess) return hip_fail(e, "event time");
    rc = AT_OK;
    for (int k = 0; k < n; ++k) {
        at_result *o = outs[k];
        o->search_ms = ms;
        o->best_obj = hs[(size_t)k].best_obj;
        o->final_obj = hs[(size_t)k].final_obj;
        o->iters_done = hs[(size_t)k].iters_done;
        o->best_iter = hs[(size_t)k].best_iter;
        o->status = hs[(size_t)k].status;
        if (o->status == AT_EINFEAS && rc == AT_OK)
            rc = fail(AT_EINFEAS, "solve %d: Algorithm 1 found no feasible start", k);
        else if ((o->status == AT_EINVAL || o->status == AT_ERANGE) && rc == AT_OK)
            rc = fail(o->status, "solve %d: a constrained-model input is out of range", k);
        else if (o->status != AT_OK && rc == AT_OK)
            rc = fail(AT_EDEVICE, "solve %d failed on the device (status %d)", k, o->status);
    }
    return rc;
}

static int solve_common(int32_t n_inst, const at_instance *insts, const at_params *params,
                        int32_t n_restarts, void *ws, size_t ws_bytes, void *stream, at_result *out,
                        bool single, bool timed = true)
{
    for (int32_t i = 0; i < n_inst; ++i) {
        int rc = check_scalars(&insts[i], &params[i]);
        if (rc) return rc;
    }
    if (!ws) return fail(AT_EINVAL, "null workspace");
    const int64_t nj = (int64_t)n_inst * n_restarts;
    if (nj > (1 << 24)) return fail(AT_EINVAL, "too many solves in one call");
    for (int64_t k = 0; k < nj; ++k)
        if (!out[k].route_off || (insts[k / n_restarts].n_missions > 0 && !out[k].route_seq))
            return fail(AT_EINVAL, "solve %lld: null route output", (long long)k);
    for (int64_t k = 0; k < nj; ++k)
        if (out[k].final_off && insts[k / n_restarts].n_missions > 0 && !out[k].final_seq)
            return fail(AT_EINVAL, "solve %lld: final_off without final_seq", (long long)k);
    WsPlan p = plan_ws(n_inst, insts, params, n_restarts);
    if (ws_bytes < p.end) return fail(AT_ENOMEM, "workspace %zu bytes, need %zu", ws_bytes, p.end);
    hipStream_t s = (hipStream_t)stream;
    char *base = (char *)ws;
    std::vector<InstDev> ih((size_t)n_inst);
    for (int32_t i = 0; i < n_inst; ++i)
        carve_inst(ih[(size_t)i], insts[i], base + p.inst_off[(size_t)i], may_need_global(insts[i], params[i]));
    int rc = prepare_instances(n_inst, (InstDev *)(base + p.insts), ih, s);
    if (rc) return rc;
    std::vector<JobHost> jobs((size_t)nj);
    std::vector<at_result *> outs((size_t)nj);
    for (int64_t k = 0; k < nj; ++k) {
        const int i = (int)(k / n_restarts), r = (int)(k % n_restarts);
        JobHost &h = jobs[(size_t)k];
        h.inst = i;
        h.pr = params[i];
        h.seed = single ? params[i].restart_seed : (r == 0 ? 0 : params[i].restart_seed + (uint64_t)r);
        h.out = out[k];
        h.gstate = p.gstate_off[(size_t)k] ? (GlobalBufs *)(base + p.gstate_off[(size_t)k]) : nullptr;
        if (nj > 1 && h.pr.schedule == AT_SCHED_MULTI) h.pr.schedule = AT_SCHED_AUTO;
        outs[(size_t)k] = &out[k];
    }
    return run_jobs(jobs, ih, base, p, s, outs.data(), timed);
}

// ---------------------------------------------------------------------------
// at_solve_noalloc: at_solve with its workspace in a fixed device array
// ---------------------------------------------------------------------------
// The workspace of the allocation-free entry point: one array per device, held
// until the process ends.  Host code never passes its name to a kernel (the
// name is a host-side stand-in); it uses the device address that
// hipGetSymbolAddress returns for the current device, looked up once per
// device.  Calls on one device are serialised by that device's lock.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu[kMaxDevices];
static void *g_scratch_ptr[kMaxDevices] = {};

// The scratch address of device `dev`, the current device (looked up on its
// first use; the caller holds that device's lock).
static int scratch_address(int dev, void **ptr)
{
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "scratch: symbol address");
        if (!p) return fail(AT_EDEVICE, "scratch: null symbol address");
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return AT_OK;
}

}  // namespace at

using namespace at;

extern "C" {

const char *at_last_error(void) { return last_error(); }

int at_shutdown(void) { return release_class_streams(); }

int at_build_travel(int32_t n, const double *lat_deg, const double *lon_deg, double speed_kmh,
                    int32_t *travel)
{
    if (n < 1 || n > kMaxLocs) return fail(AT_EINVAL, "n %d outside [1, %d]", n, kMaxLocs);
    if (!(speed_kmh > 0.0) || !std::isfinite(speed_kmh)) return fail(AT_EINVAL, "speed must be positive");
    if (!lat_deg || !lon_deg || !travel) return fail(AT_EINVAL, "null pointer");
    return host_travel(n, lat_deg, lon_deg, speed_kmh, travel)
               ? AT_OK
               : fail(AT_ERANGE, "a travel time does not fit int32 seconds");
}

int at_build_travel_device(int32_t n, const double *lat_deg, const double *lon_deg, double speed_kmh,
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
    if ((int64_t)n_inst * n_restarts > (1 << 24)) return 0;
    return plan_ws(n_inst, insts, params, n_restarts).end;
}

int at_solve_batch(int32_t n_inst, const at_instance *insts, const at_params *params,
                   int32_t n_restarts, void *ws, size_t ws_bytes, void *stream, at_result *out)
{
    if (n_inst < 1 || !insts || !params || !out || n_restarts < 1)
        return fail(AT_EINVAL, "bad batch arguments");
    return solve_common(n_inst, insts, params, n_restarts, ws, ws_bytes, stream, out, false);
}

int at_solve(const at_instance *inst, const at_params *params, void *ws, size_t ws_bytes,
             void *stream, at_result *out)
{
    if (!inst || !params || !out) return fail(AT_EINVAL, "null argument");
    return solve_common(1, inst, params, 1, ws, ws_bytes, stream, out, true);
}

int at_solve_noalloc(const at_instance *inst, const at_params *params, void *stream, at_result *out)
{
    if (!inst || !params || !out) return fail(AT_EINVAL, "null argument");
    int rc = check_scalars(inst, params);
    if (rc) return rc;
    const size_t need = plan_ws(1, inst, params, 1).end;
    if (need > kScratchBytes)
        return fail(AT_ENOMEM, "at_solve_noalloc: this solve needs %zu bytes of workspace, the fixed array "
                               "holds %zu (use at_solve with a caller workspace)", need, kScratchBytes);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "current device");
    if (dev < 0 || dev >= kMaxDevices) return fail(AT_EDEVICE, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu[dev]);
    void *ws = nullptr;
    if ((rc = scratch_address(dev, &ws)) != AT_OK) return rc;
    return solve_common(1, inst, params, 1, ws, kScratchBytes, stream, out, true, false);
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
    WsPlan p = plan_ws(1, inst, params, 1);
    if (ws_bytes < p.end) return fail(AT_ENOMEM, "workspace %zu bytes, need %zu", ws_bytes, p.end);
    hipStream_t s = (hipStream_t)stream;
    char *base = (char *)ws;
    std::vector<InstDev> ih(1);
    carve_inst(ih[0], *inst, base + p.inst_off[0], may_need_global(*inst, *params));
    rc = prepare_instances(1, (InstDev *)(base + p.insts), ih, s);
    if (rc) return rc;
    const InstDev &d = ih[0];
    const bool wave = constrained(d) || params->schedule == AT_SCHED_WAVE;
    const uint32_t lds = wave ? wave_lds_bytes(d.M, d.V, d.R, d.Cs, constrained(d) ? 4 : d.esz, d.T2 != nullptr)
                              : lds_layout(d.M, d.V, d.R, d.Cs, d.esz, 4).total;
    if (lds > kLdsLimit) return fail(AT_ENOMEM, "instance too large for the LDS-resident key dump");
    JobHost h;
    h.inst = 0;
    h.pr = *params;
    h.pr.trace = 0;
    h.seed = 0;
    std::memset(&h.out, 0, sizeof(h.out));
    h.out.route_off = (int32_t *)route_off;
    h.out.route_seq = (int32_t *)route_seq;
    h.slots = n_slots(d.M, d.V);
    h.chunk = pick_chunk(*params, h.slots);
    h.rchunk = std::min(64, 2 * h.chunk);
    h.tb16 = 0;
    h.gstate = nullptr;
    JobDev j;
    rc = fill_job(j, h, (const InstDev *)(base + p.insts), (JobScal *)(base + p.scal));
    if (rc) return rc;
    JobDev *dj = (JobDev *)(base + p.jobs);
    hipError_t e = hipMemcpyAsync(dj, &j, sizeof(JobDev), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "upload job");
    const int block = params->block ? params->block : 256;
    if (wave)
        e = launch_debug_keys_wave(dj, route_off, route_seq, tabu_until, t, cur, best, keys_out, lds,
                                   !constrained(d) && d.esz == 2, s);
    else
        e = launch_debug_keys(dj, route_off, route_seq, tabu_until, t, cur, best, keys_out, block, lds,
                              d.esz == 2, s);
    if (e != hipSuccess) return hip_fail(e, "key dump launch");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "key dump");
    return AT_OK;
}

}  // extern "C"
