// server.hip -- continuous-batching serving loop (at_server_* in atabu.h).
//
// The server owns one device arena of `hbm_budget_bytes`.  A submitted request
// waits in a FIFO until a slot and enough arena memory are free; it is then
// admitted: its instance is prepared into the arena (checks + compact travel
// block), and it joins the resident solves.  Every at_server_progress call
// that finds the device idle retires finished solves, admits waiting
// requests, and launches the next chunk: every resident solve advances at
// least `chunk_iters` iterations (or to its end) from its saved state
// (routes, tabu table, iteration, objectives), so a request that arrives while
// others run starts at the next launch and shares the GPU with them.  Because
// every solve is deterministic and resumes exactly where it stopped, its
// result does not depend on what else is resident or on the chunking.
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <vector>

#include "atabu.h"
#include "atabu_internal.h"
#include "engine.h"

namespace at {

namespace {

// Move slots per iteration of the reference solve for chunk lengths: a
// one-workgroup solve with S slots runs max(1, kChunkSlots / S) chunks' worth
// of iterations per launch.
constexpr int64_t kChunkSlots = 1 << 20;

// Requests whose small records (saved-state table, prepared instance, HBM state
// table) one scatter round places; larger admission batches take several rounds.
constexpr int kScatterBatch = 256;

// One record of an admission batch: `bytes` (a multiple of 4) at `off` in the
// staging buffer go to `dst`.
struct Scatter {
    char *dst;
    uint32_t off, bytes;
};

// Copy each staged record to its place: one workgroup per record.
__global__ void k_scatter(const Scatter *e, const char *stage)
{
    const Scatter x = e[blockIdx.x];
    const uint32_t *src = (const uint32_t *)(stage + x.off);
    uint32_t *dst = (uint32_t *)x.dst;
    for (uint32_t i = threadIdx.x; i < x.bytes / 4; i += blockDim.x) dst[i] = src[i];
}

constexpr size_t kStageRecord = al16c(sizeof(SolveState)) + al16c(sizeof(InstDev)) + al16c(sizeof(GlobalBufs));
static_assert(sizeof(SolveState) % 4 == 0 && sizeof(InstDev) % 4 == 0 && sizeof(GlobalBufs) % 4 == 0,
              "scattered records are copied in 4-byte words");

struct Arena {
    char *base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free_;   // offset -> bytes, coalesced

    void init(char *b, size_t n) { base = b; size = n; free_.clear(); free_[0] = n; }

    char *alloc(size_t n)
    {
        n = al256(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t off = it->first, left = it->second - n;
            free_.erase(it);
            if (left) free_[off + n] = left;
            return base + off;
        }
        return nullptr;
    }

    void release(char *p, size_t n)
    {
        n = al256(n);
        size_t off = (size_t)(p - base);
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + n == next->first) { n += next->second; next = free_.erase(next); }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) { prev->second += n; return; }
        }
        free_[off] = n;
    }
};

struct Request {
    uint64_t ticket = 0;
    at_instance inst{};
    at_params pr{};
    size_t bytes = 0;
    char *mem = nullptr;
    // carved from mem
    InstDev *dinst = nullptr;
    JobScal *scal = nullptr;          // the server's result slot `slot`
    int slot = -1;
    SolveState *st = nullptr;
    at_result out{};                  // device arrays in mem
    InstDev host_inst{};
    SolveState st_host{};             // upload sources: stay valid until the copies ran
    GlobalBufs gb_host{};
    JobHost job;
    int t = 0;
    bool admitted = false, done = false;
    JobScal last{};
};

size_t request_bytes(const at_instance &in, const at_params &pr)
{
    const size_t M = (size_t)in.n_missions, V = (size_t)in.n_vehicles;
    size_t b = al256(sizeof(InstDev)) + al256(sizeof(SolveState));
    b += inst_bytes(in, may_need_global(in, pr));
    b += al256(4 * M) + al256(4 * (V + 1)) + al256(4 * M * V);          // saved routes + tabu
    b += al256(4 * (V + 1)) + 2 * al256(4 * (M ? M : 1));                // best routes
    b += al256(4 * (V + 1)) + al256(4 * (M ? M : 1));                    // final routes
    if (pr.trace) {
        const size_t n = (size_t)(pr.max_iters > 0 ? pr.max_iters : 1);
        b += al256(4 * n) * 2 + al256(8 * n) + al256(n);
    }
    if (may_need_global(in, pr)) b += gstate_bytes(in, pr);
    return b;
}

}  // namespace

struct Server {
    hipStream_t s = nullptr;
    char *dev = nullptr;
    size_t budget = 0;
    int max_slots = 0, chunk = 0;
    Arena arena;
    JobDev *djobs = nullptr;
    Xchg *xs = nullptr;
    JobScal *dscal = nullptr;         // per-slot results, read back with one copy per chunk
    std::vector<JobScal> hscal;
    std::vector<int> free_slots;
    hipEvent_t done_ev = nullptr;
    // The solves run on an internal stream: admission (reading the caller's
    // instance arrays) and result copies stay on the caller's stream `s`, so a
    // poll never waits for the launch in flight.  adm_ev marks the end of the
    // last admission's uploads, which the next launch waits for.
    hipStream_t ls = nullptr;
    hipEvent_t adm_ev = nullptr;
    bool in_flight = false;
    uint64_t next_ticket = 1;
    std::deque<uint64_t> finished;    // tickets done and not yet listed by at_server_completed
    std::deque<Request *> waiting;
    std::vector<Request *> active;
    std::map<uint64_t, Request *> all;
    std::vector<JobDev> table;        // host copy of the last launch's job table
    // admission: prepared-instance table, and the staging of the records one
    // scatter launch places (device, and pinned host memory)
    InstDev *dprep = nullptr;
    std::vector<InstDev> hprep;
    char *dstage = nullptr, *hstage = nullptr;
    Scatter *dscat = nullptr, *hscat = nullptr;

    ~Server()
    {
        if (in_flight && done_ev) (void)hipEventSynchronize(done_ev);
        if (ls) {
            (void)hipStreamSynchronize(ls);
            (void)hipStreamDestroy(ls);
        }
        if (adm_ev) (void)hipEventDestroy(adm_ev);
        for (auto &kv : all) delete kv.second;
        if (done_ev) (void)hipEventDestroy(done_ev);
        if (hstage) (void)hipHostFree(hstage);
        if (hscat) (void)hipHostFree(hscat);
        if (dev) (void)hipFree(dev);
    }

    // Lay out a request's arena block; returns the saved-state table to upload.
    SolveState carve(Request &r)
    {
        char *p = r.mem;
        const size_t M = (size_t)r.inst.n_missions, V = (size_t)r.inst.n_vehicles;
        r.dinst = (InstDev *)p; p += al256(sizeof(InstDev));
        r.st = (SolveState *)p; p += al256(sizeof(SolveState));
        const bool with_t = may_need_global(r.inst, r.pr);
        carve_inst(r.host_inst, r.inst, p, with_t); p += inst_bytes(r.inst, with_t);
        SolveState st{};
        st.seq = (int32_t *)p; p += al256(4 * M);
        st.off = (int32_t *)p; p += al256(4 * (V + 1));
        st.tabu = (int32_t *)p; p += al256(4 * M * V);
        r.out.route_off = (int32_t *)p; p += al256(4 * (V + 1));
        r.out.route_seq = (int32_t *)p; p += al256(4 * (M ? M : 1));
        r.out.route_of = (int32_t *)p; p += al256(4 * (M ? M : 1));
        r.out.final_off = (int32_t *)p; p += al256(4 * (V + 1));
        r.out.final_seq = (int32_t *)p; p += al256(4 * (M ? M : 1));
        if (r.pr.trace) {
            const size_t n = (size_t)(r.pr.max_iters > 0 ? r.pr.max_iters : 1);
            r.out.tr_move = (uint32_t *)p; p += al256(4 * n);
            r.out.tr_delta = (int32_t *)p; p += al256(4 * n);
            r.out.tr_obj = (int64_t *)p; p += al256(8 * n);
            r.out.tr_flags = (uint8_t *)p; p += al256(n);
        }
        r.job.gstate = may_need_global(r.inst, r.pr) ? (GlobalBufs *)p : nullptr;
        r.job.out = r.out;
        return st;
    }

    // Admit a batch of requests whose arena blocks are allocated: prepare every
    // instance in one set of launches (one stream synchronisation for the batch),
    // plan their solves, and place their state tables and prepared instances with
    // one copy and one scatter launch.  A request that fails is finished with its
    // error status and its memory released; the others are returned in `ok`.
    void admit_batch(const std::vector<Request *> &batch, std::vector<Request *> &ok)
    {
        const size_t n = batch.size();
        std::vector<int> rc(n, AT_OK);
        hprep.resize(n);
        for (size_t k = 0; k < n; ++k) {
            Request &r = *batch[k];
            r.slot = free_slots.back();
            free_slots.pop_back();
            r.scal = dscal + r.slot;
            // state table: pointers, valid = 0 (the first chunk starts from the greedy solution)
            r.st_host = carve(r);
            hprep[k] = r.host_inst;
        }
        // every instance of the batch in one set of prepare launches
        const int prc = prepare_enqueue((int32_t)n, dprep, hprep.data(), s);
        hipError_t e = prc == AT_OK ? hipStreamSynchronize(s) : hipSuccess;
        std::vector<Request *> cand;
        for (size_t k = 0; k < n; ++k) {
            Request &r = *batch[k];
            if (prc) rc[k] = prc;
            else if (e != hipSuccess) rc[k] = hip_fail(e, "server: prepare");
            if (rc[k] == AT_OK) {
                r.host_inst = hprep[k];
                rc[k] = prepare_check(1, &r.host_inst);
            }
            if (rc[k] == AT_OK) {
                r.job.inst = 0;
                r.job.pr = r.pr;
                r.job.pr.schedule = r.pr.schedule == AT_SCHED_MULTI ? AT_SCHED_AUTO : r.pr.schedule;
                r.job.seed = r.pr.restart_seed;
                r.job.chunked = true;
                rc[k] = plan_job(r.job, r.host_inst, false);
            }
            if (rc[k] == AT_OK && r.job.kind == AT_SCHED_GLOBAL)
                carve_gstate(r.gb_host, r.host_inst.M, r.host_inst.V, ring_slots(r.pr), (char *)r.job.gstate);
            if (rc[k] != AT_OK) {
                finish_failed(r, rc[k]);
                continue;
            }
            cand.push_back(&r);
        }
        // their records (saved-state table, prepared instance, HBM state table) placed
        // by one copy and one scatter launch per round of kScatterBatch requests
        int src = AT_OK;
        for (size_t a = 0; a < cand.size() && src == AT_OK; a += kScatterBatch) {
            const size_t b = std::min(cand.size(), a + kScatterBatch);
            if (a > 0 && (e = hipStreamSynchronize(s)) != hipSuccess) {   // the staging is reused
                src = hip_fail(e, "server: admission");
                break;
            }
            uint32_t off = 0, ne = 0;
            auto put = [&](void *dst, const void *rec, size_t bytes) {
                std::memcpy(hstage + off, rec, bytes);
                hscat[ne++] = Scatter{(char *)dst, off, (uint32_t)bytes};
                off += (uint32_t)al16c(bytes);
            };
            for (size_t q = a; q < b; ++q) {
                Request &r = *cand[q];
                put(r.st, &r.st_host, sizeof(SolveState));
                put(r.dinst, &r.host_inst, sizeof(InstDev));
                if (r.job.kind == AT_SCHED_GLOBAL) put(r.job.gstate, &r.gb_host, sizeof(GlobalBufs));
            }
            if ((e = hipMemcpyAsync(dstage, hstage, off, hipMemcpyHostToDevice, s)) != hipSuccess ||
                (e = hipMemcpyAsync(dscat, hscat, sizeof(Scatter) * ne, hipMemcpyHostToDevice, s)) != hipSuccess) {
                src = hip_fail(e, "server: admission upload");
                break;
            }
            k_scatter<<<dim3(ne), dim3(256), 0, s>>>(dscat, dstage);
            if ((e = hipGetLastError()) != hipSuccess) src = hip_fail(e, "server: admission scatter");
        }
        // the next launch (on the internal stream) waits for these uploads
        if (src == AT_OK && (e = hipEventRecord(adm_ev, s)) != hipSuccess) src = hip_fail(e, "server: admission event");
        for (Request *r : cand) {
            if (src != AT_OK) {
                finish_failed(*r, src);
                continue;
            }
            r->admitted = true;
            r->t = 0;
            ok.push_back(r);
        }
    }

    // A request that could not be admitted: finished with its error status, its
    // memory and slot released.
    void finish_failed(Request &r, int status)
    {
        r.done = true;
        finished.push_back(r.ticket);
        r.last.status = status;
        arena.release(r.mem, r.bytes);
        r.mem = nullptr;
        free_slots.push_back(r.slot);
        r.slot = -1;
    }

    // Retire finished solves after the last launch completed.
    int collect()
    {
        if (active.empty()) return AT_OK;
        hipError_t e = hipMemcpyAsync(hscal.data(), dscal, sizeof(JobScal) * hscal.size(), hipMemcpyDeviceToHost, ls);
        if (e != hipSuccess) return hip_fail(e, "server: read back");
        if ((e = hipStreamSynchronize(ls)) != hipSuccess) return hip_fail(e, "server: chunk");
        std::vector<Request *> keep;
        for (Request *r : active) {
            const JobScal &h = hscal[(size_t)r->slot];
            r->last = h;
            r->t = h.iters_done;
            if (h.status != AT_OK || h.stopped || r->t >= r->pr.max_iters) {
                r->done = true;
                finished.push_back(r->ticket);
                free_slots.push_back(r->slot);
                r->slot = -1;
            } else {
                keep.push_back(r);
            }
        }
        active.swap(keep);
        return AT_OK;
    }

    // Estimated times, from rates measured on gfx950 (300 to 2000 missions): a
    // one-workgroup solve evaluates about 2.5e9 move slots/s, a workgroup of the
    // HBM-resident schedule about 1.9e9, plus about 15 us per iteration for its
    // exchange, apply and record rebuild.
    static constexpr double kWgRate = 2.5e9, kGlRate = 1.9e9, kGlIter = 15e-6;

    // Launch the next chunk of every active solve.
    int launch()
    {
        if (active.empty()) return AT_OK;
        const size_t n = active.size();
        std::vector<JobHost> jobs(n);
        bool same = true;
        uint32_t lds = 0;
        for (size_t k = 0; k < n; ++k) {
            jobs[k] = active[k]->job;
            jobs[k].inst = (int)k;
            same = same && jobs[k].esz16 == jobs[0].esz16 && jobs[k].tb16 == jobs[0].tb16;
            lds = std::max(lds, jobs[k].lds);
        }
        const int cap = same ? max_groups_mixed(lds, jobs[0].tb16, jobs[0].esz16) : 0;
        int rc = cap >= 1 ? plan_pooled(jobs, cap) : plan_classes(jobs);
        if (rc) return rc;
        hipError_t e;
        if ((e = hipEventRecord(done_ev, ls)) != hipSuccess) return hip_fail(e, "server: event");
        in_flight = true;
        return AT_OK;
    }

    // Fill the job table in `order` (iterations from jobs[].iters) and upload it
    // on the launch stream once the admitted records are in place.
    int upload_table(const std::vector<JobHost> &jobs, const std::vector<int> &order)
    {
        std::vector<JobDev> hj(order.size());
        for (size_t k = 0; k < order.size(); ++k) {
            Request *r = active[(size_t)order[k]];
            int rc = fill_job(hj[k], jobs[(size_t)order[k]], r->dinst, r->scal);
            if (rc) return rc;
            hj[k].t_begin = r->t;
            hj[k].t_end = (int)(r->t + jobs[(size_t)order[k]].iters);
            hj[k].resume = 1;
            hj[k].save = 1;
            hj[k].st = r->st;
        }
        // the host copy of the table stays alive until the launch has completed
        table.swap(hj);
        hipError_t e = hipStreamWaitEvent(ls, adm_ev, 0);
        if (e == hipSuccess)
            e = hipMemcpyAsync(djobs, table.data(), sizeof(JobDev) * table.size(), hipMemcpyHostToDevice, ls);
        return e == hipSuccess ? AT_OK : hip_fail(e, "server: job upload");
    }

    // One grid for every solve (all of one entry and tabu width; `cap` workgroups
    // fit the device).  For a launch length T: a solve whose remaining iterations
    // fit T on one workgroup goes to the workers' queue with all of them; a longer
    // (HBM-resident) one gets a range of workgroups, as few as let chunk_iters
    // iterations fit T (at most one per 16384 move slots); the workers are as
    // many as the queue's total time over T.  T is the shortest length whose plan
    // fits the grid.  A solve with its own range that would finish before the
    // launch's longest part runs more iterations, up to all that remain.  A worker
    // that finishes a solve takes the next (longest first), so no workgroup waits
    // out the launch while solves are queued.
    int plan_pooled(std::vector<JobHost> &jobs, int cap)
    {
        const size_t n = jobs.size();
        std::vector<int64_t> rem(n);
        std::vector<double> full(n);   // all remaining iterations on one workgroup
        for (size_t k = 0; k < n; ++k) {
            const JobHost &h = jobs[k];
            rem[k] = active[k]->pr.max_iters - active[k]->t;
            full[k] = h.kind == AT_SCHED_GLOBAL ? (double)rem[k] * ((double)h.slots / kGlRate + kGlIter)
                                                : (double)rem[k] * (double)h.slots / kWgRate;
        }
        std::vector<int> g(n, 0);
        auto per_iter = [&](size_t k, int groups) {
            return (double)jobs[k].slots / ((double)groups * kGlRate) + kGlIter;
        };
        auto plan = [&](double T, bool keep) {
            int64_t need = 0;
            double pooled = 0;
            for (size_t k = 0; k < n; ++k) {
                int gk = 0;
                if (jobs[k].kind == AT_SCHED_GLOBAL && full[k] > T) {
                    const double it = (double)std::min<int64_t>(rem[k], chunk);
                    const double per = T / it - kGlIter;
                    const int64_t ask = std::max<int64_t>(1, jobs[k].slots / 16384);
                    const int64_t x = per <= 0 ? ask : (int64_t)std::ceil((double)jobs[k].slots / (kGlRate * per));
                    gk = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(x, ask), cap));
                    need += gk;
                } else {
                    pooled += full[k];
                }
                if (keep) g[k] = gk;
            }
            if (pooled > 0) need += std::max<int64_t>(1, (int64_t)std::ceil(pooled / T));
            return need;
        };
        double lo = 1e-5, hi = 1e4;   // seconds
        for (int i = 0; i < 64; ++i) {
            const double mid = std::sqrt(lo * hi);
            if (plan(mid, false) <= cap) hi = mid; else lo = mid;
        }
        if (plan(hi, true) > cap) return fail(AT_EDEVICE, "server: the resident solves do not fit one launch");
        double span = hi;
        int ranged = 0;
        std::vector<int> pool, own;
        for (size_t k = 0; k < n; ++k) {
            if (g[k] > 0) {
                ranged += g[k];
                own.push_back((int)k);
                span = std::max(span, (double)std::min<int64_t>(rem[k], chunk) * per_iter(k, g[k]));
            } else {
                pool.push_back((int)k);
                span = std::max(span, full[k]);
            }
        }
        for (size_t k = 0; k < n; ++k) {
            JobHost &h = jobs[k];
            if (g[k] > 0) {
                const int64_t more = (int64_t)(span / per_iter(k, g[k]));
                h.groups = g[k];
                h.iters = std::min<int64_t>(rem[k], std::max<int64_t>(std::min<int64_t>(rem[k], chunk), more));
            } else {
                h.groups = 1;
                h.iters = rem[k];
            }
            if (h.kind == AT_SCHED_GLOBAL) set_block_size(h);
        }
        std::stable_sort(pool.begin(), pool.end(), [&](int a, int b) { return full[(size_t)a] > full[(size_t)b]; });
        int g0 = 0;
        for (int k : own) {
            jobs[(size_t)k].g0 = g0;
            g0 += jobs[(size_t)k].groups;
        }
        std::vector<int> order = pool;
        order.insert(order.end(), own.begin(), own.end());
        uint32_t lds = 0;
        for (const JobHost &h : jobs) lds = std::max(lds, h.lds);
        int rc = upload_table(jobs, order);
        if (rc) return rc;
        const int workers = pool.empty() ? 0 : cap - ranged;
        hipError_t e = fill_u32(xs->queues, 0u, 1, ls);
        if (e == hipSuccess)
            e = launch_search_mixed(djobs + pool.size(), (int)own.size(), ranged, djobs, (int)pool.size(),
                                    &xs->queues[0], workers, lds, jobs[0].tb16, jobs[0].esz16, ls);
        return e == hipSuccess ? AT_OK : hip_fail(e, "server: search launch");
    }

    // Solves of several entry or tabu widths: one launch per class of
    // one-workgroup solves (concurrently), then the HBM-resident ones.  Each
    // advances chunk_iters iterations; a one-workgroup solve with S move slots,
    // S < 2^20, floor(2^20 / S) times as many, up to all that remain.
    int plan_classes(std::vector<JobHost> &jobs)
    {
        for (size_t k = 0; k < jobs.size(); ++k) {
            JobHost &h = jobs[k];
            int64_t it = chunk;
            if (h.kind == AT_SCHED_WG) it *= std::max<int64_t>(1, kChunkSlots / std::max<int64_t>(1, h.slots));
            h.iters = std::min<int64_t>(active[k]->pr.max_iters - active[k]->t, it);
        }
        const std::vector<int> order = order_jobs(jobs);
        int rc = assign_groups(jobs, order);
        if (!rc) rc = upload_table(jobs, order);
        if (!rc) rc = launch_jobs(jobs, order, djobs, xs, ls);
        return rc;
    }
};

}  // namespace at

using namespace at;

extern "C" {

int at_server_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t chunk_iters, void *stream,
                     void **server)
{
    if (!server) return fail(AT_EINVAL, "null server handle");
    if (max_slots < 1 || max_slots > 65536) return fail(AT_EINVAL, "max_slots outside [1, 65536]");
    if (chunk_iters < 1) return fail(AT_EINVAL, "chunk_iters must be positive");
    const size_t nstage = (size_t)std::min(max_slots, kScatterBatch);
    const size_t fixed = al256(sizeof(Xchg)) + al256(sizeof(JobDev) * (size_t)max_slots)
                       + al256(sizeof(JobScal) * (size_t)max_slots) + al256(sizeof(InstDev) * (size_t)max_slots)
                       + al256(kStageRecord * nstage) + al256(3 * sizeof(Scatter) * nstage);
    if (hbm_budget_bytes < fixed + (1 << 20)) return fail(AT_ENOMEM, "budget too small");
    Server *sv = new Server();
    sv->s = (hipStream_t)stream;
    sv->budget = hbm_budget_bytes;
    sv->max_slots = max_slots;
    sv->chunk = chunk_iters;
    hipError_t e = hipMalloc((void **)&sv->dev, hbm_budget_bytes);
    if (e != hipSuccess) { delete sv; return hip_fail(e, "server arena"); }
    sv->xs = (Xchg *)sv->dev;
    sv->djobs = (JobDev *)(sv->dev + al256(sizeof(Xchg)));
    size_t o = al256(sizeof(Xchg)) + al256(sizeof(JobDev) * (size_t)max_slots);
    sv->dscal = (JobScal *)(sv->dev + o);
    o += al256(sizeof(JobScal) * (size_t)max_slots);
    sv->dprep = (InstDev *)(sv->dev + o);
    o += al256(sizeof(InstDev) * (size_t)max_slots);
    sv->dstage = sv->dev + o;
    o += al256(kStageRecord * nstage);
    sv->dscat = (Scatter *)(sv->dev + o);
    if ((e = hipHostMalloc((void **)&sv->hstage, kStageRecord * nstage, hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void **)&sv->hscat, 3 * sizeof(Scatter) * nstage, hipHostMallocDefault)) != hipSuccess) {
        delete sv;
        return hip_fail(e, "server staging");
    }
    sv->hscal.assign((size_t)max_slots, JobScal{});
    for (int k = max_slots - 1; k >= 0; --k) sv->free_slots.push_back(k);
    sv->arena.init(sv->dev + fixed, hbm_budget_bytes - fixed);
    if ((e = hipEventCreateWithFlags(&sv->done_ev, hipEventDisableTiming)) != hipSuccess) {
        delete sv;
        return hip_fail(e, "server event");
    }
    if ((e = hipEventCreateWithFlags(&sv->adm_ev, hipEventDisableTiming)) != hipSuccess) {
        sv->adm_ev = nullptr;
        delete sv;
        return hip_fail(e, "server event");
    }
    // default priority, and no implicit ordering with the caller's (possibly null) stream
    if ((e = hipStreamCreateWithFlags(&sv->ls, hipStreamNonBlocking)) != hipSuccess) {
        sv->ls = nullptr;
        delete sv;
        return hip_fail(e, "server launch stream");
    }
    *server = sv;
    return AT_OK;
}

int at_server_submit(void *server, const at_instance *inst, const at_params *params, uint64_t *ticket)
{
    Server *sv = (Server *)server;
    if (!sv || !ticket) return fail(AT_EINVAL, "null argument");
    int rc = check_scalars(inst, params);
    if (rc) return rc;
    if (inst->travel_plane || inst->vehicle_type || inst->deadline || inst->heli_only || inst->flight_limit > 0 ||
        params->form != AT_FORM_BEST || params->schedule == AT_SCHED_WAVE)
        return fail(AT_EINVAL, "served requests run the best form on the unconstrained model");
    Request *r = new Request();
    r->inst = *inst;
    r->pr = *params;
    r->bytes = request_bytes(*inst, *params);
    if (r->bytes > sv->arena.size) {
        delete r;
        return fail(AT_ENOMEM, "request needs %zu bytes, the server budget holds %zu", r->bytes, sv->arena.size);
    }
    r->ticket = sv->next_ticket++;
    sv->waiting.push_back(r);
    sv->all[r->ticket] = r;
    *ticket = r->ticket;
    return AT_OK;
}

int at_server_progress(void *server, int32_t *n_active)
{
    Server *sv = (Server *)server;
    if (!sv) return fail(AT_EINVAL, "null server");
    if (sv->in_flight) {
        hipError_t q = hipEventQuery(sv->done_ev);
        if (q == hipErrorNotReady) {
            if (n_active) *n_active = (int32_t)sv->active.size();
            return AT_OK;
        }
        if (q != hipSuccess) return hip_fail(q, "server: chunk");
        sv->in_flight = false;
        int rc = sv->collect();
        if (rc) return rc;
    }
    // admit in arrival order while a slot and memory are free
    std::vector<Request *> batch;
    while (!sv->waiting.empty() && (int)(sv->active.size() + batch.size()) < sv->max_slots) {
        Request *r = sv->waiting.front();
        r->mem = sv->arena.alloc(r->bytes);
        if (!r->mem) break;
        sv->waiting.pop_front();
        batch.push_back(r);
    }
    if (!batch.empty()) sv->admit_batch(batch, sv->active);
    int rc = sv->launch();
    if (n_active) *n_active = (int32_t)(sv->active.size() + sv->waiting.size());
    return rc;
}

int at_server_poll(void *server, uint64_t ticket, at_result *out)
{
    Server *sv = (Server *)server;
    if (!sv || !out) return fail(AT_EINVAL, "null argument");
    auto it = sv->all.find(ticket);
    if (it == sv->all.end()) return fail(AT_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Request *r = it->second;
    if (!r->done) return AT_EAGAIN;
    hipError_t e = hipSuccess;
    if (r->mem && r->last.status == AT_OK) {
        const size_t M = (size_t)r->inst.n_missions, V = (size_t)r->inst.n_vehicles;
        if (out->route_off) e = hipMemcpyAsync(out->route_off, r->out.route_off, 4 * (V + 1), hipMemcpyDeviceToDevice, sv->s);
        if (e == hipSuccess && out->route_seq && M) e = hipMemcpyAsync(out->route_seq, r->out.route_seq, 4 * M, hipMemcpyDeviceToDevice, sv->s);
        if (e == hipSuccess && out->route_of && M) e = hipMemcpyAsync(out->route_of, r->out.route_of, 4 * M, hipMemcpyDeviceToDevice, sv->s);
        if (e == hipSuccess && out->final_off) e = hipMemcpyAsync(out->final_off, r->out.final_off, 4 * (V + 1), hipMemcpyDeviceToDevice, sv->s);
        if (e == hipSuccess && out->final_off && out->final_seq && M) e = hipMemcpyAsync(out->final_seq, r->out.final_seq, 4 * M, hipMemcpyDeviceToDevice, sv->s);
        const size_t n = (size_t)r->last.iters_done;
        if (e == hipSuccess && r->pr.trace && n) {
            if (out->tr_move) e = hipMemcpyAsync(out->tr_move, r->out.tr_move, 4 * n, hipMemcpyDeviceToDevice, sv->s);
            if (e == hipSuccess && out->tr_delta) e = hipMemcpyAsync(out->tr_delta, r->out.tr_delta, 4 * n, hipMemcpyDeviceToDevice, sv->s);
            if (e == hipSuccess && out->tr_obj) e = hipMemcpyAsync(out->tr_obj, r->out.tr_obj, 8 * n, hipMemcpyDeviceToDevice, sv->s);
            if (e == hipSuccess && out->tr_flags) e = hipMemcpyAsync(out->tr_flags, r->out.tr_flags, n, hipMemcpyDeviceToDevice, sv->s);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(sv->s);
    }
    out->best_obj = r->last.best_obj;
    out->final_obj = r->last.final_obj;
    out->iters_done = r->last.iters_done;
    out->best_iter = r->last.best_iter;
    out->status = r->last.status;
    out->search_ms = 0.f;
    const int status = r->last.status;
    if (r->mem) sv->arena.release(r->mem, r->bytes);
    sv->all.erase(it);
    delete r;
    if (e != hipSuccess) return hip_fail(e, "server: result copy");
    return status == AT_OK ? AT_OK : fail(status, "request failed with status %d", status);
}

int at_server_completed(void *server, uint64_t *tickets, int32_t capacity, int32_t *n_out)
{
    Server *sv = (Server *)server;
    if (!sv || !n_out || (capacity > 0 && !tickets)) return fail(AT_EINVAL, "null argument");
    if (capacity < 0) return fail(AT_EINVAL, "negative capacity");
    int32_t n = 0;
    while (n < capacity && !sv->finished.empty()) {
        const uint64_t t = sv->finished.front();
        sv->finished.pop_front();
        if (sv->all.count(t)) tickets[n++] = t;   // skip tickets already polled
    }
    *n_out = n;
    return AT_OK;
}

int at_server_destroy(void *server)
{
    Server *sv = (Server *)server;
    if (!sv) return fail(AT_EINVAL, "null server");
    delete sv;
    return AT_OK;
}

}  // extern "C"
