// search.hip -- persistent Tabu / neighbourhood search on gfx950, one launch
// for all iterations of a solve.
//
// Each iteration (Algorithm 3 in the best-move form; Algorithm 2 when the tabu
// rules are off):
//   prep    from the routes, every position's neighbours and every gap's ends
//           (O(M+V), one item per thread)
//   eval    every relocate move (mission -> gap) and every swap of two missions
//           gets its cost delta, a tabu bit (the move puts a mission into a
//           vehicle it left within `tenure` iterations and does not beat the
//           best objective) and is packed into a 64-bit key
//              blocked << 63 | (delta + 2^30) << 32 | slot index,
//           so the smallest key is the best admissible move, ties going to the
//           smallest index; each lane keeps a running minimum, then wavefront
//           shuffles and one LDS pass give the workgroup minimum (and, with
//           several workgroups per solve, a 64-bit atomic minimum in HBM)
//   apply   every thread decodes the winner; the flat route array is shifted in
//           two LDS phases; the moved missions become tabu for the vehicles
//           they left; the trace record and, on a new best, the routes are
//           written out.
//
// Work layout of eval: lanes own 64 consecutive route positions (a "tile"),
// each lane one mission, and walk the columns of a unit -- a run of `chunk`
// gaps (relocate) or partner positions (swap) -- so the per-column values are
// wave-uniform broadcasts and the per-lane values stay in registers.  The two
// gathers of a relocate and four of a swap hit the compact travel block in
// LDS.  Units are dealt round-robin to every wavefront of the solve.
#include "atabu_internal.h"
#include "atabu.h"

namespace at {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
constexpr uint32_t kSpinLimit = 1u << 24;

struct Ctx {
    int32_t *mrow, *mcol, *vrow, *vcol, *off;
    uint16_t *seq, *rt, *rof, *pof;
    int32_t *xr, *yc, *outv, *link, *ga, *gb, *gc;
    uint16_t *gr;
    uint64_t *red;
    int M, V, NG;
    uint32_t R;   // relocate slots M*(M+V)
};

__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }

__device__ __forceinline__ uint64_t wave_min(uint64_t k)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)k, o, 64);
        const uint32_t hi = __shfl_xor((uint32_t)(k >> 32), o, 64);
        const uint64_t x = ((uint64_t)hi << 32) | lo;
        k = x < k ? x : k;
    }
    return k;
}

__device__ __forceinline__ uint64_t pack_key(bool blocked, int delta, uint32_t idx)
{
    return ((uint64_t)blocked << 63) | ((uint64_t)(uint32_t)(delta + kDeltaBias) << 32) | idx;
}

__device__ __forceinline__ uint64_t splitmix_at(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + k * kGamma;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// vehicle of flat position k: the largest r with off[r] <= k
__device__ __forceinline__ int route_of_pos(const int32_t *off, int V, int k)
{
    int lo = 0, hi = V - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= k) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// prep: per-position neighbours and per-gap ends of the current routes
// ---------------------------------------------------------------------------
template <typename TE>
__device__ __forceinline__ void prep(const Ctx &c, const TE *tc, int tid, int nthr)
{
    for (int i = tid; i < c.M; i += nthr) {
        const int m = c.seq[i], r = c.rt[i];
        const int x = (i == c.off[r]) ? c.vrow[r] : c.mrow[c.seq[i - 1]];
        const int y = (i + 1 == c.off[r + 1]) ? c.vcol[r] : c.mcol[c.seq[i + 1]];
        const int mc = c.mcol[m], mr = c.mrow[m];
        const int a = tc[x + mc], bb = tc[mr + y], l = tc[x + y];
        c.xr[i] = x;
        c.yc[i] = y;
        c.outv[i] = a + bb;
        c.link[i] = l;
        const int G = i + r;
        c.ga[G] = x;
        c.gb[G] = mc;
        c.gc[G] = a;
        c.gr[G] = (uint16_t)r;
    }
    for (int r = tid; r < c.V; r += nthr) {
        const int e = c.off[r + 1], G = e + r;
        const int x = (c.off[r] == e) ? c.vrow[r] : c.mrow[c.seq[e - 1]];
        c.ga[G] = x;
        c.gb[G] = c.vcol[r];
        c.gc[G] = tc[x + c.vcol[r]];
        c.gr[G] = (uint16_t)r;
    }
}

// ---------------------------------------------------------------------------
// eval units
// ---------------------------------------------------------------------------
template <typename TE, typename TB, bool DBG>
__device__ __forceinline__ uint64_t relocate_unit(const Ctx &c, const TE *tc, const TB *tabu,
                                                  int tl, int G0, int G1, int lane, int t,
                                                  int thr, bool use_tabu, uint64_t *keys_out)
{
    const int i = tl * kWave + lane;
    const bool act = i < c.M;
    const int ii = act ? i : 0;
    const int m = c.seq[ii];
    const int mr = c.mrow[m], mc = c.mcol[m];
    const int rem = c.link[ii] - c.outv[ii];
    const int Gi = ii + c.rt[ii];
    const uint32_t ibase = (uint32_t)m * (uint32_t)c.NG;
    uint64_t best = kKeyNone;
    for (int G = G0; G < G1; ++G) {
        const int a = c.ga[G], b = c.gb[G], gcv = c.gc[G], r = c.gr[G];
        const int d = rem + (int)tc[a + mc] + (int)tc[mr + b] - gcv;
        const bool ok = act && (unsigned)(G - Gi) >= 2u;
        const bool tb = use_tabu && (int)tabu[r * c.M + m] > t;
        const bool blocked = tb && !(d < thr);
        const uint64_t key = ok ? pack_key(blocked, d, ibase + (uint32_t)G) : kKeyNone;
        if (DBG) {
            if (act) keys_out[ibase + (uint32_t)G] = key;
        } else {
            best = umin64(best, key);
        }
    }
    return best;
}

template <typename TE, typename TB, bool DBG>
__device__ __forceinline__ uint64_t swap_unit(const Ctx &c, const TE *tc, const TB *tabu,
                                              int tl, int j0, int j1, int lane, int t, int thr,
                                              bool use_tabu, uint64_t *keys_out)
{
    const int i = tl * kWave + lane;
    const bool act = i < c.M;
    const int ii = act ? i : 0;
    const int mi = c.seq[ii];
    const int mri = c.mrow[mi], mci = c.mcol[mi];
    const int xri = c.xr[ii], yci = c.yc[ii], outi = c.outv[ii], ri = c.rt[ii];
    const uint32_t M = (uint32_t)c.M;
    uint64_t best = kKeyNone;
    for (int j = j0; j < j1; ++j) {
        const int mj = c.seq[j];
        const int mrj = c.mrow[mj], mcj = c.mcol[mj];
        const int xrj = c.xr[j], ycj = c.yc[j], outj = c.outv[j], rj = c.rt[j];
        int d;
        if (j == i + 1 && ri == rj) {
            // i directly before j:  P i j N  ->  P j i N
            d = (int)tc[xri + mcj] + (int)tc[mrj + mci] + (int)tc[mri + ycj]
              - ((int)tc[xri + mci] + (int)tc[mri + mcj] + (int)tc[mrj + ycj]);
        } else {
            d = (int)tc[xri + mcj] + (int)tc[mrj + yci] + (int)tc[xrj + mci] + (int)tc[mri + ycj]
              - outi - outj;
        }
        const bool ok = act && j > i;
        const bool tb = use_tabu && ((int)tabu[rj * c.M + mi] > t || (int)tabu[ri * c.M + mj] > t);
        const bool blocked = tb && !(d < thr);
        const uint32_t a = (uint32_t)min(mi, mj), bm = (uint32_t)max(mi, mj);
        const uint32_t idx = c.R + a * M - (a * (a + 1u)) / 2u + (bm - a - 1u);
        const uint64_t key = pack_key(blocked, d, idx);
        if (DBG) {
            if (ok) keys_out[idx] = key;
        } else {
            best = ok ? umin64(best, key) : best;
        }
    }
    return best;
}

// Deal eval units round-robin over the TW wavefronts of the solve; gw is this
// wavefront's rank.  Returns this lane's minimum key.
template <typename TE, typename TB, bool DBG>
__device__ __forceinline__ uint64_t eval_all(const Ctx &c, const TE *tc, const TB *tabu, int chunk,
                                             int gw, int TW, int lane, int t, int thr,
                                             bool use_tabu, uint64_t *keys_out)
{
    uint64_t best = kKeyNone;
    const int nT = (c.M + kWave - 1) / kWave;
    const int nRC = (c.NG + chunk - 1) / chunk;
    int u = 0, mine = gw;
    for (int tl = 0; tl < nT; ++tl) {
        for (int k = 0; k < nRC; ++k, ++u) {
            if (u != mine) continue;
            mine += TW;
            const int G0 = k * chunk, G1 = min(c.NG, G0 + chunk);
            best = umin64(best, relocate_unit<TE, TB, DBG>(c, tc, tabu, tl, G0, G1, lane, t, thr,
                                                           use_tabu, keys_out));
        }
        const int jb = tl * kWave;
        const int nSC = (c.M - jb + chunk - 1) / chunk;
        for (int k = 0; k < nSC; ++k, ++u) {
            if (u != mine) continue;
            mine += TW;
            const int j0 = jb + k * chunk, j1 = min(c.M, j0 + chunk);
            best = umin64(best, swap_unit<TE, TB, DBG>(c, tc, tabu, tl, j0, j1, lane, t, thr,
                                                       use_tabu, keys_out));
        }
    }
    return best;
}

// ---------------------------------------------------------------------------
// LDS setup
// ---------------------------------------------------------------------------
template <typename TE, typename TB>
__device__ __forceinline__ Ctx make_ctx(char *smem, const Lay &ly, int M, int V)
{
    Ctx c;
    c.mrow = (int32_t *)(smem + ly.mrow);
    c.mcol = (int32_t *)(smem + ly.mcol);
    c.vrow = (int32_t *)(smem + ly.vrow);
    c.vcol = (int32_t *)(smem + ly.vcol);
    c.off = (int32_t *)(smem + ly.off);
    c.seq = (uint16_t *)(smem + ly.seq);
    c.rt = (uint16_t *)(smem + ly.rt);
    c.rof = (uint16_t *)(smem + ly.rof);
    c.pof = (uint16_t *)(smem + ly.pof);
    c.xr = (int32_t *)(smem + ly.xr);
    c.yc = (int32_t *)(smem + ly.yc);
    c.outv = (int32_t *)(smem + ly.outv);
    c.link = (int32_t *)(smem + ly.link);
    c.ga = (int32_t *)(smem + ly.ga);
    c.gb = (int32_t *)(smem + ly.gb);
    c.gc = (int32_t *)(smem + ly.gc);
    c.gr = (uint16_t *)(smem + ly.gr);
    c.red = (uint64_t *)(smem + ly.red);
    c.M = M;
    c.V = V;
    c.NG = M + V;
    c.R = (uint32_t)M * (uint32_t)(M + V);
    return c;
}

__device__ __forceinline__ void copy_words(uint32_t *dst, const uint32_t *src, int n, int tid, int nthr)
{
    for (int k = tid; k < n; k += nthr) dst[k] = src[k];
}

// route-of-position, position-of-mission and vehicle-of-mission from seq/off
__device__ __forceinline__ void index_routes(const Ctx &c, int tid, int nthr)
{
    for (int i = tid; i < c.M; i += nthr) {
        const int r = route_of_pos(c.off, c.V, i);
        const int m = c.seq[i];
        c.rt[i] = (uint16_t)r;
        c.pof[m] = (uint16_t)i;
        c.rof[m] = (uint16_t)r;
    }
}

// Algorithm 1 without feasibility checks: missions in a SplitMix64-driven
// Fisher-Yates order (identity for seed 0), each appended to the vehicle whose
// route time grows least (ties to the lowest vehicle).  Returns the objective.
template <typename TE>
__device__ int64_t greedy(const Ctx &c, const TE *tc, uint64_t seed, int64_t svc_sum, int tid,
                          int nthr)
{
    const int M = c.M, V = c.V;
    int32_t *pi = c.link;      // mission order
    int32_t *draw = c.xr;      // j of each Fisher-Yates step
    int32_t *lastx = c.ga;     // exit row offset at the end of each route
    int32_t *cnt = c.gb;       // missions per vehicle
    int32_t *veh = c.outv;     // vehicle chosen at each step
    int32_t *cur = c.gc;       // placement cursor per vehicle
    for (int i = tid; i < M; i += nthr) {
        pi[i] = i;
        if (i >= 1) draw[i] = (int32_t)(splitmix_at(seed, (uint64_t)(M - i)) % (uint64_t)(i + 1));
    }
    for (int v = tid; v < V; v += nthr) { lastx[v] = c.vrow[v]; cnt[v] = 0; }
    __syncthreads();
    if (seed != 0 && tid == 0) {
        for (int i = M - 1; i >= 1; --i) {
            const int j = draw[i];
            const int tmp = pi[i]; pi[i] = pi[j]; pi[j] = tmp;
        }
    }
    __syncthreads();
    if (tid < kWave) {
        const int lane = tid;
        int64_t acc = 0;
        for (int s = 0; s < M; ++s) {
            const int m = pi[s];
            const int mc = c.mcol[m], mr = c.mrow[m];
            uint64_t k = kKeyNone;
            for (int v = lane; v < V; v += kWave) {
                const int x = lastx[v], vc = c.vcol[v];
                const int add = (int)tc[x + mc] + (int)tc[mr + vc] - (int)tc[x + vc];
                k = umin64(k, ((uint64_t)(uint32_t)(add + kDeltaBias) << 32) | (uint32_t)v);
            }
            k = wave_min(k);
            const int vs = (int)(uint32_t)k;
            acc += (int64_t)(int32_t)(uint32_t)(k >> 32) - kDeltaBias;
            if ((vs & (kWave - 1)) == lane) { lastx[vs] = mr; cnt[vs] += 1; }
            if (lane == 0) veh[s] = vs;
        }
        if (lane == 0) c.red[40] = (uint64_t)acc;
    }
    __syncthreads();
    if (tid == 0) {
        int o = 0;
        for (int v = 0; v < V; ++v) { c.off[v] = o; cur[v] = o; o += cnt[v]; }
        c.off[V] = o;
        for (int s = 0; s < M; ++s) {
            const int v = veh[s];
            c.seq[cur[v]++] = (uint16_t)pi[s];
        }
    }
    __syncthreads();
    index_routes(c, tid, nthr);
    const int64_t acc = (int64_t)c.red[40];
    __syncthreads();
    return acc + svc_sum;
}

// write the current routes as the best solution
__device__ __forceinline__ void snapshot(const Ctx &c, const JobDev &J, int tid, int nthr)
{
    for (int i = tid; i < c.M; i += nthr) {
        const int m = c.seq[i];
        J.out_seq[i] = m;
        if (J.out_of) J.out_of[m] = c.rt[i];
    }
    for (int v = tid; v <= c.V; v += nthr) J.out_off[v] = c.off[v];
}

// ---------------------------------------------------------------------------
// one solve, state in LDS.  MULTI: gridDim.x workgroups cooperate on job[0].
// ---------------------------------------------------------------------------
template <typename TE, typename TB, bool MULTI>
__device__ void run_job(const JobDev &J, char *smem, int wg, int nwg, Xchg *xs)
{
    const InstDev &I = *J.inst;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & (kWave - 1), wave = tid / kWave, nwaves = nthr / kWave;
    const int M = I.M, V = I.V;
    const Lay ly = lds_layout(M, V, I.R, I.Cs, (int)sizeof(TE), (int)sizeof(TB));
    Ctx c = make_ctx<TE, TB>(smem, ly, M, V);
    TE *tc = (TE *)(smem + ly.tc);
    TB *tabu = (TB *)(smem + ly.tabu);
    const bool writer = !MULTI || wg == 0;

    copy_words((uint32_t *)tc, (const uint32_t *)I.tc, (int)(((int64_t)I.R * I.Cs * sizeof(TE)) / 4), tid, nthr);
    copy_words((uint32_t *)c.mrow, (const uint32_t *)I.mrow, M, tid, nthr);
    copy_words((uint32_t *)c.mcol, (const uint32_t *)I.mcol, M, tid, nthr);
    copy_words((uint32_t *)c.vrow, (const uint32_t *)I.vrow, V, tid, nthr);
    copy_words((uint32_t *)c.vcol, (const uint32_t *)I.vcol, V, tid, nthr);
    __syncthreads();

    int64_t cur, best;
    int best_iter, stopped;
    SolveState *st = J.st;
    if (J.resume && st && st->valid) {
        for (int i = tid; i < M; i += nthr) c.seq[i] = (uint16_t)st->seq[i];
        for (int v = tid; v <= V; v += nthr) c.off[v] = st->off[v];
        for (int k = tid; k < M * V; k += nthr) tabu[k] = (TB)st->tabu[k];
        cur = st->cur;
        best = st->best;
        best_iter = st->best_iter;
        stopped = st->stopped;
        __syncthreads();
        index_routes(c, tid, nthr);
        __syncthreads();
    } else {
        cur = greedy<TE>(c, tc, J.seed, I.svc_sum, tid, nthr);
        for (int k = tid; k < M * V; k += nthr) tabu[k] = (TB)0;
        best = cur;
        best_iter = -1;
        stopped = 0;
        if (writer) snapshot(c, J, tid, nthr);
        __syncthreads();
    }

    const bool use_tabu = J.variant == AT_TABU;
    const int gw = wg * nwaves + wave, TW = nwaves * nwg;
    int t = J.t_begin;
    bool aborted = false;
    for (; t < J.t_end && !stopped; ++t) {
        prep<TE>(c, tc, tid, nthr);
        __syncthreads();
        int thr = INT32_MIN;
        if (J.aspiration) {
            const int64_t g = best - cur;
            thr = g < (int64_t)INT32_MIN ? INT32_MIN : (int)g;
        }
        uint64_t k = eval_all<TE, TB, false>(c, tc, tabu, J.chunk, gw, TW, lane, t, thr, use_tabu, nullptr);
        k = wave_min(k);
        if (lane == 0) c.red[wave] = k;
        __syncthreads();
        if (tid < kWave) {
            uint64_t w = lane < nwaves ? c.red[lane] : kKeyNone;
            w = wave_min(w);
            if (MULTI && lane == 0) {
                uint64_t *slot = &xs->key[t % 3];
                __hip_atomic_fetch_min(slot, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(&xs->cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t target = (uint32_t)nwg * (uint32_t)(t - J.t_begin + 1);
                uint32_t spins = 0;
                uint32_t ab = 0;
                while (__hip_atomic_load(&xs->cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                    ab = __hip_atomic_load(&xs->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (ab) break;
                    if (++spins > kSpinLimit) {
                        __hip_atomic_store(&xs->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ab = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                w = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (wg == 0)
                    __hip_atomic_store(&xs->key[(t + 2) % 3], kKeyNone, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                c.red[65] = ab;
            }
            if (lane == 0) c.red[64] = w;
        }
        __syncthreads();
        if (MULTI && c.red[65]) { aborted = true; break; }
        const uint64_t key = c.red[64];
        if (key == kKeyNone) {
            // no move exists (at most one mission on a single vehicle)
            if (!use_tabu) { stopped = 1; break; }
            if (writer && tid == 0 && J.trace) {
                J.tr_move[t] = 0xFFFFFFFFu; J.tr_delta[t] = 0; J.tr_obj[t] = cur; J.tr_flags[t] = 0;
            }
            continue;
        }
        const bool blocked = (key >> 63) != 0;
        const int d = (int)((uint32_t)(key >> 32) & 0x7FFFFFFFu) - kDeltaBias;
        const uint32_t idx = (uint32_t)key;
        if (!use_tabu && d >= 0) { stopped = 1; break; }
        const int tval = t + J.tenure + 1;
        bool was_tabu;
        bool is_swap = idx >= c.R;
        if (!is_swap) {
            const int m = (int)(idx / (uint32_t)c.NG);
            const int G = (int)(idx - (uint32_t)m * (uint32_t)c.NG);
            const int v = c.gr[G];
            const int g = G - c.off[v] - v;
            const int s = c.pof[m];
            const int rs = c.rt[s];
            const int fp = c.off[v] + g;
            const int q = fp - (fp > s ? 1 : 0);
            was_tabu = use_tabu && (int)tabu[v * M + m] > t;
            const int lo = min(s, q), hi = max(s, q);
            __syncthreads();
            int32_t *tmp = c.xr;
            for (int kk = lo + tid; kk <= hi; kk += nthr)
                tmp[kk] = (kk == q) ? m : (q >= s ? c.seq[kk + 1] : c.seq[kk - 1]);
            if (v > rs) for (int r = rs + 1 + tid; r <= v; r += nthr) c.off[r] -= 1;
            if (v < rs) for (int r = v + 1 + tid; r <= rs; r += nthr) c.off[r] += 1;
            if (tid == 0 && use_tabu) tabu[rs * M + m] = (TB)tval;
            __syncthreads();
            for (int kk = lo + tid; kk <= hi; kk += nthr) {
                const int mm = tmp[kk];
                const int r = route_of_pos(c.off, V, kk);
                c.seq[kk] = (uint16_t)mm;
                c.rt[kk] = (uint16_t)r;
                c.pof[mm] = (uint16_t)kk;
                c.rof[mm] = (uint16_t)r;
            }
        } else {
            const uint32_t sp = idx - c.R;
            const double A = 2.0 * (double)M - 1.0;
            int a = (int)floor((A - sqrt(A * A - 8.0 * (double)sp)) * 0.5);
            a = max(0, min(a, M - 2));
            auto rowstart = [&](int64_t x) { return x * M - x * (x + 1) / 2; };
            while (a + 1 <= M - 2 && rowstart(a + 1) <= (int64_t)sp) ++a;
            while (a > 0 && rowstart(a) > (int64_t)sp) --a;
            const int m1 = a, m2 = (int)(a + 1 + ((int64_t)sp - rowstart(a)));
            const int s1 = c.pof[m1], s2 = c.pof[m2];
            const int r1 = c.rt[s1], r2 = c.rt[s2];
            was_tabu = use_tabu && ((int)tabu[r2 * M + m1] > t || (int)tabu[r1 * M + m2] > t);
            __syncthreads();
            if (tid == 0) {
                c.seq[s1] = (uint16_t)m2;
                c.seq[s2] = (uint16_t)m1;
                c.pof[m1] = (uint16_t)s2;
                c.pof[m2] = (uint16_t)s1;
                c.rof[m1] = (uint16_t)r2;
                c.rof[m2] = (uint16_t)r1;
                if (use_tabu) {
                    tabu[r1 * M + m1] = (TB)tval;
                    tabu[r2 * M + m2] = (TB)tval;
                }
            }
        }
        __syncthreads();
        cur += d;
        if (writer && tid == 0 && J.trace) {
            J.tr_move[t] = idx;
            J.tr_delta[t] = d;
            J.tr_obj[t] = cur;
            J.tr_flags[t] = (uint8_t)((is_swap ? 1 : 0) | ((was_tabu && !blocked) ? 2 : 0) | (blocked ? 4 : 0));
        }
        if (cur < best) {
            best = cur;
            best_iter = t;
            if (writer) snapshot(c, J, tid, nthr);
        }
    }
    if (!writer) return;
    if (tid == 0) {
        J.scal->best_obj = best;
        J.scal->final_obj = cur;
        J.scal->iters_done = t;
        J.scal->best_iter = best_iter;
        J.scal->stopped = stopped;
        J.scal->status = aborted ? AT_EDEVICE : AT_OK;
    }
    if (J.save && st) {
        for (int i = tid; i < M; i += nthr) st->seq[i] = c.seq[i];
        for (int v = tid; v <= V; v += nthr) st->off[v] = c.off[v];
        for (int k = tid; k < M * V; k += nthr) st->tabu[k] = (int32_t)tabu[k];
        if (tid == 0) {
            st->cur = cur;
            st->best = best;
            st->t = t;
            st->best_iter = best_iter;
            st->stopped = stopped;
            st->valid = 1;
        }
    }
}

// One workgroup per job; jobs are taken from an atomic queue until exhausted.
template <typename TE, typename TB>
__global__ void __launch_bounds__(1024) k_search_wg(const JobDev *jobs, int n_jobs, Xchg *xs)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __shared__ int s_job;
    for (;;) {
        if (threadIdx.x == 0)
            s_job = (int)__hip_atomic_fetch_add(&xs->queue, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int j = s_job;
        __syncthreads();
        if (j >= n_jobs) return;
        run_job<TE, TB, false>(jobs[j], smem, 0, 1, xs);
        __syncthreads();
    }
}

template <typename TE, typename TB>
__global__ void __launch_bounds__(1024) k_search_multi(const JobDev *job, Xchg *xs)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    run_job<TE, TB, true>(*job, smem, (int)blockIdx.x, (int)gridDim.x, xs);
}

// every slot's key for a given state (test hook)
template <typename TE>
__global__ void __launch_bounds__(1024) k_debug_keys(const JobDev *jp, const int32_t *off,
                                                     const int32_t *seq, const int32_t *tabu_until,
                                                     int32_t t, int64_t cur, int64_t best,
                                                     uint64_t *keys)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const JobDev &J = *jp;
    const InstDev &I = *J.inst;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & (kWave - 1), wave = tid / kWave, nwaves = nthr / kWave;
    const int M = I.M, V = I.V;
    const Lay ly = lds_layout(M, V, I.R, I.Cs, (int)sizeof(TE), 4);
    Ctx c = make_ctx<TE, int32_t>(smem, ly, M, V);
    TE *tc = (TE *)(smem + ly.tc);
    int32_t *tabu = (int32_t *)(smem + ly.tabu);
    copy_words((uint32_t *)tc, (const uint32_t *)I.tc, (int)(((int64_t)I.R * I.Cs * sizeof(TE)) / 4), tid, nthr);
    copy_words((uint32_t *)c.mrow, (const uint32_t *)I.mrow, M, tid, nthr);
    copy_words((uint32_t *)c.mcol, (const uint32_t *)I.mcol, M, tid, nthr);
    copy_words((uint32_t *)c.vrow, (const uint32_t *)I.vrow, V, tid, nthr);
    copy_words((uint32_t *)c.vcol, (const uint32_t *)I.vcol, V, tid, nthr);
    for (int i = tid; i < M; i += nthr) c.seq[i] = (uint16_t)seq[i];
    for (int v = tid; v <= V; v += nthr) c.off[v] = off[v];
    // external entry m*V + v holds the last blocked iteration; internal [v][m] holds it + 1
    for (int k = tid; k < M * V; k += nthr) {
        const int m = k / V, v = k - m * V;
        tabu[v * M + m] = tabu_until[k] + 1;
    }
    __syncthreads();
    index_routes(c, tid, nthr);
    __syncthreads();
    prep<TE>(c, tc, tid, nthr);
    __syncthreads();
    int thr = INT32_MIN;
    if (J.aspiration) {
        const int64_t g = best - cur;
        thr = g < (int64_t)INT32_MIN ? INT32_MIN : (int)g;
    }
    eval_all<TE, int32_t, true>(c, tc, tabu, J.chunk, wave, nwaves, lane, t, thr,
                                J.variant == AT_TABU, keys);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename F>
static hipError_t set_lds(F *f, uint32_t bytes)
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(f),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_search_wg(const JobDev *jobs, int32_t n_jobs, Xchg *xs, int grid, int block,
                            uint32_t lds_bytes, int tb16, int esz16, hipStream_t s)
{
    hipError_t e;
#define AT_WG(TE, TB)                                                                      \
    do {                                                                                   \
        if ((e = set_lds(k_search_wg<TE, TB>, lds_bytes)) != hipSuccess) return e;         \
        hipLaunchKernelGGL((k_search_wg<TE, TB>), dim3(grid), dim3(block), lds_bytes, s,   \
                           jobs, n_jobs, xs);                                              \
    } while (0)
    if (esz16 && tb16) AT_WG(uint16_t, uint16_t);
    else if (esz16) AT_WG(uint16_t, int32_t);
    else if (tb16) AT_WG(int32_t, uint16_t);
    else AT_WG(int32_t, int32_t);
#undef AT_WG
    return hipGetLastError();
}

template <typename TE, typename TB>
static hipError_t coop_launch(const JobDev *job, Xchg *xs, int n_groups, int block,
                              uint32_t lds_bytes, hipStream_t s)
{
    hipError_t e = set_lds(k_search_multi<TE, TB>, lds_bytes);
    if (e != hipSuccess) return e;
    void *args[] = {(void *)&job, (void *)&xs};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_search_multi<TE, TB>),
                                      dim3(n_groups), dim3(block), args, lds_bytes, s);
}

hipError_t launch_search_multi(const JobDev *job, Xchg *xs, int n_groups, int block,
                               uint32_t lds_bytes, int tb16, int esz16, hipStream_t s)
{
    if (esz16 && tb16) return coop_launch<uint16_t, uint16_t>(job, xs, n_groups, block, lds_bytes, s);
    if (esz16) return coop_launch<uint16_t, int32_t>(job, xs, n_groups, block, lds_bytes, s);
    if (tb16) return coop_launch<int32_t, uint16_t>(job, xs, n_groups, block, lds_bytes, s);
    return coop_launch<int32_t, int32_t>(job, xs, n_groups, block, lds_bytes, s);
}

template <typename TE, typename TB>
static int occupancy_multi(int block, uint32_t lds_bytes)
{
    if (set_lds(k_search_multi<TE, TB>, lds_bytes) != hipSuccess) return 0;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_search_multi<TE, TB>, block,
                                                     lds_bytes) != hipSuccess)
        return 0;
    return per_cu * num_cus();
}

int max_groups_multi(int block, uint32_t lds_bytes, int tb16, int esz16)
{
    if (esz16 && tb16) return occupancy_multi<uint16_t, uint16_t>(block, lds_bytes);
    if (esz16) return occupancy_multi<uint16_t, int32_t>(block, lds_bytes);
    if (tb16) return occupancy_multi<int32_t, uint16_t>(block, lds_bytes);
    return occupancy_multi<int32_t, int32_t>(block, lds_bytes);
}

hipError_t launch_debug_keys(const JobDev *job, const int32_t *off, const int32_t *seq,
                             const int32_t *tabu_until, int32_t t, int64_t cur, int64_t best,
                             uint64_t *keys, int block, uint32_t lds_bytes, int esz16,
                             hipStream_t s)
{
    hipError_t e;
    if (esz16) {
        if ((e = set_lds(k_debug_keys<uint16_t>, lds_bytes)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_debug_keys<uint16_t>, dim3(1), dim3(block), lds_bytes, s, job, off,
                           seq, tabu_until, t, cur, best, keys);
    } else {
        if ((e = set_lds(k_debug_keys<int32_t>, lds_bytes)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_debug_keys<int32_t>, dim3(1), dim3(block), lds_bytes, s, job, off,
                           seq, tabu_until, t, cur, best, keys);
    }
    return hipGetLastError();
}

uint32_t max_lds_bytes()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 65536;
    return (uint32_t)v;
}

int num_cus()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1;
    return v;
}

}  // namespace at
