// search.hip -- persistent Tabu / neighbourhood search on gfx950, one launch
// for all iterations of a solve.
//
// Each iteration (Algorithm 3 in the best-move form; Algorithm 2 when the tabu
// rules are off):
//   prep    from the routes, every position's neighbours and every gap's ends
//           as 16-byte records (O(M+V), one item per thread)
//   eval    every relocate move (mission -> gap) and every swap of two missions
//           gets its cost delta; the move is blocked if it puts a mission into
//           a vehicle it left within `tenure` iterations and does not beat the
//           best objective (aspiration); the best move is the smallest 64-bit
//              blocked << 63 | (delta + 2^30) << 32 | move index
//           (the slot index, or inside the LDS-resident schedules an
//           order-preserving packing of it that decodes with shifts)
//   apply   the winner is decoded (by wavefront 0 of each workgroup in the
//           LDS-resident schedules, by every workgroup's threads in the
//           HBM-resident one) and the flat route array shifted; the moved
//           missions become tabu for the vehicles they left; the trace record
//           and, on a new best, the routes are written out.
//
// Work layout of eval.  Lanes own 64 consecutive route positions (a tile), one
// mission each, whose values stay in registers; a unit is a run of `chunk`
// partner positions (swap) or `2 chunk` gaps (relocate).  Units are dealt
// round-robin to every wavefront of the solve.  In the one-workgroup schedule
// a relocate unit's columns are cut at vehicle boundaries; inside a segment
// the tabu status of a relocate depends only on (mission, vehicle), so each
// lane keeps a 32-bit running minimum of (delta + 2^25) << 6 | column rank and
// turns it into a 64-bit key once per segment (a blocked move can only win a
// segment if every move of the segment with the same or smaller delta is
// blocked too, since aspiration only depends on the delta); the
// multi-workgroup schedule's relocate units fold a per-lane tabu mask into one
// minimum over the unit.  Swap units keep one minimum of blocked << 31 |
// (delta + 2^25) << 5 | rank over the whole unit (two, tabu and not tabu, for
// 64-partner units).  Column ranks follow the slot index order for a fixed
// lane: the gap offset for relocates, the partner's mission id for swaps
// (ranked inside the chunk by prep), so ties resolve to the smallest slot
// index exactly as the full 64-bit comparison would.
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "atabu_internal.h"
#include "atabu.h"

namespace at {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
constexpr uint32_t kSpinLimit = 1u << 24;
constexpr int32_t kPackBias = 1 << 25;       // |delta| < 4 * 2^23

struct Ctx {
    int32_t *mrow, *mcol, *vrow, *vcol, *off;
    uint16_t *seq, *rt, *rof, *pof;
    int4 *posA, *posB, *gap;
    uint16_t *gend;  // per gap: the first gap of the next route (LDS schedules only)
    int2 *posC;     // global schedule only (row indices), else null
    uint8_t *prank;
    uint64_t *red;
    int M, V, NG, chunk, rchunk, Cs;   // chunk: swap unit width, rchunk: relocate unit width
    uint32_t R;   // relocate slots M*(M+V)
};

__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }

// Barrier of the threads that run one solve: the workgroup, or (WAVE) one
// wavefront, whose lanes run in lockstep: then only the LDS writes before it
// must be seen by the reads after it.
template <bool WAVE>
__device__ __forceinline__ void bsync()
{
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Global-memory views of a pointer: accesses through them compile to global_*
// instructions, which count on the vector-memory counter only.  The flat
// instructions a generic pointer gets also hold the LDS counter, so every LDS
// wait would also wait for the HBM accesses in flight.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *gld(const T *p)
{
    return (const __attribute__((address_space(1))) T *)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gst(T *p)
{
    return (__attribute__((address_space(1))) T *)p;
}
typedef int v4i_t __attribute__((ext_vector_type(4)));
typedef int v2i_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ int4 gld4(const int4 *p, size_t i)
{
    const v4i_t x = ((const __attribute__((address_space(1))) v4i_t *)p)[i];
    return make_int4(x.x, x.y, x.z, x.w);
}
__device__ __forceinline__ int2 gld2(const int2 *p, size_t i)
{
    const v2i_t x = ((const __attribute__((address_space(1))) v2i_t *)p)[i];
    return make_int2(x.x, x.y);
}
__device__ __forceinline__ void gst4(int4 *p, size_t i, int4 v)
{
    v4i_t x;
    x.x = v.x; x.y = v.y; x.z = v.z; x.w = v.w;
    ((__attribute__((address_space(1))) v4i_t *)p)[i] = x;
}
__device__ __forceinline__ void gst2(int2 *p, size_t i, int2 v)
{
    v2i_t x;
    x.x = v.x; x.y = v.y;
    ((__attribute__((address_space(1))) v2i_t *)p)[i] = x;
}
// 16 bytes at a global address held as an integer
__device__ __forceinline__ uint4 gld16(uint64_t addr, int o)
{
    typedef unsigned v4u_t __attribute__((ext_vector_type(4)));
    const v4u_t x = ((const __attribute__((address_space(1))) v4u_t *)addr)[o];
    return make_uint4(x.x, x.y, x.z, x.w);
}

__device__ __forceinline__ uint64_t wave_min(uint64_t k) { return wave_min_u64(k); }

__device__ __forceinline__ uint64_t pack_key(bool blocked, int delta, uint32_t idx)
{
    return ((uint64_t)blocked << 63) | ((uint64_t)(uint32_t)(delta + kDeltaBias) << 32) | idx;
}

// 64-bit key <-> exchange slot: the slot keeps the key's order in its low 63
// bits (blocked, delta + 2^29, index; |delta| < 2^29) and the tag in bit 63.
__device__ __forceinline__ uint64_t encode_slot(uint64_t key, uint64_t tag)
{
    if (key == kKeyNone) return (tag << 63) | 0x7FFFFFFFFFFFFFFFull;
    const uint64_t bl = key >> 63;
    const uint64_t f = ((key >> 32) & 0x7FFFFFFFull) - (1ull << 29);
    return (tag << 63) | (bl << 62) | (f << 32) | (key & 0xFFFFFFFFull);
}

__device__ __forceinline__ uint64_t decode_slot(uint64_t v)
{
    const uint64_t low = v & 0x7FFFFFFFFFFFFFFFull;
    if (low == 0x7FFFFFFFFFFFFFFFull) return kKeyNone;
    const uint64_t bl = (low >> 62) & 1;
    const uint64_t f = ((low >> 32) & 0x3FFFFFFFull) + (1ull << 29);
    return (bl << 63) | (f << 32) | (low & 0xFFFFFFFFull);
}

__device__ __forceinline__ uint32_t swap_index(uint32_t R, uint32_t M, uint32_t a, uint32_t b)
{
    // a < b
    return R + a * M - (a * (a + 1u)) / 2u + (b - a - 1u);
}

// Move index inside the LDS-resident schedules' keys: relocate of mission m to
// gap G as m << 16 | G, swap of missions a < b as 2^31 | a << 16 | b.  It orders
// the moves as the slot index does (every relocate before every swap, each kind
// by its pair), so the minimum key names the same move, and the decode on the
// iteration's critical path is shifts instead of a division or a square root.
// Needs M < 2^15 and M + V < 2^16 (the planner keeps larger solves on the
// HBM-resident schedule).  The trace and the key dump take the slot index.
__device__ __forceinline__ uint32_t lidx_swap(uint32_t a, uint32_t b)
{
    return 0x80000000u | (a << 16) | b;
}

__device__ __forceinline__ uint32_t lidx_slot(uint32_t ix, uint32_t R, uint32_t M, uint32_t NG)
{
    return (ix >> 31) ? swap_index(R, M, (ix >> 16) & 0x7FFFu, ix & 0xFFFFu) : (ix >> 16) * NG + (ix & 0xFFFFu);
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
// prep: per-position neighbours, per-gap ends, per-chunk ranks
// ---------------------------------------------------------------------------
// GEND: also the per-gap route ends (gend), which only the segmented relocate
// units read
template <typename TE, bool GEND = true>
__device__ __forceinline__ void prep(const Ctx &c, const TE *tc, int tid, int nthr)
{
    const int CH = c.chunk, M = c.M;
    for (int i = tid; i < M; i += nthr) {
        // three rounds of LDS reads, each independent of the others in its round:
        // positions (the neighbours' entries at clamped indices; a position opens
        // its route when the one before it is in another route, and closes it when
        // the one after it is), then missions and vehicles, then travel entries
        const int im = max(i - 1, 0), ip = min(i + 1, M - 1), ip2 = min(i + 2, M - 1);
        const int m = c.seq[i], r = c.rt[i];
        const int mp = c.seq[im], mn = c.seq[ip], mn2 = c.seq[ip2];
        const int rp = c.rt[im], rn = c.rt[ip], rn2 = c.rt[ip2];
        // rank of m among the missions of this position's chunk: the entries read 8
        // at a time from the 8-entry boundary at or below the chunk's start (16-byte
        // aligned; the array is padded to whole 8-entry groups), counting only those
        // in the chunk (a 4-entry chunk is half of one group)
        const int base = i & ~(CH - 1), end = min(M, base + CH);   // CH: a power of two, >= 4
        const int w0 = base & ~7;
        const uint4 q0 = *(const uint4 *)(c.seq + w0);
        const bool first = i == 0 || rp != r;
        const bool last = i + 1 == M || rn != r;
        const bool last2 = i + 2 >= M || rn2 != r;   // for !last: position i + 1 closes the route
        const int vr = c.vrow[r], vc = c.vcol[r], endr = GEND ? c.off[r + 1] : 0;
        const int mc = c.mcol[m], mr = c.mrow[m];
        const int xp = c.mrow[mp], yn = c.mcol[mn], mrn = c.mrow[mn], yn2 = c.mcol[mn2];
        const int x = first ? vr : xp;
        const int y = last ? vc : yn;
        const int y2 = last2 ? vc : yn2;
        const int a = tc[x + mc], bb = tc[mr + y], l = tc[x + y];
        const int s1 = tc[mrn + mc], s2 = tc[mr + y2], s3 = tc[mrn + y2];
        int rank = 0;
        if (CH == 4) {
            // the chunk is the group's low or high half
            const bool hi = base != w0;
            const uint32_t e[2] = {hi ? q0.z : q0.x, hi ? q0.w : q0.y};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                rank += (base + 2 * h < end && (int)(e[h] & 0xFFFFu) < m) ? 1 : 0;
                rank += (base + 2 * h + 1 < end && (int)(e[h] >> 16) < m) ? 1 : 0;
            }
        } else {
            const uint32_t e[4] = {q0.x, q0.y, q0.z, q0.w};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                rank += (base + 2 * h < end && (int)(e[h] & 0xFFFFu) < m) ? 1 : 0;
                rank += (base + 2 * h + 1 < end && (int)(e[h] >> 16) < m) ? 1 : 0;
            }
        }
        for (int w = w0 + 8; w < end; w += 8) {
            const uint4 q = *(const uint4 *)(c.seq + w);
            const uint32_t e[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                rank += (w + 2 * h < end && (int)(e[h] & 0xFFFFu) < m) ? 1 : 0;
                rank += (w + 2 * h + 1 < end && (int)(e[h] >> 16) < m) ? 1 : 0;
            }
        }
        // swapping m with its successor in the same route: P m n N -> P n m N
        const int adj = last ? 0 : l + s1 + s2 - a - bb - s3;
        c.prank[base + rank] = (uint8_t)(i - base);
        c.posA[i] = make_int4(mr, mc, x, y);
        c.posB[i] = make_int4(a + bb, l, (int)((uint32_t)m | ((uint32_t)r << 16)),
                              (int)((uint32_t)rank | ((uint32_t)(adj + kPackBias) << 6)));
        c.gap[i + r] = make_int4(x, mc, a, r);
        if (GEND) c.gend[i + r] = (uint16_t)(endr + r + 1);
        if (last) {
            // the gap after the route's last mission: from m's exit row to the base
            c.gap[i + 1 + r] = make_int4(mr, vc, bb, r);
            if (GEND) c.gend[i + 1 + r] = (uint16_t)(endr + r + 1);
        }
    }
    // the only gap of each empty route: on the highest threads, which have no
    // position of their own when M < nthr
    for (int r = nthr - 1 - tid; r < c.V; r += nthr) {
        const int e = c.off[r + 1], o = c.off[r], x = c.vrow[r], y = c.vcol[r];
        if (o == e) {
            c.gap[e + r] = make_int4(x, y, (int)tc[x + y], r);
            if (GEND) c.gend[e + r] = (uint16_t)(e + r + 1);
        }
    }
}

// ---------------------------------------------------------------------------
// eval: relocate unit (columns G0..G1 of one tile)
// ---------------------------------------------------------------------------
// Relocate unit of the multi-workgroup schedule, 16-bit travel entries
// (|delta| < 2^19): the tabu entries of the unit's vehicles (gaps are
// route-ordered, so a unit of at most 64 gaps spans at most 64 vehicles) are
// gathered up front into a 64-bit mask per lane, then one 32-bit minimum of
// blocked << 31 | (delta + 2^24) << 6 | column rank runs over all the unit's
// columns with no per-route step, so a unit over many short routes takes no
// longer than another (the iteration waits for the slowest wavefront).  For a
// fixed lane the slot index grows with the rank: ties resolve as the 64-bit keys
// would.
constexpr int32_t kFlatBias = 1 << 24;

template <typename TE, typename TB>
__device__ __forceinline__ uint64_t relocate_unit_flat(const Ctx &c, const TE *tc, const TB *tabu,
                                                       int tl, int G0, int G1, int lane, int t, int thr,
                                                       bool use_tabu)
{
    const int i = tl * kWave + lane;
    const bool act = i < c.M;
    const int ii = act ? i : tl * kWave;
    const int4 pa = c.posA[ii], pb = c.posB[ii];
    const int m = pb.z & 0xFFFF, ri = (int)((uint32_t)pb.z >> 16);
    const int mr = pa.x, mc = pa.y;
    const int remb = pb.y - pb.x + kFlatBias;
    const int thrb = thr < -kFlatBias ? 0 : thr + kFlatBias;   // d >= thr on the biased delta
    const int Gi = ii + ri;
    const int r0 = c.gap[G0].w & 0xFFFF, r1 = c.gap[G1 - 1].w & 0xFFFF;
    uint64_t tmask = 0;
    if (use_tabu) {
#pragma unroll 4
        for (int r = r0; r <= r1; ++r)
            tmask |= (uint64_t)((int)tabu[r * c.M + m] > t ? 1u : 0u) << (r - r0);
    }
    uint32_t pm = 0xFFFFFFFFu;
    // the lane's own two gaps (no move) get the all-ones key: a select on the key,
    // not on the update, keeps the column's gathers out of a branch
#define AT_RELOC_FLAT(gv, Gv)                                                                  \
    do {                                                                                       \
        const int db_ = remb + (int)tc[(gv).x + mc] + (int)tc[mr + (gv).y] - (gv).z;           \
        const uint32_t bl_ = (uint32_t)(tmask >> (((gv).w & 0xFFFF) - r0)) & (db_ >= thrb ? 1u : 0u); \
        const uint32_t own_ = ((unsigned)((Gv) - Gi) < 2u) ? 0xFFFFFFFFu : 0u;                 \
        pm = min(pm, (bl_ << 31) | ((uint32_t)db_ << 6) | (uint32_t)((Gv) - G0) | own_);       \
    } while (0)
    int G = G0;
    for (; G + 8 <= G1; G += 8) {
        const int4 g0 = c.gap[G], g1 = c.gap[G + 1], g2 = c.gap[G + 2], g3 = c.gap[G + 3];
        const int4 g4 = c.gap[G + 4], g5 = c.gap[G + 5], g6 = c.gap[G + 6], g7 = c.gap[G + 7];
        AT_RELOC_FLAT(g0, G);
        AT_RELOC_FLAT(g1, G + 1);
        AT_RELOC_FLAT(g2, G + 2);
        AT_RELOC_FLAT(g3, G + 3);
        AT_RELOC_FLAT(g4, G + 4);
        AT_RELOC_FLAT(g5, G + 5);
        AT_RELOC_FLAT(g6, G + 6);
        AT_RELOC_FLAT(g7, G + 7);
    }
    for (; G + 4 <= G1; G += 4) {
        const int4 g0 = c.gap[G], g1 = c.gap[G + 1], g2 = c.gap[G + 2], g3 = c.gap[G + 3];
        AT_RELOC_FLAT(g0, G);
        AT_RELOC_FLAT(g1, G + 1);
        AT_RELOC_FLAT(g2, G + 2);
        AT_RELOC_FLAT(g3, G + 3);
    }
    for (; G < G1; ++G) {
        const int4 g0 = c.gap[G];
        AT_RELOC_FLAT(g0, G);
    }
#undef AT_RELOC_FLAT
    if (!act || pm == 0xFFFFFFFFu) return kKeyNone;
    const int d = (int)((pm >> 6) & 0x1FFFFFFu) - kFlatBias;
    const uint32_t Gw = (uint32_t)G0 + (pm & 63u);
    return pack_key((pm >> 31) != 0, d, ((uint32_t)m << 16) | Gw);
}

template <typename TE, typename TB>
__device__ __forceinline__ uint64_t relocate_unit(const Ctx &c, const TE *tc, const TB *tabu,
                                                  int tl, int G0, int G1, int lane, int t, int thr,
                                                  bool use_tabu, int rlo, int rhi)
{
    const int i = tl * kWave + lane;
    const bool act = i < c.M;
    const int ii = act ? i : tl * kWave;
    const int4 pa = c.posA[ii], pb = c.posB[ii];
    const int m = pb.z & 0xFFFF, ri = (int)((uint32_t)pb.z >> 16);
    const int mr = pa.x, mc = pa.y;
    const int remb = pb.y - pb.x + kPackBias;
    const int Gi = ii + ri;
    const uint32_t ibase = (uint32_t)m << 16;
    // the unit's gap records (at most 64 columns), one per lane, read once and
    // handed to the column loop with readlane: one coalesced LDS read per unit
    // instead of a 16-byte broadcast per column
    const int gl_i = G0 + (lane < G1 - G0 ? lane : 0);
    const int4 gl = c.gap[gl_i];
    const int gel = c.gend[gl_i];
    auto col = [&](int G) {
        const int k = G - G0;
        return make_int4(__builtin_amdgcn_readlane(gl.x, k), __builtin_amdgcn_readlane(gl.y, k),
                         __builtin_amdgcn_readlane(gl.z, k), 0);
    };
    uint64_t best = kKeyNone;
    int G = G0;
    while (G < G1) {
        // the segment's vehicle and end
        const int r = __builtin_amdgcn_readlane(gl.w, G - G0) & 0xFFFF;
        const int Gend = min(G1, __builtin_amdgcn_readlane(gel, G - G0));
        const bool tb = use_tabu && (int)tabu[r * c.M + m] > t;
        uint32_t pm = 0xFFFFFFFFu;
        // four columns per step: all their LDS reads are in flight together
#define AT_RELOC(gv, Gv) \
    min(pm, ((uint32_t)(remb + (int)tc[(gv).x + mc] + (int)tc[mr + (gv).y] - (gv).z) << 6) | (uint32_t)((Gv) - G0))
        if (r < rlo || r > rhi) {
            // no lane of this tile flies vehicle r: no gap is a lane's own
            for (; G + 4 <= Gend; G += 4) {
                const int4 g0 = col(G), g1 = col(G + 1), g2 = col(G + 2), g3 = col(G + 3);
                pm = AT_RELOC(g0, G);
                pm = AT_RELOC(g1, G + 1);
                pm = AT_RELOC(g2, G + 2);
                pm = AT_RELOC(g3, G + 3);
            }
            for (; G < Gend; ++G) {
                const int4 g0 = col(G);
                pm = AT_RELOC(g0, G);
            }
        } else {
            for (; G + 4 <= Gend; G += 4) {
                const int4 g0 = col(G), g1 = col(G + 1), g2 = col(G + 2), g3 = col(G + 3);
                const uint32_t p0 = AT_RELOC(g0, G), p1 = AT_RELOC(g1, G + 1);
                const uint32_t p2 = AT_RELOC(g2, G + 2), p3 = AT_RELOC(g3, G + 3);
                pm = ((unsigned)(G - Gi) >= 2u) ? p0 : pm;
                pm = ((unsigned)(G + 1 - Gi) >= 2u) ? min(pm, p1) : pm;
                pm = ((unsigned)(G + 2 - Gi) >= 2u) ? min(pm, p2) : pm;
                pm = ((unsigned)(G + 3 - Gi) >= 2u) ? min(pm, p3) : pm;
            }
            for (; G < Gend; ++G) {
                const int4 g0 = col(G);
                const uint32_t p0 = AT_RELOC(g0, G);
                pm = ((unsigned)(G - Gi) >= 2u) ? p0 : pm;
            }
        }
#undef AT_RELOC
        if (act && pm != 0xFFFFFFFFu) {
            const int d = (int)(pm >> 6) - kPackBias;
            const int Gw = G0 + (int)(pm & 63u);
            const bool blocked = tb && !(d < thr);
            best = umin64(best, pack_key(blocked, d, ibase + (uint32_t)Gw));
        }
    }
    return best;
}

// ---------------------------------------------------------------------------
// eval: swap unit (partner positions j0..j1 of one tile, j0 a chunk start).
// With units of at most 32 columns (PACK5) one 32-bit minimum per segment holds
// the blocked bit, Δ + 2^25 and the 5-bit rank; with 64-column units the rank
// needs 6 bits and tabu / non-tabu moves keep separate minima.
// ---------------------------------------------------------------------------
template <typename TE, typename TB, bool PACK5>
__device__ __forceinline__ uint64_t swap_unit(const Ctx &c, const TE *tc, const TB *tabu, int tl,
                                              int j0, int j1, int lane, int t, int thr,
                                              bool use_tabu)
{
    const int i = tl * kWave + lane;
    const bool act = i < c.M;
    const int ii = act ? i : tl * kWave;
    const int4 pa = c.posA[ii], pb = c.posB[ii];
    const int mi = pb.z & 0xFFFF, ri = (int)((uint32_t)pb.z >> 16);
    const int mri = pa.x, mci = pa.y, xri = pa.z, yci = pa.w;
    const int outb = kPackBias - pb.x;
    const int adjb = (int)((uint32_t)pb.w >> 6);   // delta of swapping with the successor, + 2^25
    const int thrb = thr + kPackBias;              // aspiration threshold on the biased delta (thr <= 0)
    const uint32_t M = (uint32_t)c.M;
    // partners at or before the lane, or directly after it, need the masked path
    const bool diag = j0 <= tl * kWave + kWave;
    const TB *tabu_ri = tabu + ri * c.M;
    const int th = use_tabu ? t : INT32_MAX;     // no entry exceeds INT32_MAX: nothing is tabu
    // minima over the whole unit: the ranks are the chunk's, so they order every
    // partner of the unit as its slot index does (for a fixed lane), and the
    // rank's mission is looked up once at the end
    uint32_t mF = 0xFFFFFFFFu, mT = 0xFFFFFFFFu;
    int j = j0;
    while (j < j1) {
        const int r = __builtin_amdgcn_readfirstlane((int)((uint32_t)c.posB[j].z >> 16));
        const int jend = __builtin_amdgcn_readfirstlane(min(j1, c.off[r + 1]));
        const bool t1 = (int)tabu[r * c.M + mi] > th;
        // off_: all ones for a partner that is no move for this lane (diagonal units)
#define AT_SWAP(a, b, dd, off_)                                                                \
    do {                                                                                       \
        const bool tb_ = t1 | ((int)tabu_ri[(b).z & 0xFFFF] > th);                             \
        if (PACK5) {                                                                           \
            const bool bl_ = tb_ & !((dd) < thrb);                                             \
            mF = min(mF, (bl_ ? 0x80000000u : 0u) | ((uint32_t)(dd) << 5) | ((uint32_t)(b).w & 31u) | (off_)); \
        } else {                                                                               \
            const uint32_t p_ = ((uint32_t)(dd) << 6) | ((uint32_t)(b).w & 63u) | (off_);      \
            mT = tb_ ? min(mT, p_) : mT;                                                       \
            mF = tb_ ? mF : min(mF, p_);                                                       \
        }                                                                                      \
    } while (0)
#define AT_SWAP_D(a, b) (outb - (b).x + (int)tc[xri + (a).y] + (int)tc[(a).x + yci]            \
                         + (int)tc[(a).z + mci] + (int)tc[mri + (a).w])
        if (!diag) {
            for (; j + 2 <= jend; j += 2) {
                const int4 a0 = c.posA[j], b0 = c.posB[j], a1 = c.posA[j + 1], b1 = c.posB[j + 1];
                const int d0 = AT_SWAP_D(a0, b0), d1 = AT_SWAP_D(a1, b1);
                AT_SWAP(a0, b0, d0, 0u);
                AT_SWAP(a1, b1, d1, 0u);
            }
            for (; j < jend; ++j) {
                const int4 a0 = c.posA[j], b0 = c.posB[j];
                const int d0 = AT_SWAP_D(a0, b0);
                AT_SWAP(a0, b0, d0, 0u);
            }
        } else {
            // partners at or before the lane are masked; the lane's mission directly
            // before the partner in one route takes its delta from prep
#define AT_SWAP_DIAG(a, b, jj)                                                                 \
    do {                                                                                       \
        const int dg_ = AT_SWAP_D(a, b);                                                       \
        const int d_ = ((jj) == i + 1 && ri == r) ? adjb : dg_;                                \
        AT_SWAP(a, b, d_, (jj) > i ? 0u : 0xFFFFFFFFu);                                        \
    } while (0)
            for (; j + 2 <= jend; j += 2) {
                const int4 a0 = c.posA[j], b0 = c.posB[j], a1 = c.posA[j + 1], b1 = c.posB[j + 1];
                AT_SWAP_DIAG(a0, b0, j);
                AT_SWAP_DIAG(a1, b1, j + 1);
            }
            for (; j < jend; ++j) {
                const int4 a0 = c.posA[j], b0 = c.posB[j];
                AT_SWAP_DIAG(a0, b0, j);
            }
#undef AT_SWAP_DIAG
        }
#undef AT_SWAP_D
#undef AT_SWAP
    }
    uint64_t best = kKeyNone;
    if (act) {
        if (PACK5) {
            if (mF != 0xFFFFFFFFu) {
                const int d = (int)((mF >> 5) & 0x3FFFFFFu) - kPackBias;
                const int jw = j0 + c.prank[j0 + (int)(mF & 31u)];
                const uint32_t mj = c.seq[jw];
                const uint32_t a = min((uint32_t)mi, mj), bm = max((uint32_t)mi, mj);
                best = pack_key((mF >> 31) != 0, d, lidx_swap(a, bm));
            }
        } else {
            if (mF != 0xFFFFFFFFu) {
                const int d = (int)(mF >> 6) - kPackBias;
                const int jw = j0 + c.prank[j0 + (int)(mF & 63u)];
                const uint32_t mj = c.seq[jw];
                const uint32_t a = min((uint32_t)mi, mj), bm = max((uint32_t)mi, mj);
                best = pack_key(false, d, lidx_swap(a, bm));
            }
            if (mT != 0xFFFFFFFFu) {
                const int d = (int)(mT >> 6) - kPackBias;
                const int jw = j0 + c.prank[j0 + (int)(mT & 63u)];
                const uint32_t mj = c.seq[jw];
                const uint32_t a = min((uint32_t)mi, mj), bm = max((uint32_t)mi, mj);
                best = umin64(best, pack_key(!(d < thr), d, lidx_swap(a, bm)));
            }
        }
    }
    return best;
}

// Deal eval units round-robin over the TW wavefronts of the solve; gw is this
// wavefront's rank.  Units are numbered tile by tile (a tile's relocate units,
// then its swap units); a wavefront walks the tiles once, jumping straight to
// each of its units.  Returns this lane's minimum key.
// Where a wavefront's units begin: the tile of unit gw and the number of that
// tile's first unit, and the solve's unit count (fixed for a solve, so computed
// once instead of walking the tiles every iteration).
struct UnitStart { int tl, u, n; };

__device__ __forceinline__ UnitStart unit_start(const Ctx &c, int gw)
{
    const int nT = (c.M + kWave - 1) / kWave;
    const int nRC = (c.NG + c.rchunk - 1) / c.rchunk;
    UnitStart s{nT, 0, 0};
    for (int tl = 0; tl < nT; ++tl) {
        const int nU = nRC + (c.M - tl * kWave + c.chunk - 1) / c.chunk;
        if (s.tl == nT && gw < s.n + nU) { s.tl = tl; s.u = s.n; }
        s.n += nU;
    }
    return s;
}

template <typename TE, typename TB, bool FLAT = false>
__device__ __forceinline__ uint64_t eval_all(const Ctx &c, const TE *tc, const TB *tabu, int gw,
                                             int TW, const UnitStart &us, int lane, int t, int thr,
                                             bool use_tabu)
{
    uint64_t best = kKeyNone;
    const int CH = c.chunk, RCH = c.rchunk;
    const int nT = (c.M + kWave - 1) / kWave;
    const int nRC = (c.NG + RCH - 1) / RCH;
    const int lgCH = __builtin_ctz((unsigned)CH);   // CH: a power of two
    int tl = us.tl, u = us.u;   // u: number of the first unit of tile tl
    for (int mine = gw; mine < us.n; mine += TW) {
        while (tl < nT) {
            const int nSC = (c.M - tl * kWave + CH - 1) >> lgCH;
            if (mine < u + nRC + nSC) break;
            u += nRC + nSC;
            ++tl;
        }
        if (tl >= nT) break;
        const int k = mine - u;
        const int jb = tl * kWave;
        if (k < nRC) {
            const int rlo = __builtin_amdgcn_readfirstlane(c.rt[jb]);
            const int rhi = __builtin_amdgcn_readfirstlane(c.rt[min(c.M, jb + kWave) - 1]);
            const int G0 = k * RCH, G1 = min(c.NG, G0 + RCH);
            if constexpr (FLAT && sizeof(TE) == 2)
                best = umin64(best, relocate_unit_flat<TE, TB>(c, tc, tabu, tl, G0, G1, lane, t, thr,
                                                               use_tabu));
            else
                best = umin64(best, relocate_unit<TE, TB>(c, tc, tabu, tl, G0, G1, lane, t, thr,
                                                          use_tabu, rlo, rhi));
        } else {
            const int j0 = jb + (k - nRC) * CH, j1 = min(c.M, j0 + CH);
            if (CH <= 32)
                best = umin64(best, swap_unit<TE, TB, true>(c, tc, tabu, tl, j0, j1, lane, t, thr, use_tabu));
            else
                best = umin64(best, swap_unit<TE, TB, false>(c, tc, tabu, tl, j0, j1, lane, t, thr, use_tabu));
        }
    }
    return best;
}

// ---------------------------------------------------------------------------
// every slot's key, one move at a time (test hook; no segment tricks)
// ---------------------------------------------------------------------------
template <typename TE>
__device__ void dump_keys(const Ctx &c, const TE *tc, const int32_t *tabu, int tid, int nthr, int t,
                          int thr, bool use_tabu, uint64_t *keys)
{
    const int M = c.M;
    for (int i = tid; i < M; i += nthr) {
        const int4 pa = c.posA[i], pb = c.posB[i];
        const int m = pb.z & 0xFFFF, ri = (int)((uint32_t)pb.z >> 16);
        const int rem = pb.y - pb.x;
        for (int G = 0; G < c.NG; ++G) {
            const int4 g = c.gap[G];
            const int d = rem + (int)tc[g.x + pa.y] + (int)tc[pa.x + g.y] - g.z;
            const bool noop = (unsigned)(G - (i + ri)) < 2u;
            const bool tb = use_tabu && tabu[(g.w & 0xFFFF) * M + m] > t;
            keys[(uint32_t)m * c.NG + G] = noop ? kKeyNone : pack_key(tb && !(d < thr), d, (uint32_t)m * c.NG + G);
        }
        for (int j = i + 1; j < M; ++j) {
            const int4 a = c.posA[j], b = c.posB[j];
            const int mj = b.z & 0xFFFF, rj = (int)((uint32_t)b.z >> 16);
            int d;
            if (j == i + 1 && ri == rj)
                d = (int)tc[pa.z + a.y] + (int)tc[a.x + pa.y] + (int)tc[pa.x + a.w]
                  - ((int)tc[pa.z + pa.y] + (int)tc[pa.x + a.y] + (int)tc[a.x + a.w]);
            else
                d = (int)tc[pa.z + a.y] + (int)tc[a.x + pa.w] + (int)tc[a.z + pa.y] + (int)tc[pa.x + a.w]
                  - pb.x - b.x;
            const bool tb = use_tabu && (tabu[rj * M + m] > t || tabu[ri * M + mj] > t);
            const uint32_t idx = swap_index(c.R, (uint32_t)M, (uint32_t)min(m, mj), (uint32_t)max(m, mj));
            keys[idx] = pack_key(tb && !(d < thr), d, idx);
        }
    }
}

// ---------------------------------------------------------------------------
// LDS setup
// ---------------------------------------------------------------------------
__device__ __forceinline__ Ctx make_ctx(char *smem, const Lay &ly, int M, int V, int chunk, int rchunk, int Cs)
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
    c.posA = (int4 *)(smem + ly.posA);
    c.posB = (int4 *)(smem + ly.posB);
    c.gap = (int4 *)(smem + ly.gap);
    c.gend = (uint16_t *)(smem + ly.gend);
    c.prank = (uint8_t *)(smem + ly.prank);
    c.posC = nullptr;
    c.red = (uint64_t *)(smem + ly.red);
    c.M = M;
    c.V = V;
    c.NG = M + V;
    c.chunk = chunk;
    c.rchunk = rchunk;
    c.Cs = Cs;
    c.R = (uint32_t)M * (uint32_t)(M + V);
    return c;
}

template <typename TE>
__device__ __forceinline__ void load_instance(const InstDev &I, const Ctx &c, TE *tc, int tid, int nthr)
{
    const int words = (int)(((int64_t)I.R * I.Cs * (int64_t)sizeof(TE)) / 4);
    const uint32_t *src = (const uint32_t *)I.tc;
    uint32_t *dst = (uint32_t *)tc;
    for (int k = tid; k < words; k += nthr) dst[k] = src[k];
    for (int k = tid; k < c.M; k += nthr) { c.mrow[k] = I.mrow[k]; c.mcol[k] = I.mcol[k]; }
    for (int k = tid; k < c.V; k += nthr) { c.vrow[k] = I.vrow[k]; c.vcol[k] = I.vcol[k]; }
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
template <typename TE, bool WAVE = false>
__device__ int64_t greedy(const Ctx &c, const TE *tc, uint64_t seed, int64_t svc_sum, int tid,
                          int nthr)
{
    const int M = c.M, V = c.V;
    int32_t *scr = (int32_t *)c.posA;      // 4M ints
    int32_t *pi = scr, *draw = scr + M, *veh = scr + 2 * M;
    int32_t *scv = (int32_t *)c.gap;       // 4(M+V) ints
    int32_t *lastx = scv, *cnt = scv + V, *curv = scv + 2 * V;
    for (int i = tid; i < M; i += nthr) {
        pi[i] = i;
        if (i >= 1) draw[i] = (int32_t)(splitmix_at(seed, (uint64_t)(M - i)) % (uint64_t)(i + 1));
    }
    for (int v = tid; v < V; v += nthr) { lastx[v] = c.vrow[v]; cnt[v] = 0; }
    bsync<WAVE>();
    if (seed != 0 && tid == 0) {
        for (int i = M - 1; i >= 1; --i) {
            const int j = draw[i];
            const int tmp = pi[i]; pi[i] = pi[j]; pi[j] = tmp;
        }
    }
    bsync<WAVE>();
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
        if (lane == 0) c.red[100] = (uint64_t)acc;
    }
    bsync<WAVE>();
    if (tid == 0) {
        int o = 0;
        for (int v = 0; v < V; ++v) { c.off[v] = o; curv[v] = o; o += cnt[v]; }
        c.off[V] = o;
        for (int s = 0; s < M; ++s) {
            const int v = veh[s];
            c.seq[curv[v]++] = (uint16_t)pi[s];
        }
    }
    bsync<WAVE>();
    index_routes(c, tid, nthr);
    const int64_t acc = (int64_t)c.red[100];
    bsync<WAVE>();
    return acc + svc_sum;
}

// The missions' steps of greedy_staged with the per-vehicle state in registers:
// lane l holds vehicles l, l + 64, ... (VPL of them, V <= 64 VPL) with their
// route end, return leg and count, so a step is one round of travel gathers
// (all of a lane's issued together), one wavefront minimum and the winner's
// lane updating its own registers; the next mission's row and column are read
// a step ahead.  Writes each step's vehicle and rank, and each vehicle's count;
// returns the sum of the added times.  M >= 1.
template <typename TE, int VPL>
__device__ int64_t greedy_steps_regs(const Ctx &c, const TE *tc, bool seeded, const int32_t *pi,
                                     int32_t *cnt, uint16_t *veh, uint16_t *rnk, int lane)
{
    const int M = c.M, V = c.V;
    const auto g = [](const TE *p, int k) { return (int)gld(p)[k]; };
    int lx[VPL], vc[VPL], ec[VPL], n[VPL];
#pragma unroll
    for (int j = 0; j < VPL; ++j) {
        // lanes past the fleet read the last vehicle and never take part
        const int v = min(lane + j * kWave, V - 1);
        lx[j] = gld(c.vrow)[v];
        vc[j] = gld(c.vcol)[v];
        n[j] = 0;
    }
#pragma unroll
    for (int j = 0; j < VPL; ++j) ec[j] = g(tc, lx[j] + vc[j]);
    int64_t acc = 0;
    int mn = seeded ? pi[0] : 0;
    int mcn = gld(c.mcol)[mn], mrn = gld(c.mrow)[mn];
    for (int s = 0; s < M; ++s) {
        const int mc = mcn, mr = mrn;
        if (s + 1 < M) {
            mn = seeded ? pi[s + 1] : s + 1;
            mcn = gld(c.mcol)[mn];
            mrn = gld(c.mrow)[mn];
        }
        int a[VPL], r[VPL];
#pragma unroll
        for (int j = 0; j < VPL; ++j) {
            a[j] = g(tc, lx[j] + mc);
            r[j] = g(tc, mr + vc[j]);
        }
        uint64_t k = kKeyNone;
        int kj = 0;
#pragma unroll
        for (int j = 0; j < VPL; ++j) {
            const int v = lane + j * kWave;
            const uint64_t kv = v < V ? ((uint64_t)(uint32_t)(a[j] + r[j] - ec[j] + kDeltaBias) << 32) | (uint32_t)v
                                      : kKeyNone;
            if (kv < k) { k = kv; kj = j; }
        }
        const uint64_t kw = wave_min(k);
        acc += (int64_t)(int32_t)(uint32_t)(kw >> 32) - kDeltaBias;
        if (kw == k) {   // the winner's lane (keys are unique: they hold the vehicle)
            int rank = 0;
#pragma unroll
            for (int j = 0; j < VPL; ++j)
                if (j == kj) {
                    rank = n[j];
                    n[j] = rank + 1;
                    lx[j] = mr;
                    ec[j] = r[j];   // the return leg after the new last mission
                }
            veh[s] = (uint16_t)(uint32_t)kw;
            rnk[s] = (uint16_t)rank;
        }
    }
#pragma unroll
    for (int j = 0; j < VPL; ++j)
        if (lane + j * kWave < V) cnt[lane + j * kWave] = n[j];
    return acc;
}

// Algorithm 1 as greedy() computes it, for the HBM-resident schedule: the
// per-mission results (vehicle, rank within the vehicle) live in the
// workgroup's LDS `lds` (at least greedy_staged_bytes), and so does the
// per-vehicle state (route end, return leg, count) beyond 256 vehicles (up to
// 256 it stays in registers: greedy_steps_regs), so each mission's step waits
// only for its travel gathers from HBM (one round of them: the next mission's
// row and column are read a step ahead; the winner's new return leg is the
// gather its lane already made); the routes are then written by all threads at
// once, each mission at its vehicle's offset plus its rank.  Returns the
// objective.
__host__ __device__ inline uint32_t greedy_staged_bytes(int M, int V, bool seeded)
{
    return 16u * (uint32_t)V + 4u * (uint32_t)M + (seeded ? 8u * (uint32_t)M : 0u) + 64u;
}

template <typename TE>
__device__ int64_t greedy_staged(const Ctx &c, const TE *tc, uint64_t seed, int64_t svc_sum, char *lds,
                                 int tid, int nthr)
{
    const int M = c.M, V = c.V;
    int32_t *lastx = (int32_t *)lds, *endc = lastx + V, *cnt = endc + V, *vcl = cnt + V;
    uint16_t *veh = (uint16_t *)(vcl + V), *rnk = veh + M;
    int32_t *pi = (int32_t *)(rnk + M + (M & 1)), *drw = pi + M;     // seeded only
    int64_t *acc_out = (int64_t *)c.red;
    const auto g = [](const TE *p, int k) { return (int)gld(p)[k]; };
    for (int v = tid; v < V; v += nthr) {
        const int x = gld(c.vrow)[v], vc = gld(c.vcol)[v];
        lastx[v] = x;
        vcl[v] = vc;
        endc[v] = g(tc, x + vc);
        cnt[v] = 0;
    }
    if (seed != 0)
        for (int i = tid; i < M; i += nthr) {
            pi[i] = i;
            if (i >= 1) drw[i] = (int32_t)(splitmix_at(seed, (uint64_t)(M - i)) % (uint64_t)(i + 1));
        }
    __syncthreads();
    if (seed != 0 && tid == 0)
        for (int i = M - 1; i >= 1; --i) {
            const int j = drw[i];
            const int tmp = pi[i]; pi[i] = pi[j]; pi[j] = tmp;
        }
    __syncthreads();
    if (tid < kWave && M > 0 && V <= 4 * kWave) {
        const int lane = tid;
        int64_t acc;
        if (V <= kWave) acc = greedy_steps_regs<TE, 1>(c, tc, seed != 0, pi, cnt, veh, rnk, lane);
        else if (V <= 2 * kWave) acc = greedy_steps_regs<TE, 2>(c, tc, seed != 0, pi, cnt, veh, rnk, lane);
        else acc = greedy_steps_regs<TE, 4>(c, tc, seed != 0, pi, cnt, veh, rnk, lane);
        if (lane == 0) acc_out[100] = acc;
    } else if (tid < kWave) {
        const int lane = tid;
        int64_t acc = 0;
        int mn = M > 0 ? (seed ? pi[0] : 0) : 0;
        int mcn = M > 0 ? gld(c.mcol)[mn] : 0, mrn = M > 0 ? gld(c.mrow)[mn] : 0;
        for (int s = 0; s < M; ++s) {
            const int mc = mcn, mr = mrn;
            if (s + 1 < M) {
                mn = seed ? pi[s + 1] : s + 1;
                mcn = gld(c.mcol)[mn];
                mrn = gld(c.mrow)[mn];
            }
            // each lane keeps the return leg of its own best vehicle: the winner's
            // lane then has the new route end without another gather
            uint64_t k = kKeyNone;
            int kret = 0;
            for (int v = lane; v < V; v += kWave) {
                const int x = lastx[v], vc = vcl[v];
                const int ret = g(tc, mr + vc);
                const int add = g(tc, x + mc) + ret - endc[v];
                const uint64_t kv = ((uint64_t)(uint32_t)(add + kDeltaBias) << 32) | (uint32_t)v;
                if (kv < k) { k = kv; kret = ret; }
            }
            const uint64_t kw = wave_min(k);
            const int vs = (int)(uint32_t)kw;
            acc += (int64_t)(int32_t)(uint32_t)(kw >> 32) - kDeltaBias;
            if (kw == k) {   // the winner's lane (keys are unique: they hold the vehicle)
                const int r = cnt[vs];
                endc[vs] = kret;
                lastx[vs] = mr;
                cnt[vs] = r + 1;
                veh[s] = (uint16_t)vs;
                rnk[s] = (uint16_t)r;
            }
            bsync<true>();
        }
        if (lane == 0) acc_out[100] = acc;
    }
    __syncthreads();
    if (tid == 0) {
        int o = 0;
        for (int v = 0; v < V; ++v) {
            const int n = cnt[v];
            cnt[v] = o;
            gst(c.off)[v] = o;
            o += n;
        }
        gst(c.off)[V] = o;
    }
    __syncthreads();
    for (int s2 = tid; s2 < M; s2 += nthr) {
        const int v = veh[s2], m = seed ? pi[s2] : s2, q = cnt[v] + rnk[s2];
        gst(c.seq)[q] = (uint16_t)m;
        gst(c.rt)[q] = (uint16_t)v;
        gst(c.pof)[m] = (uint16_t)q;
        gst(c.rof)[m] = (uint16_t)v;
    }
    const int64_t acc = acc_out[100];
    __syncthreads();
    return acc + svc_sum;
}

// write the current routes (and, when `of` is given, each mission's vehicle)
__device__ __forceinline__ void write_routes(const Ctx &c, int32_t *off, int32_t *seq, int32_t *of,
                                             int tid, int nthr)
{
    for (int i = tid; i < c.M; i += nthr) {
        const int m = c.seq[i];
        seq[i] = m;
        if (of) of[m] = c.rt[i];
    }
    for (int v = tid; v <= c.V; v += nthr) off[v] = c.off[v];
}

// write the current routes as the best solution
__device__ __forceinline__ void snapshot(const Ctx &c, const JobDev &J, int tid, int nthr)
{
    write_routes(c, J.out_off, J.out_seq, J.out_of, tid, nthr);
}

// ---------------------------------------------------------------------------
// one solve, state in LDS.  MULTI: gridDim.x workgroups cooperate on job[0].
// ---------------------------------------------------------------------------
// The move an iteration applies, decoded by wave 0 of each workgroup
// (LDS schedules) or by every thread (global schedule).
struct GMove {
    int kind;                  // 0 none, 1 relocate, 2 swap
    int m, v, q, lo, hi, dir;  // relocate: mission, target vehicle, final position, shifted range and shift
    int rs;                    // relocate: the mission's vehicle before the move
    int s1, s2, m1, m2;        // swap: the two positions and their missions
};

// Apply a decoded move to the LDS state with one wavefront.  A relocate moves
// every entry between the old and the new place by one position (each takes its
// neighbour's mission and vehicle: only the moved mission changes vehicle), 512
// positions at a time read into registers and then written, the chunks taken in
// the direction of the shift so that no chunk reads what an earlier one wrote;
// the route offsets between the two vehicles move by one.  A swap exchanges two
// entries.
__device__ __forceinline__ void apply_wave(const Ctx &c, const GMove &mv, int lane)
{
    if (mv.kind == 1) {
        constexpr int U = 8;
        const int lo = mv.lo, hi = mv.hi, q = mv.q, n = hi - lo + 1;
        const bool up = mv.dir > 0;
        // the offsets of the routes after the left one, up to the right one, move by
        // one: the first 64 are read here, beside the shifted entries, and written
        // with them
        const int rlo = min(mv.v, mv.rs) + 1, rhi = max(mv.v, mv.rs), dlt = mv.v > mv.rs ? -1 : 1;
        const int r0 = rlo + lane;
        const int o0 = r0 <= rhi ? c.off[r0] : 0;
        for (int c0 = 0; c0 < n; c0 += U * kWave) {
            int val[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int ix = c0 + u * kWave + lane;
                const int kk = up ? lo + ix : hi - ix;
                const int src = up ? kk + 1 : kk - 1;
                val[u] = ix >= n ? 0
                       : kk == q ? (mv.m | (mv.v << 16)) : ((int)c.seq[src] | ((int)c.rt[src] << 16));
            }
            // lanes read what their neighbours then overwrite: keep every read of the
            // chunk ahead of its writes, and its writes ahead of the next chunk's reads
            __asm__ volatile("" ::: "memory");
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int ix = c0 + u * kWave + lane;
                if (ix < n) {
                    const int kk = up ? lo + ix : hi - ix;
                    const int mm = val[u] & 0xFFFF, r = (int)((uint32_t)val[u] >> 16);
                    c.seq[kk] = (uint16_t)mm;
                    c.rt[kk] = (uint16_t)r;
                    c.pof[mm] = (uint16_t)kk;
                    c.rof[mm] = (uint16_t)r;
                }
            }
            __asm__ volatile("" ::: "memory");
        }
        if (r0 <= rhi) c.off[r0] = o0 + dlt;
        for (int r = r0 + kWave; r <= rhi; r += kWave) c.off[r] += dlt;
    } else if (mv.kind == 2 && lane == 0) {
        c.seq[mv.s1] = (uint16_t)mv.m2;
        c.seq[mv.s2] = (uint16_t)mv.m1;
        c.pof[mv.m1] = (uint16_t)mv.s2;
        c.pof[mv.m2] = (uint16_t)mv.s1;
        c.rof[mv.m1] = (uint16_t)mv.rs;
        c.rof[mv.m2] = (uint16_t)mv.v;
    }
}

// Exchange polling of the multi-workgroup schedule (wave 0 of a workgroup, all
// lanes active): the minimum of the keys in the nwg slots (one per 128-byte line)
// once every slot carries `tag`, or kKeyNone with ab = 1 when give_up(spins) says
// so.  NQ slots per lane (2 up to 128 workgroups, else 4: kMaxGroups = 4 x 64),
// two loads of each in flight: the older is checked while the newer travels, so a
// slot is seen about half a round trip sooner after it is written than with one
// load at a time (a third load in flight measured slower).  Every lane loads every
// round (lanes past the last slot reread slot 0 and ignore it): no branch around a
// load, so only the older loads are waited for.
template <typename GiveUp>
__device__ __forceinline__ uint64_t poll_slots(const uint64_t *slots, int nwg, uint64_t tag, int lane,
                                               uint32_t &ab, GiveUp give_up)
{
    static_assert(kMaxGroups <= 4 * kWave, "four slots per lane");
    uint64_t bestk = kKeyNone;
    ab = 0;
    auto run = [&](auto nq) {
        constexpr int NQ = decltype(nq)::value;
        uint64_t v[NQ], va[NQ], vb[NQ];
        bool ready[NQ];
        const uint64_t *src[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int w = q * kWave + lane;
            ready[q] = w >= nwg;
            src[q] = &slots[(w < nwg ? w : 0) * kSlotStride];
            v[q] = 0;
        }
        auto reload = [&](uint64_t (&x)[NQ]) {
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                x[q] = __hip_atomic_load(src[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        };
        auto check = [&](const uint64_t (&x)[NQ]) {
            bool all = true;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const bool now = !ready[q] && (x[q] >> 63) == tag;
                v[q] = now ? x[q] : v[q];
                ready[q] = ready[q] || now;
                all = all && ready[q];
            }
            return __all(all);
        };
        reload(va);
        __builtin_amdgcn_s_sleep(4);
        reload(vb);
        uint32_t spins = 0;
        // unrolled by two, so that neither load is copied: check the older, reload
        // it, check the other
        for (;;) {
            if (check(va)) break;
            if (give_up(++spins)) { ab = 1; break; }
            reload(va);
            if (check(vb)) break;
            if (give_up(++spins)) { ab = 1; break; }
            reload(vb);
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (q * kWave + lane < nwg && ready[q]) bestk = umin64(bestk, decode_slot(v[q]));
    };
    if (nwg <= 2 * kWave)
        run(std::integral_constant<int, 2>{});
    else
        run(std::integral_constant<int, 4>{});
    return bestk;
}

template <typename TE, typename TB, bool MULTI, bool WAVE = false>
__device__ __forceinline__ void run_job(const JobDev &J, char *smem, int wg, int nwg, Xchg *xs)
{
    const InstDev &I = *J.inst;
    // WAVE: one wavefront runs the solve in its own LDS region
    const int tid = WAVE ? (int)(threadIdx.x & (kWave - 1)) : (int)threadIdx.x;
    const int nthr = WAVE ? kWave : (int)blockDim.x;
    const int lane = tid & (kWave - 1), wave = wave_id(tid), nwaves = nthr / kWave;
    const int M = uniform(I.M), V = uniform(I.V), R = uniform(I.R), Cs = uniform(I.Cs);
    const Lay ly = lds_layout(M, V, R, Cs, (int)sizeof(TE), (int)sizeof(TB));
    const Ctx c = make_ctx(smem, ly, M, V, J.chunk, J.rchunk, Cs);
    TE *tc = (TE *)(smem + ly.tc);
    TB *tabu = (TB *)(smem + ly.tabu);
    const bool writer = !MULTI || wg == 0;

    load_instance<TE>(I, c, tc, tid, nthr);
    bsync<WAVE>();

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
        bsync<WAVE>();
        index_routes(c, tid, nthr);
        bsync<WAVE>();
    } else {
        cur = greedy<TE, WAVE>(c, tc, J.seed, I.svc_sum, tid, nthr);
        for (int k = tid; k < M * V; k += nthr) tabu[k] = (TB)0;
        best = cur;
        best_iter = -1;
        stopped = 0;
        if (writer) snapshot(c, J, tid, nthr);
        bsync<WAVE>();
    }

    const bool use_tabu = J.variant == AT_TABU;
    const int gw = wg * nwaves + wave, TW = nwaves * nwg;
    const UnitStart us0 = unit_start(c, gw);
    int t = J.t_begin;
    bool aborted = false;
    // the thread that sets each move's tabu entries and writes the trace: lane 0 of
    // the first wavefront with no position to prepare, when there is one
    const int tx = (M + kWave - 1) / kWave * kWave < nthr ? (M + kWave - 1) / kWave * kWave : 0;
    // the per-gap route ends serve the segmented relocate units only (the
    // multi-workgroup schedule's units with 16-bit entries have no segments)
    constexpr bool kGend = !(MULTI && sizeof(TE) == 2);
    if (t < J.t_end && !stopped) {
        prep<TE, kGend>(c, tc, tid, nthr);
        bsync<WAVE>();
    }
    for (; t < J.t_end && !stopped; ++t) {
        int thr = INT32_MIN;
        if (J.aspiration) {
            const int64_t g = best - cur;
            thr = g < (int64_t)INT32_MIN ? INT32_MIN : (int)g;
        }
        uint64_t k = eval_all<TE, TB, MULTI>(c, tc, tabu, gw, TW, us0, lane, t, thr, use_tabu);
        k = wave_min(k);
        if (lane == 0) c.red[wave] = k;
        bsync<WAVE>();
        GMove mv{};
        if (tid < kWave) {
            uint64_t w = lane < nwaves ? c.red[lane] : kKeyNone;
            w = wave_min(w);
            uint32_t xab = 0;   // the exchange gave up waiting (uniform over the wave)
            if (MULTI) {
                // Each workgroup publishes its minimum in its own slot, tagged with
                // bit 1 of the iteration; wave 0 of every workgroup polls all slots
                // (poll_slots) until every tag matches.  A workgroup can be at
                // most one iteration ahead of another, so parity buffers plus the tag
                // never confuse iterations t and t+2.
                const int rel = t - J.t_begin;
                const uint64_t tag = (uint64_t)((rel >> 1) & 1);
                uint64_t *slots = xs->slots[J.mx][rel & 1];
                if (lane == 0)
                    __hip_atomic_store(&slots[wg * kSlotStride], encode_slot(w, tag), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                uint32_t ab = 0;
                const uint64_t bestk = poll_slots(slots, nwg, tag, lane, ab,
                                                  [](uint32_t spins) { return spins > kSpinLimit; });
                w = wave_min(bestk);
                xab = ab;
                if (lane == 0) c.red[65] = ab;
            }
            if (lane == 0) {
                c.red[64] = w;
                c.red[66] = 0;   // no move (kind 0) unless one is decoded below
            }
            if (!xab && w != kKeyNone) {
                // decode the move (uniform over the wave) and apply it
                const uint32_t ix = (uint32_t)w;
                if (!(ix >> 31)) {
                    const int m = (int)(ix >> 16);
                    const int G = (int)(ix & 0xFFFFu);
                    const int v = c.gap[G].w & 0xFFFF;
                    const int s = c.pof[m];
                    const int rs = c.rof[m];          // loads alongside pof[m]
                    const int fp = G - v;             // off[v] + (G - off[v] - v)
                    const int q = fp - (fp > s ? 1 : 0);
                    mv.kind = 1;
                    mv.m = m; mv.v = v; mv.q = q; mv.rs = rs;
                    mv.lo = min(s, q); mv.hi = max(s, q); mv.dir = q >= s ? 1 : -1;
                } else {
                    const int m1 = (int)((ix >> 16) & 0x7FFFu), m2 = (int)(ix & 0xFFFFu);
                    const int s1 = c.pof[m1], s2 = c.pof[m2];
                    const int r1 = c.rof[m1], r2 = c.rof[m2];
                    mv.kind = 2;
                    mv.s1 = s1; mv.s2 = s2; mv.m1 = m1; mv.m2 = m2;
                    mv.v = r1; mv.rs = r2;            // the two vehicles
                }
                // the move for the thread that sets its tabu entries (below)
                if (lane == 0) {
                    c.red[66] = (uint64_t)mv.kind | ((uint64_t)(mv.kind == 1 ? mv.m : mv.m1) << 16) |
                                ((uint64_t)mv.v << 32) | ((uint64_t)mv.rs << 48);
                    c.red[67] = (uint64_t)mv.m2;
                }
                // apply it before the barrier that publishes the key (the neighbourhood
                // search stops without applying a move that does not improve)
                const int dw = (int)((uint32_t)(w >> 32) & 0x7FFFFFFFu) - kDeltaBias;
                if (use_tabu || dw < 0) apply_wave(c, mv, lane);
            }
        }
        bsync<WAVE>();   // the move is decoded and applied
        if (MULTI && c.red[65]) { aborted = true; break; }
        const uint64_t key = c.red[64];
        uint32_t tr_idx = 0xFFFFFFFFu;   // this iteration's trace record (thread 0)
        int tr_d = 0;
        uint8_t tr_fl = 0;
        if (key == kKeyNone) {
            // no move exists (at most one mission on a single vehicle)
            if (!use_tabu) { stopped = 1; break; }
        } else {
            const bool blocked = (key >> 63) != 0;
            const int d = (int)((uint32_t)(key >> 32) & 0x7FFFFFFFu) - kDeltaBias;
            const uint32_t idx = (uint32_t)key;
            if (!use_tabu && d >= 0) { stopped = 1; break; }
            cur += d;
            tr_idx = idx;
            tr_d = d;
            tr_fl = (uint8_t)(((idx >> 31) ? 1 : 0) | (blocked ? 4 : 0));
            if (cur < best) {
                best = cur;
                best_iter = t;
                if (writer) snapshot(c, J, tid, nthr);
            }
        }
        // the next iteration's records (they depend on the routes only)
        if (t + 1 < J.t_end) prep<TE, kGend>(c, tc, tid, nthr);
        if (tid == tx) {
            // one thread reads whether the move was tabu and makes the moved missions
            // tabu for the vehicles they leave: nothing reads the tabu table before
            // the next eval, after the barrier below.  It is a thread with no records
            // to write when there is one, so its round trips stay off the barrier's path
            bool was_tabu = false;
            const uint64_t p0 = c.red[66];
            const int kind = (int)(p0 & 0xFFFFu);
            if (use_tabu && kind != 0) {
                const int tval = t + J.tenure + 1;
                const int m1 = (int)((p0 >> 16) & 0xFFFFu), v = (int)((p0 >> 32) & 0xFFFFu);
                const int rs = (int)(p0 >> 48);
                if (kind == 1) {
                    was_tabu = (int)tabu[v * M + m1] > t;
                    tabu[rs * M + m1] = (TB)tval;
                } else {
                    const int m2 = (int)(c.red[67] & 0xFFFFu);
                    was_tabu = (int)tabu[rs * M + m1] > t || (int)tabu[v * M + m2] > t;
                    tabu[v * M + m1] = (TB)tval;
                    tabu[rs * M + m2] = (TB)tval;
                }
            }
            if (writer && J.trace) {
                const bool blocked = (tr_fl & 4) != 0;
                J.tr_move[t] = tr_idx == 0xFFFFFFFFu ? tr_idx : lidx_slot(tr_idx, c.R, (uint32_t)M, (uint32_t)c.NG);
                J.tr_delta[t] = tr_d;
                J.tr_obj[t] = cur;
                J.tr_flags[t] = (uint8_t)(tr_fl | ((was_tabu && !blocked) ? 2 : 0));
            }
        }
        bsync<WAVE>();   // the records and the tabu entries are written
    }
    if (!writer) return;
    if (J.fin_off && !aborted) write_routes(c, J.fin_off, J.fin_seq, nullptr, tid, nthr);
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

// ---------------------------------------------------------------------------
// global schedule: state in HBM.  Each solve runs on its own range of the
// launch's workgroups, which meet at two barriers per iteration: after the
// argmin exchange, and after the move is applied and the next iteration's
// records are written.
// ---------------------------------------------------------------------------
constexpr uint64_t kBarrierTicks = 20ull * 100000000ull;   // 20 s of the 100 MHz wall clock

// Barrier and argmin exchange of the workgroups of one HBM-resident solve.
// Each workgroup publishes its minimum key in its own slot of the barrier's
// buffer (barrier b uses buffer b & 1), tagged with bit 1 of b; wave 0 polls
// every slot (one lane per slot) until all carry the tag, and the minimum of
// all keys goes to every thread.  A workgroup is at most one barrier ahead of
// any other, so parity buffers plus the tag never confuse barrier b with b + 2;
// no two workgroups write one address, so arrivals do not queue on an atomic.
// Waits are bounded by wall clock: a workgroup that runs out sets the solve's
// abort flag, which every waiter sees.  Returns false on abort.
__device__ __forceinline__ bool group_exchange(GlobalBufs &B, int wg, int nwg, uint32_t &nb, uint64_t key,
                                               uint64_t *red, uint64_t &out)
{
    // every wavefront's global writes are complete before the slot is published
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    const uint32_t b = nb++;
    const uint64_t tag = (b >> 1) & 1u;
    uint64_t *slots = B.slots + (size_t)(b & 1) * kMaxGroups * kSlotStride;
    if (threadIdx.x < kWave) {
        const int lane = threadIdx.x;
        if (lane == 0)
            __hip_atomic_store(&slots[wg * kSlotStride], encode_slot(key, tag), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
        // one load per slot at a time: with up to 256 workgroups polling, a second
        // load in flight per slot (as in the multi-workgroup exchange) measured slower
        const uint64_t t0 = wall_clock64();
        uint64_t best = kKeyNone;
        uint32_t ab = 0, spins = 0;
        for (int base = 0; base < nwg && !ab; base += kWave) {
            const int w2 = base + lane;
            bool ready = w2 >= nwg;
            uint64_t v = ~0ull;
            for (;;) {
                if (!ready) {
                    v = __hip_atomic_load(&slots[w2 * kSlotStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ready = (v >> 63) == tag;
                }
                if (__all(ready)) break;
                if ((++spins & 63u) == 0) {
                    ab = __hip_atomic_load(&B.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (!ab && wall_clock64() - t0 > kBarrierTicks) {
                        if (lane == 0) __hip_atomic_store(&B.abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ab = 1;
                    }
                    if (ab) break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            if (w2 < nwg && ready) best = umin64(best, decode_slot(v));
        }
        best = wave_min(best);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (lane == 0) {
            red[66] = ab;
            red[67] = best;
        }
    }
    __syncthreads();
    out = red[67];
    return red[66] == 0;
}

// Routes of parity p (p = 0, 1: double-buffered) and the records built from them.
__device__ __forceinline__ Ctx global_ctx(const InstDev &I, const GlobalBufs &B, int p, uint64_t *red)
{
    Ctx c;
    c.mrow = I.mrow;
    c.mcol = I.mcol;
    c.vrow = I.vrow;
    c.vcol = I.vcol;
    c.off = B.off[p];
    c.seq = B.seq[p];
    c.rt = B.rt[p];
    c.rof = B.rof[p];
    c.pof = B.pof[p];
    c.posA = B.posA[p];
    c.posB = B.posB[p];
    c.gap = B.gap[p];
    c.gend = nullptr;
    c.posC = B.posC[p];
    c.prank = nullptr;
    c.red = red;
    c.M = uniform(I.M);
    c.V = uniform(I.V);
    c.NG = c.M + c.V;
    c.chunk = 0;
    c.rchunk = 0;
    c.Cs = uniform(I.Cs);
    c.R = (uint32_t)c.M * (uint32_t)c.NG;
    return c;
}

// Mission, vehicle and route offsets of the routes after `mv`, read from the
// routes before it (o): the missions between the old and new position of a
// relocated mission shift by one place; a swap exchanges two entries.
__device__ __forceinline__ int next_seq(const Ctx &o, const GMove &mv, int k)
{
    if (mv.kind == 1) {
        if (k == mv.q) return mv.m;
        return gld(o.seq)[(k >= mv.lo && k <= mv.hi) ? k + mv.dir : k];
    }
    if (mv.kind == 2) {
        if (k == mv.s1) return mv.m2;
        if (k == mv.s2) return mv.m1;
    }
    return gld(o.seq)[k];
}

__device__ __forceinline__ int next_rt(const Ctx &o, const GMove &mv, int k)
{
    if (mv.kind == 1) {
        if (k == mv.q) return mv.v;
        return gld(o.rt)[(k >= mv.lo && k <= mv.hi) ? k + mv.dir : k];
    }
    return gld(o.rt)[k];
}

__device__ __forceinline__ int next_off(const Ctx &o, const GMove &mv, int r)
{
    int x = gld(o.off)[r];
    if (mv.kind == 1) {
        if (mv.v > mv.rs && r > mv.rs && r <= mv.v) x -= 1;
        if (mv.v < mv.rs && r > mv.v && r <= mv.rs) x += 1;
    }
    return x;
}

// Apply `mv` to the routes of `o` and build the records of the result (the
// per-position and per-gap records of prep, without chunk ranks, plus the row
// indices of each position's own exit and its predecessor's) into `n`; with
// write_routes the routes after the move are written to `n` as well.  Every
// value comes from `o` and the instance, so the workgroups of a solve need no
// barrier between applying the move and building the records.
template <typename TE>
__device__ void prep_next(const Ctx &o, const Ctx &n, const GMove &mv, const TE *tc, bool write_routes,
                          int tid, int nthr)
{
    const uint32_t Cs = (uint32_t)o.Cs;
    const int M = o.M, V = o.V;
    for (int i = tid; i < M; i += nthr) {
        const int m = next_seq(o, mv, i), r = next_rt(o, mv, i);
        const int sp = i > 0 ? next_seq(o, mv, i - 1) : 0;
        const int sn = i + 1 < M ? next_seq(o, mv, i + 1) : 0;
        const int sn2 = i + 2 < M ? next_seq(o, mv, i + 2) : 0;
        const int o0 = next_off(o, mv, r), o1 = next_off(o, mv, r + 1);
        const bool first = i == o0, last = i + 1 == o1;
        const int x = first ? gld(o.vrow)[r] : gld(o.mrow)[sp];
        const int y = last ? gld(o.vcol)[r] : gld(o.mcol)[sn];
        const int mc = gld(o.mcol)[m], mr = gld(o.mrow)[m];
        const int a = gld(tc)[x + mc], bb = gld(tc)[mr + y], l = gld(tc)[x + y];
        int adj = 0;
        if (!last) {
            // swapping m with its successor in the same route: P m n N -> P n m N
            const int y2 = (i + 2 == o1) ? gld(o.vcol)[r] : gld(o.mcol)[sn2];
            const int mrn = gld(o.mrow)[sn];
            adj = l + (int)gld(tc)[mrn + mc] + (int)gld(tc)[mr + y2] - a - bb - (int)gld(tc)[mrn + y2];
        }
        // every field of a record the sweeps read is used (an unused component's
        // register would be reused while its load is in flight, serialising the loads)
        gst4(n.posA, i, make_int4(mc, y, a + bb, (int)((uint32_t)m | ((uint32_t)r << 16))));
        gst4(n.posB, i, make_int4(l - a - bb, adj, 0, 0));
        gst4(n.gap, i + r, make_int4((int)((uint32_t)x / Cs), mc, a, r));
        gst2(n.posC, i, make_int2((int)((uint32_t)mr / Cs), (int)((uint32_t)x / Cs)));
        if (write_routes) {
            gst(n.seq)[i] = (uint16_t)m;
            gst(n.rt)[i] = (uint16_t)r;
            gst(n.pof)[m] = (uint16_t)i;
            gst(n.rof)[m] = (uint16_t)r;
        }
    }
    for (int r = tid; r <= V; r += nthr) {
        const int o0 = next_off(o, mv, r);
        if (write_routes) gst(n.off)[r] = o0;
        if (r == V) continue;
        // the gap after the route's last mission
        const int e = next_off(o, mv, r + 1);
        const int x = (o0 == e) ? gld(o.vrow)[r] : gld(o.mrow)[next_seq(o, mv, e - 1)];
        gst4(n.gap, e + r, make_int4((int)((uint32_t)x / Cs), gld(o.vcol)[r], (int)gld(tc)[x + gld(o.vcol)[r]], r));
    }
}

// Eval of the global schedule: blocks of K (at most kGlobalKMax) consecutive
// route positions, dealt to the solve's workgroups in rounds, every other round
// in reverse order (one block per workgroup where LDS allows).  For each block the four travel vectors its
// missions' moves read -- the block column of the pickup and of the successor
// (rows of the transposed block), the block row of the delivery and of the
// predecessor (rows of the aligned copy) -- the missions' tabu columns and the
// tabu rows of the block's vehicles (one bit per mission: active or not) are
// staged in LDS with 16-byte loads, each thread's loads issued before its
// first store.  The sweeps map threads two-dimensionally: Q threads (a power
// of two, at least a wavefront) walk the columns -- gap records for
// relocates, later positions for swaps, several in flight -- and nthr / Q
// thread groups split the block's missions.  Inside one (mission, round) the
// keys are 32-bit -- blocked bit, delta + 2^25, then the column's rank -- and
// their minimum joins the 64-bit key of the lane.  Rounds that hold a no-op
// column, the mission's own neighbours or the tail take a checked path; all
// others skip the checks.
template <typename TE, typename TB>
__device__ uint64_t eval_staged(const Ctx &c, const InstDev &I, const TE *tc, const TE *tct,
                                const TE *tcr, const int4 *ring, int ring_len, char *smem, uint64_t *red,
                                int K, int wg, int nwg, int t, int thr, bool use_tabu)
{
    constexpr int UR = 8, US = 4;              // relocate and swap loads in flight
    constexpr int ES = (int)sizeof(TE);
    (void)tc;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & (kWave - 1), wave = wave_id(tid), nwaves = nthr / kWave;
    const int M = c.M, V = c.V, NG = c.NG, Rs = I.Rs, Cg = I.Cg;
    const int Re = staged_rows(uniform(I.R), ES), Ce = staged_cols(uniform(I.C), ES);
    const int R16 = Re * ES / 16, C16 = Ce * ES / 16;   // 16-byte chunks of a staged column / row
    const int per = 2 * Re + 2 * Ce;
    const int Wm = (M + 31) >> 5;
    uint64_t *tab = (uint64_t *)smem;             // source pointers, 4 per mission
    int4 *mi = (int4 *)(tab + 4 * K);             // {m | r << 16, rem, own gap, out}
    int4 *mi2 = mi + K;                           // {adjacent-swap delta, vehicle slot, -, -}
    int *rl = (int *)(mi2 + K);                   // the block's vehicles; their count at rl[K],
                                                  // at rl[K + 1] whether any tabu entry is active for them
    TE *vec = (TE *)(smem + global_table_bytes(K));
    TB *trow = (TB *)((char *)vec + (((size_t)K * per * sizeof(TE) + 15) & ~(size_t)15));
    uint32_t *rbits = (uint32_t *)((char *)trow + (((size_t)K * V * sizeof(TB) + 15) & ~(size_t)15));
    const int th = use_tabu ? t : INT32_MAX;
    const int nblk = (M + K - 1) / K;
    // relocate sweep shape: QR column threads, PR mission groups
    int QR = kWave;
    while (QR < nthr && QR * UR < NG) QR <<= 1;
    const int PR = nthr / QR, pr = tid / QR, qr = tid - pr * QR;
    // the ring's active entries ({vehicle, mission, expiry}), gathered by the first
    // block's setup into the reduction area (free until the sweeps are done) for all
    // the workgroup's blocks: at most kActMax of them and a ring of at most one entry
    // per thread, else each block scans the ring itself (nact < 0)
    constexpr int kActMax = 120;
    int4 *act = (int4 *)(red + 16);
    uint32_t *nact_p = (uint32_t *)(red + 8);
    const bool listed = use_tabu && ring_len <= nthr;
    int nact = -1;
    uint64_t best = kKeyNone;
    // blocks dealt in rounds of nwg, every other round in reverse: a block's swap work
    // shrinks with its position, so plain round-robin dealing would give the first
    // workgroups the most work in every round
    for (int rd = 0; rd * nwg < nblk; ++rd) {
        const int blk = rd * nwg + ((rd & 1) ? nwg - 1 - wg : wg);
        if (blk >= nblk) continue;   // uniform over the workgroup
        const int i0 = blk * K;
        const int kn = min(K, M - i0);
        __syncthreads();   // the previous block's LDS reads are done
        // the block's tabu state (filled from the ring once its vehicles are known):
        // cleared here; each thread takes one ring entry along with the records
        for (int e = tid; e < kn * Wm; e += nthr) rbits[e] = 0u;
        if (tid == 0) rl[K + 1] = 0;
        if (use_tabu)
            for (int e = tid; e < kn * V; e += nthr) trow[e] = (TB)0;
        const bool first = rd == 0;
        if (listed && first && tid == 0) *nact_p = 0;
        const int4 ren = (use_tabu && (first || nact < 0) && tid < ring_len) ? gld4(ring, tid) : make_int4(0, 0, 0, 0);
        for (int q = tid; q < 5 * kn; q += nthr) {
            if (q < kn) {
                const int4 pa = gld4(c.posA, i0 + q);     // {pickup col, successor col, out, m | r << 16}
                const int4 pb = gld4(c.posB, i0 + q);     // {rem, adjacent-swap delta, -, -}
                const int r = (int)((uint32_t)pa.w >> 16);
                mi[q] = make_int4(pa.w, pb.x, i0 + q + r, pa.z);
                mi2[q] = make_int4(pb.y, 0, 0, 0);
            } else {
                // the successor column (Y) and predecessor row (X) of a mission whose
                // neighbour in the route is also in the block are that neighbour's
                // pickup column / delivery row: not loaded again
                const int e = q - kn, k = e >> 2, ty = e & 3;
                const int4 pa = gld4(c.posA, i0 + k);
                const int2 rc = gld2(c.posC, i0 + k);
                const uint32_t rk = (uint32_t)pa.w >> 16;
                const bool same_next = k + 1 < kn && ((uint32_t)gld4(c.posA, i0 + k + 1).w >> 16) == rk;
                const bool same_prev = k > 0 && ((uint32_t)gld4(c.posA, i0 + k - 1).w >> 16) == rk;
                const TE *src = ty == 0 ? tct + (size_t)pa.x * Rs
                              : ty == 1 ? (same_next ? nullptr : tct + (size_t)pa.y * Rs)
                              : ty == 2 ? tcr + (size_t)rc.x * Cg
                                        : (same_prev ? nullptr : tcr + (size_t)rc.y * Cg);
                tab[e] = (uint64_t)(uintptr_t)src;
            }
        }
        __syncthreads();
        if (listed && first && tid < ring_len && ren.z > t) {
            const uint32_t at = atomicAdd(nact_p, 1u);
            if (at < (uint32_t)kActMax) act[at] = ren;
        }
        if (tid < kWave) {
            // the block's missions (at most kGlobalKMax <= 64) on wavefront 0: the block's
            // vehicles in order (positions are route-ordered) and each mission's vehicle
            // slot, the number of vehicle changes up to it (a ballot and a popcount)
            const int q = tid;
            const bool in = q < kn;
            const int r = in ? (int)((uint32_t)mi[q].x >> 16) : -1;
            const bool same_prev = in && q > 0 && ((uint32_t)mi[q - 1].x >> 16) == (uint32_t)r;
            const bool same_next = in && q + 1 < kn && ((uint32_t)mi[q + 1].x >> 16) == (uint32_t)r;
            const uint64_t change = __ballot(in && q > 0 && !same_prev);
            const uint64_t upto = q >= kWave - 1 ? ~0ull : ((1ull << (q + 1)) - 1);
            const int slot = (int)__popcll(change & upto);
            if (in) {
                mi2[q].y = slot;
                if (!same_prev) rl[slot] = r;
                if (q == kn - 1) rl[K] = slot + 1;
                // where the mission's predecessor row and successor column sit in LDS
                mi2[q].z = same_prev ? (q - 1) * per + 2 * Re : q * per + 2 * Re + Ce;
                mi2[q].w = same_next ? (q + 1) * per : q * per + Re;
            }
        }
        __syncthreads();
        const int nd = rl[K];
        if (listed && first) {
            nact = (int)*nact_p;
            if (nact > kActMax) nact = -1;
        }
        // the travel vectors of the block's missions: 16-byte chunk j of the staged
        // area belongs to mission k = j / P16, whose four vectors (pickup and successor
        // columns, delivery and predecessor rows) follow one another.  Each wavefront
        // loads 64 consecutive chunks straight into LDS (lane l to chunk j0 + l), so a
        // thread's loads are all in flight at once and need no registers; a null
        // source (the vector comes from an in-block neighbour) is skipped.  Quotients
        // by multiply-high where exact (dividend x divisor < 2^32, divisor > 1), else
        // by division.
        {
            const int P16 = 2 * R16 + 2 * C16, nch = kn * P16;
            const uint32_t mP = 0xFFFFFFFFu / (uint32_t)P16 + 1u;
            const bool fast = P16 > 1 && (uint64_t)nch * (uint64_t)P16 < (1ull << 32);
            char *lds = (char *)vec;
            for (int j0 = wave * kWave; j0 < nch; j0 += nwaves * kWave) {
                const int j = j0 + lane;
                const int k = fast ? (int)__umulhi((uint32_t)j, mP) : j / P16;
                const int o = j - k * P16;
                const int ty = o < R16 ? 0 : o < 2 * R16 ? 1 : o < 2 * R16 + C16 ? 2 : 3;
                const int oo = o - (ty == 0 ? 0 : ty == 1 ? R16 : ty == 2 ? 2 * R16 : 2 * R16 + C16);
                const uint64_t sa = j < nch ? tab[4 * k + ty] : 0;
                if (sa != 0)
                    __builtin_amdgcn_global_load_lds(
                        (const __attribute__((address_space(1))) void *)(uintptr_t)(sa + 16 * (uint64_t)oo),
                        (__attribute__((address_space(3))) void *)(lds + 16 * (size_t)j0), 16, 0, 0);
            }
        }
        // active ring entries: the vehicle column of a block mission (relocates of the
        // mission, swaps of it into a partner's vehicle) and the mission's bit in the
        // row of a block vehicle (swaps of a partner into that vehicle)
        if (use_tabu && nact >= 0) {
            // (entry, block mission) pairs over all threads, then (entry, block vehicle)
            bool hit = false;
            for (int p = tid; p < nact * kn; p += nthr) {
                const int e = p / kn, k = p - e * kn;
                const int4 en = act[e];
                if ((mi[k].x & 0xFFFF) == en.y) { trow[k * V + en.x] = (TB)en.z; hit = true; }
            }
            for (int p = tid; p < nact * nd; p += nthr) {
                const int e = p / nd, q = p - e * nd;
                const int4 en = act[e];
                if (rl[q] == en.x) { atomicOr(&rbits[q * Wm + (en.y >> 5)], 1u << (en.y & 31)); hit = true; }
            }
            if (hit) rl[K + 1] = 1;
        } else if (use_tabu) {
            for (int e0 = 0; e0 < ring_len; e0 += nthr) {
                const int e = e0 + tid;
                const int4 en = e0 == 0 ? ren : (e < ring_len ? gld4(ring, e) : make_int4(0, 0, 0, 0));
                if (e < ring_len && en.z > t) {
                    const int r = en.x, m = en.y;
                    bool hit = false;
                    for (int k = 0; k < kn; ++k)
                        if ((mi[k].x & 0xFFFF) == m) { trow[k * V + r] = (TB)en.z; hit = true; }
                    for (int q = 0; q < nd; ++q)
                        if (rl[q] == r) { atomicOr(&rbits[q * Wm + (m >> 5)], 1u << (m & 31)); hit = true; }
                    if (hit) rl[K + 1] = 1;
                }
            }
        }
        // the staged vectors have arrived in LDS
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        // the sweeps, with the tabu lookups only where an active entry concerns the
        // block (otherwise no move of the block is tabu)
        auto sweeps = [&](auto tab_on) {
            constexpr bool TAB = decltype(tab_on)::value;
            // relocates: every gap against the block's missions
            for (int b0 = qr; b0 < NG; b0 += UR * QR) {
                const int rb = b0 - qr;                       // first column of the round
                const bool tail = rb + UR * QR > NG;
                int4 g[UR];
#pragma unroll
                for (int u = 0; u < UR; ++u) {
                    const int G = b0 + u * QR;
                    g[u] = gld4(c.gap, G < NG ? G : 0);
                }
                for (int k = pr; k < kn; k += PR) {
                    const int4 q = mi[k];
                    const TE *v = vec + k * per;
                    const TB *tr = trow + k * V;
                    uint32_t mn = 0xFFFFFFFFu;
                    if (!tail && (q.z + 1 < rb || q.z >= rb + UR * QR)) {
#pragma unroll
                        for (int u = 0; u < UR; ++u) {
                            const int gr = g[u].w, grow = g[u].x;
                            const int d = q.y + (int)v[grow] + (int)v[2 * Re + g[u].y] - g[u].z;
                            const bool blk = (TAB && (int)tr[gr] > th) & !(d < thr);
                            const uint32_t key = (blk ? 0x80000000u : 0u) | ((uint32_t)(d + kPackBias) << 5) | (uint32_t)u;
                            mn = min(mn, key);
                        }
                    } else {
#pragma unroll
                        for (int u = 0; u < UR; ++u) {
                            const int G = b0 + u * QR;
                            const int gr = g[u].w, grow = g[u].x;
                            const int d = q.y + (int)v[grow] + (int)v[2 * Re + g[u].y] - g[u].z;
                            const bool blk = (TAB && (int)tr[gr] > th) & !(d < thr);
                            const uint32_t key = (blk ? 0x80000000u : 0u) | ((uint32_t)(d + kPackBias) << 5) | (uint32_t)u;
                            const bool skip = (G >= NG) | ((unsigned)(G - q.z) < 2u);
                            mn = skip ? mn : min(mn, key);
                        }
                    }
                    if (mn != 0xFFFFFFFFu) {
                        const int G = b0 + (int)(mn & 31u) * QR;
                        const int d = (int)((mn >> 5) & 0x3FFFFFFu) - kPackBias;
                        best = umin64(best, pack_key((mn >> 31) != 0, d,
                                                     (uint32_t)(q.x & 0xFFFF) * (uint32_t)NG + (uint32_t)G));
                    }
                }
            }
            // swaps: every later position against the block's missions
            const int j0 = i0 + 1;
            int QS = kWave;
            while (QS < nthr && QS * US < M - j0) QS <<= 1;
            const int PS = nthr / QS, ps = tid / QS, qs = tid - ps * QS;
            for (int b0 = j0 + qs; b0 < M; b0 += US * QS) {
                const int rb = b0 - qs;
                const bool tail = rb + US * QS > M;
                int4 a[US];          // {pickup column, successor column, out, m | r << 16}
                int2 rc[US];         // {delivery row, predecessor row}
                int mj[US], rk[US];
#pragma unroll
                for (int u = 0; u < US; ++u) {
                    const int j = b0 + u * QS < M ? b0 + u * QS : j0;
                    a[u] = gld4(c.posA, j);
                    rc[u] = gld2(c.posC, j);
                }
                // rank of each partner's mission among the lane's partners of the round
                // (swap indices of one mission grow with the partner's mission)
#pragma unroll
                for (int u = 0; u < US; ++u)
                    mj[u] = b0 + u * QS < M ? (a[u].w & 0xFFFF) : 0x10000 + u;
#pragma unroll
                for (int u = 0; u < US; ++u) {
                    int r = 0;
#pragma unroll
                    for (int w = 0; w < US; ++w) r += (w != u && mj[w] < mj[u]) ? 1 : 0;
                    rk[u] = r;
                }
                for (int k = ps; k < kn; k += PS) {
                    const int4 q = mi[k];
                    const int4 q2 = mi2[k];
                    const int mk = q.x & 0xFFFF, rkk = (int)((uint32_t)q.x >> 16);
                    const int jk = i0 + k;
                    const TE *v = vec + k * per;
                    const TE *vx = vec + q2.z, *vy = vec + q2.w;
                    const TB *tr = trow + k * V;
                    const uint32_t *rbit = rbits + q2.y * Wm;
                    uint32_t mn = 0xFFFFFFFFu;
                    if (!tail && rb > jk + 1) {
#pragma unroll
                        for (int u = 0; u < US; ++u) {
                            const int rj = (int)((uint32_t)a[u].w >> 16);
                            const int d = (int)vx[a[u].x] + (int)vy[rc[u].x] + (int)v[rc[u].y]
                                        + (int)v[2 * Re + a[u].y] - q.w - a[u].z;
                            const bool tb = TAB && (((int)tr[rj] > th) | (((rbit[mj[u] >> 5] >> (mj[u] & 31)) & 1u) != 0));
                            const uint32_t key = ((tb & !(d < thr)) ? 0x80000000u : 0u)
                                               | ((uint32_t)(d + kPackBias) << 5) | (uint32_t)rk[u];
                            mn = min(mn, key);
                        }
                    } else {
#pragma unroll
                        for (int u = 0; u < US; ++u) {
                            const int j = b0 + u * QS;
                            const int rj = (int)((uint32_t)a[u].w >> 16);
                            const int m2 = mj[u] & 0xFFFF;
                            const int dg = (int)vx[a[u].x] + (int)vy[rc[u].x] + (int)v[rc[u].y]
                                         + (int)v[2 * Re + a[u].y] - q.w - a[u].z;
                            const int d = (j == jk + 1 && rkk == rj) ? q2.x : dg;
                            const bool tb = TAB && (((int)tr[rj] > th) | (((rbit[m2 >> 5] >> (m2 & 31)) & 1u) != 0));
                            const uint32_t key = ((tb & !(d < thr)) ? 0x80000000u : 0u)
                                               | ((uint32_t)(d + kPackBias) << 5) | (uint32_t)rk[u];
                            mn = ((j >= M) | (j <= jk)) ? mn : min(mn, key);
                        }
                    }
                    if (mn != 0xFFFFFFFFu) {
                        const int r = (int)(mn & 31u);
                        int mw = mj[0];
#pragma unroll
                        for (int u = 1; u < US; ++u) mw = rk[u] == r ? mj[u] : mw;
                        const int d = (int)((mn >> 5) & 0x3FFFFFFu) - kPackBias;
                        const uint32_t lo = (uint32_t)min(mk, mw), hi = (uint32_t)max(mk, mw);
                        best = umin64(best, pack_key((mn >> 31) != 0, d, swap_index(c.R, (uint32_t)M, lo, hi)));
                    }
                }
            }
        };
        if (rl[K + 1]) sweeps(std::true_type{});
        else sweeps(std::false_type{});
    }
    return best;
}

// Whether the ring holds an active entry for (vehicle r1, mission m1) or for
// (r2, m2) at iteration t: one wavefront, one entry per lane.
__device__ __forceinline__ bool ring_tabu(const int4 *ring, int n, int r1, int m1, int r2, int m2, int t,
                                          int lane)
{
    bool hit = false;
    for (int e = lane; e < n; e += kWave) {
        const int4 x = gld4(ring, e);
        hit |= x.z > t && ((x.x == r1 && x.y == m1) || (x.x == r2 && x.y == m2));
    }
    return __any(hit);
}

template <typename TE, typename TB>
__device__ __forceinline__ void run_job_global(const JobDev &J, int wg, int nwg, char *smem, uint64_t *red)
{
    const InstDev &I = *J.inst;
    GlobalBufs &B = *J.gb;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & (kWave - 1), wave = wave_id(tid), nwaves = nthr / kWave;
    const int gtid = wg * nthr + tid, gthr = nwg * nthr;
    const int M = uniform(I.M), V = uniform(I.V);
    const TE *tc = (const TE *)I.tc;
    int4 *ring = B.ring;
    const int ring_n = uniform(B.ring_slots), ring_len = 2 * ring_n;
    const bool writer = wg == 0;
    SolveState *st = J.st;
    uint32_t nb = 0;
    uint64_t kx;

    int p, best_iter, stopped;
    int64_t cur, best;
    bool aborted = false, pending = false;
    if (J.resume && st && st->valid) {
        p = B.cur;
        cur = st->cur;
        best = st->best;
        best_iter = st->best_iter;
        stopped = st->stopped;
    } else {
        p = 0;
        if (wg == 0) {
            const Ctx c0 = global_ctx(I, B, 0, red);
            const uint32_t lds = global_lds_bytes(J.gk, I.R, I.C, I.M, I.V, (int)sizeof(TE), (int)sizeof(TB));
            const int64_t g = greedy_staged_bytes(M, V, J.seed != 0) + 2048u <= lds
                                  ? greedy_staged<TE>(c0, tc, J.seed, I.svc_sum, smem, tid, nthr)
                                  : greedy<TE>(c0, tc, J.seed, I.svc_sum, tid, nthr);
            if (tid == 0) __hip_atomic_store(&B.init_obj, g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            snapshot(c0, J, tid, nthr);
        }
        for (int k = gtid; k < ring_len; k += gthr) gst4(ring, k, make_int4(0, 0, 0, 0));
        if (!group_exchange(B, wg, nwg, nb, kKeyNone, red, kx)) aborted = true;
        cur = __hip_atomic_load(&B.init_obj, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        best = cur;
        best_iter = -1;
        stopped = 0;
    }
    if (!aborted) {
        // records of the current routes
        GMove none{};
        const Ctx c = global_ctx(I, B, p, red);
        prep_next<TE>(c, c, none, tc, false, gtid, gthr);
        if (!group_exchange(B, wg, nwg, nb, kKeyNone, red, kx)) aborted = true;
    }

    const bool use_tabu = J.variant == AT_TABU;
    int t = J.t_begin;
    for (; !aborted && t < J.t_end && !stopped; ++t) {
        const Ctx c = global_ctx(I, B, p, red);
        if (pending && writer) snapshot(c, J, tid, nthr);
        pending = false;
        int thr = INT32_MIN;
        if (J.aspiration) {
            const int64_t g = best - cur;
            thr = g < (int64_t)INT32_MIN ? INT32_MIN : (int)g;
        }
        uint64_t k = eval_staged<TE, TB>(c, I, tc, (const TE *)I.tct, (const TE *)I.tcr, ring, ring_len, smem,
                                         red, J.gk, wg, nwg, t, thr, use_tabu);
        k = wave_min(k);
        if (lane == 0) red[wave] = k;
        __syncthreads();
        uint64_t wk = kKeyNone;
        if (tid < kWave) wk = wave_min(lane < nwaves ? red[lane] : kKeyNone);
        uint64_t key;
        if (!group_exchange(B, wg, nwg, nb, wk, red, key)) { aborted = true; break; }
        if (key == kKeyNone) {
            if (!use_tabu) { stopped = 1; break; }
            // nothing to apply: routes and records stay as they are
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
        const bool is_swap = idx >= c.R;
        GMove mv{};
        bool was_tabu = false;
        if (!is_swap) {
            const int m = (int)(idx / (uint32_t)c.NG);
            const int G = (int)(idx - (uint32_t)m * (uint32_t)c.NG);
            // the gap's vehicle and the mission's position and vehicle: three
            // independent loads (the insertion point off[v] + g is G - v)
            const int v = c.gap[G].w & 0xFFFF;
            const int s = c.pof[m];
            const int rs = c.rof[m];
            const int fp = G - v;
            const int q = fp - (fp > s ? 1 : 0);
            mv.kind = 1;
            mv.m = m; mv.v = v; mv.q = q; mv.rs = rs;
            mv.lo = min(s, q); mv.hi = max(s, q); mv.dir = q >= s ? 1 : -1;
            if (writer && tid < kWave && use_tabu) {
                if (J.trace) was_tabu = ring_tabu(ring, ring_len, v, m, -1, -1, t, lane);
                if (tid == 0) {
                    gst4(ring, 2 * (t % ring_n), make_int4(rs, m, tval, 0));
                    gst4(ring, 2 * (t % ring_n) + 1, make_int4(0, 0, 0, 0));
                }
            }
        } else {
            int m1, m2;
            swap_pair(idx - c.R, M, m1, m2);
            const int s1 = c.pof[m1], s2 = c.pof[m2];
            mv.kind = 2;
            mv.s1 = s1; mv.s2 = s2; mv.m1 = m1; mv.m2 = m2;
            if (writer && tid < kWave && use_tabu) {
                const int r1 = c.rof[m1], r2 = c.rof[m2];
                if (J.trace) was_tabu = ring_tabu(ring, ring_len, r2, m1, r1, m2, t, lane);
                if (tid == 0) {
                    gst4(ring, 2 * (t % ring_n), make_int4(r1, m1, tval, 0));
                    gst4(ring, 2 * (t % ring_n) + 1, make_int4(r2, m2, tval, 0));
                }
            }
        }
        prep_next<TE>(c, global_ctx(I, B, p ^ 1, red), mv, tc, true, gtid, gthr);
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
            pending = true;
        }
        if (!group_exchange(B, wg, nwg, nb, kKeyNone, red, kx)) { aborted = true; break; }
        p ^= 1;
    }
    if (!writer) return;
    if (pending && !aborted) snapshot(global_ctx(I, B, p, red), J, tid, nthr);
    if (J.fin_off && !aborted) write_routes(global_ctx(I, B, p, red), J.fin_off, J.fin_seq, nullptr, tid, nthr);
    if (tid == 0) {
        J.scal->best_obj = best;
        J.scal->final_obj = cur;
        J.scal->iters_done = t;
        J.scal->best_iter = best_iter;
        J.scal->stopped = stopped;
        J.scal->status = aborted ? AT_EDEVICE : AT_OK;
        B.cur = p;
        if (J.save && st) {
            st->cur = cur;
            st->best = best;
            st->t = t;
            st->best_iter = best_iter;
            st->stopped = stopped;
            st->valid = 1;
        }
    }
}

// Solves on the global schedule, each on its range [g0, g0 + ng) of the grid.
// At most kGlobalBlock threads per workgroup: the register budget that leaves
// (256 VGPRs) keeps the per-iteration state out of scratch memory.
template <typename TE, typename TB>
__device__ __forceinline__ void global_group(const JobDev *jobs, int n_jobs, int b, char *smem)
{
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].g0 <= b) lo = mid; else hi = mid - 1;
    }
    const JobDev &J = jobs[lo];
    const InstDev &I = *J.inst;
    const uint32_t lds = global_lds_bytes(J.gk, I.R, I.C, I.M, I.V, (int)sizeof(TE), (int)sizeof(TB));
    uint64_t *red = (uint64_t *)(smem + lds - 2048);
    run_job_global<TE, TB>(J, b - J.g0, J.ng, smem, red);
}

template <typename TE, typename TB>
__global__ void __launch_bounds__(kGlobalBlock) k_search_global(const JobDev *jobs, int n_jobs)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    global_group<TE, TB>(jobs, n_jobs, (int)blockIdx.x, smem);
}

// One-workgroup jobs and HBM-resident jobs of one launch in one grid:
// workgroups [0, n_ggroups) run the global jobs of `gjobs` as k_search_global
// does, the others (workers) take jobs of `wjobs` from the queue: one-workgroup
// jobs as k_search_wg does (with this kernel's block size), and global jobs on
// one workgroup.  The two kinds share the device inside one cooperative launch,
// so every workgroup is resident and nothing waits for another stream, and a
// worker that finishes a solve takes the next instead of idling until the
// launch ends.  A worker passes the job index through the first word of its
// LDS between two barriers, before the job's own use of it.
template <typename TE, typename TB>
__global__ void __launch_bounds__(kGlobalBlock) k_search_mixed(const JobDev *gjobs, int n_gjobs, int n_ggroups,
                                                              const JobDev *wjobs, int n_wjobs, uint32_t *queue)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    if ((int)blockIdx.x < n_ggroups) {
        global_group<TE, TB>(gjobs, n_gjobs, (int)blockIdx.x, smem);
        return;
    }
    int *s_job = (int *)smem;
    for (;;) {
        if (threadIdx.x == 0)
            *s_job = (int)__hip_atomic_fetch_add(queue, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int j = __builtin_amdgcn_readfirstlane(*s_job);   // scalar: the job's fields load as scalars
        __syncthreads();
        if (j >= n_wjobs) return;
        const JobDev &J = wjobs[j];
        if (J.sched == AT_SCHED_GLOBAL) {
            const InstDev &I = *J.inst;
            const uint32_t lds = global_lds_bytes(J.gk, I.R, I.C, I.M, I.V, (int)sizeof(TE), (int)sizeof(TB));
            run_job_global<TE, TB>(J, 0, 1, smem, (uint64_t *)(smem + lds - 2048));
        } else {
            run_job<TE, TB, false>(J, smem, 0, 1, nullptr);
        }
        __syncthreads();
    }
}

// Reset the exchange state of every solve of a global-schedule launch (one
// workgroup per solve): every slot gets tag 1, which no first use of a buffer
// carries, and the abort flag is cleared.
__global__ void k_reset_global(const JobDev *jobs, int n_jobs)
{
    if (jobs[blockIdx.x].sched != AT_SCHED_GLOBAL) return;   // a one-workgroup job of a mixed launch
    GlobalBufs &B = *jobs[blockIdx.x].gb;
    for (int w = (int)threadIdx.x; w < 2 * kMaxGroups; w += (int)blockDim.x) B.slots[w * kSlotStride] = ~0ull;
    if (threadIdx.x == 0) B.abort = 0;
}

// One workgroup per job; jobs are taken from an atomic queue until exhausted.
template <typename TE, typename TB>
__global__ void __launch_bounds__(1024) k_search_wg(const JobDev *jobs, int n_jobs, uint32_t *queue)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __shared__ int s_job;
    for (;;) {
        if (threadIdx.x == 0)
            s_job = (int)__hip_atomic_fetch_add(queue, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int j = __builtin_amdgcn_readfirstlane(s_job);   // scalar: the job's fields load as scalars
        __syncthreads();
        if (j >= n_jobs) return;
        run_job<TE, TB, false>(jobs[j], smem, 0, 1, nullptr);
        __syncthreads();
    }
}

// One wavefront per job: each wavefront takes jobs from the atomic queue and
// runs them in its own LDS region (lds_per_solve bytes at its index in the
// workgroup) with the one-workgroup schedule's code, its barriers wavefront-
// wide.
template <typename TE, typename TB>
__global__ void __launch_bounds__(256) k_search_wg_wave(const JobDev *jobs, int n_jobs, uint32_t *queue,
                                                       uint32_t lds_per_solve)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = threadIdx.x & (kWave - 1), wave = wave_id((int)threadIdx.x);
    char *base = smem + (size_t)wave * lds_per_solve;
    for (;;) {
        int j = 0;
        if (lane == 0) j = (int)__hip_atomic_fetch_add(queue, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        j = __builtin_amdgcn_readfirstlane(j);   // lane 0's, as a scalar
        if (j >= n_jobs) return;
        run_job<TE, TB, false, true>(jobs[j], base, 0, 1, nullptr);
    }
}

template <typename TE, typename TB>
__global__ void __launch_bounds__(1024) k_search_multi(const JobDev *jobs, int n_jobs, Xchg *xs)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    // the solve whose workgroup range holds this workgroup
    const int b = (int)blockIdx.x;
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].g0 <= b) lo = mid; else hi = mid - 1;
    }
    const JobDev &J = jobs[lo];
    run_job<TE, TB, true>(J, smem, b - J.g0, J.ng, xs);
}

// Test hook: every slot's key for a given state (keys[0..n_slots)), and the
// minimum the search's own eval finds for that state (keys[n_slots]).
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
    const int lane = tid & (kWave - 1), wave = wave_id(tid), nwaves = nthr / kWave;
    const int M = uniform(I.M), V = uniform(I.V), R = uniform(I.R), Cs = uniform(I.Cs);
    const Lay ly = lds_layout(M, V, R, Cs, (int)sizeof(TE), 4);
    const Ctx c = make_ctx(smem, ly, M, V, J.chunk, J.rchunk, Cs);
    TE *tc = (TE *)(smem + ly.tc);
    int32_t *tabu = (int32_t *)(smem + ly.tabu);
    load_instance<TE>(I, c, tc, tid, nthr);
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
    const bool use_tabu = J.variant == AT_TABU;
    dump_keys<TE>(c, tc, tabu, tid, nthr, t, thr, use_tabu, keys);
    uint64_t k = eval_all<TE, int32_t>(c, tc, tabu, wave, nwaves, unit_start(c, wave), lane, t, thr, use_tabu);
    k = wave_min(k);
    if (lane == 0) c.red[wave] = k;
    __syncthreads();
    if (tid < kWave) {
        uint64_t w = lane < nwaves ? c.red[lane] : kKeyNone;
        w = wave_min(w);
        if (w != kKeyNone) w = (w & 0xFFFFFFFF00000000ull) | lidx_slot((uint32_t)w, c.R, (uint32_t)M, (uint32_t)c.NG);
        if (lane == 0) keys[n_slots(M, V)] = w;
    }
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

hipError_t launch_search_wg(const JobDev *jobs, int32_t n_jobs, uint32_t *queue, int grid, int block,
                            uint32_t lds_bytes, int tb16, int esz16, hipStream_t s)
{
    hipError_t e;
#define AT_WG(TE, TB)                                                                      \
    do {                                                                                   \
        if ((e = set_lds(k_search_wg<TE, TB>, lds_bytes)) != hipSuccess) return e;         \
        hipLaunchKernelGGL((k_search_wg<TE, TB>), dim3(grid), dim3(block), lds_bytes, s,   \
                           jobs, n_jobs, queue);                                           \
    } while (0)
    if (esz16 && tb16) AT_WG(uint16_t, uint16_t);
    else if (esz16) AT_WG(uint16_t, int32_t);
    else if (tb16) AT_WG(int32_t, uint16_t);
    else AT_WG(int32_t, int32_t);
#undef AT_WG
    return hipGetLastError();
}

hipError_t launch_search_wg_wave(const JobDev *jobs, int32_t n_jobs, uint32_t *queue, int grid,
                                 int waves_per_group, uint32_t lds_per_solve, int tb16, int esz16,
                                 hipStream_t s)
{
    hipError_t e;
    const uint32_t lds = lds_per_solve * (uint32_t)waves_per_group;
#define AT_WW(TE, TB)                                                                          \
    do {                                                                                       \
        if ((e = set_lds(k_search_wg_wave<TE, TB>, lds)) != hipSuccess) return e;              \
        hipLaunchKernelGGL((k_search_wg_wave<TE, TB>), dim3(grid), dim3(kWave * waves_per_group), lds, \
                           s, jobs, n_jobs, queue, lds_per_solve);                             \
    } while (0)
    if (esz16 && tb16) AT_WW(uint16_t, uint16_t);
    else if (esz16) AT_WW(uint16_t, int32_t);
    else if (tb16) AT_WW(int32_t, uint16_t);
    else AT_WW(int32_t, int32_t);
#undef AT_WW
    return hipGetLastError();
}

template <typename TE, typename TB>
static hipError_t coop_launch(const JobDev *jobs, int n_jobs, Xchg *xs, int n_groups, int block,
                              uint32_t lds_bytes, hipStream_t s)
{
    hipError_t e = set_lds(k_search_multi<TE, TB>, lds_bytes);
    if (e != hipSuccess) return e;
    void *args[] = {(void *)&jobs, (void *)&n_jobs, (void *)&xs};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_search_multi<TE, TB>),
                                      dim3(n_groups), dim3(block), args, lds_bytes, s);
}

hipError_t launch_search_multi(const JobDev *jobs, int n_jobs, Xchg *xs, int n_groups, int block,
                               uint32_t lds_bytes, int tb16, int esz16, hipStream_t s)
{
    if (esz16 && tb16) return coop_launch<uint16_t, uint16_t>(jobs, n_jobs, xs, n_groups, block, lds_bytes, s);
    if (esz16) return coop_launch<uint16_t, int32_t>(jobs, n_jobs, xs, n_groups, block, lds_bytes, s);
    if (tb16) return coop_launch<int32_t, uint16_t>(jobs, n_jobs, xs, n_groups, block, lds_bytes, s);
    return coop_launch<int32_t, int32_t>(jobs, n_jobs, xs, n_groups, block, lds_bytes, s);
}

template <typename TE, typename TB>
static hipError_t coop_launch_global(const JobDev *jobs, int n_jobs, int n_groups, int block,
                                     uint32_t lds_bytes, hipStream_t s)
{
    hipError_t e = set_lds(k_search_global<TE, TB>, lds_bytes);
    if (e != hipSuccess) return e;
    void *args[] = {(void *)&jobs, (void *)&n_jobs};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_search_global<TE, TB>),
                                      dim3(n_groups), dim3(block), args, lds_bytes, s);
}

hipError_t launch_search_global(const JobDev *jobs, int n_jobs, int n_groups, int block,
                                uint32_t lds_bytes, int tb16, int esz16, hipStream_t s)
{
    k_reset_global<<<dim3((unsigned)n_jobs), dim3(256), 0, s>>>(jobs, n_jobs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (esz16 && tb16) return coop_launch_global<uint16_t, uint16_t>(jobs, n_jobs, n_groups, block, lds_bytes, s);
    if (esz16) return coop_launch_global<uint16_t, int32_t>(jobs, n_jobs, n_groups, block, lds_bytes, s);
    if (tb16) return coop_launch_global<int32_t, uint16_t>(jobs, n_jobs, n_groups, block, lds_bytes, s);
    return coop_launch_global<int32_t, int32_t>(jobs, n_jobs, n_groups, block, lds_bytes, s);
}

template <typename TE, typename TB>
static hipError_t coop_launch_mixed(const JobDev *gjobs, int n_gjobs, int n_ggroups, const JobDev *wjobs,
                                    int n_wjobs, uint32_t *queue, int n_workers, uint32_t lds_bytes, hipStream_t s)
{
    hipError_t e = set_lds(k_search_mixed<TE, TB>, lds_bytes);
    if (e != hipSuccess) return e;
    void *args[] = {(void *)&gjobs, (void *)&n_gjobs, (void *)&n_ggroups, (void *)&wjobs, (void *)&n_wjobs,
                    (void *)&queue};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_search_mixed<TE, TB>),
                                      dim3(n_ggroups + n_workers), dim3(kGlobalBlock), args, lds_bytes, s);
}

hipError_t launch_search_mixed(const JobDev *gjobs, int n_gjobs, int n_ggroups, const JobDev *wjobs, int n_wjobs,
                               uint32_t *queue, int n_workers, uint32_t lds_bytes, int tb16, int esz16,
                               hipStream_t s)
{
    // the two lists are consecutive in the table (workers' jobs first)
    const JobDev *all = n_wjobs > 0 ? wjobs : gjobs;
    if (n_wjobs > 0 && n_gjobs > 0 && gjobs != wjobs + n_wjobs) return hipErrorInvalidValue;
    if (n_wjobs + n_gjobs > 0) k_reset_global<<<dim3((unsigned)(n_wjobs + n_gjobs)), dim3(256), 0, s>>>(all, n_wjobs + n_gjobs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
#define AT_MX(TE, TB) \
    return coop_launch_mixed<TE, TB>(gjobs, n_gjobs, n_ggroups, wjobs, n_wjobs, queue, n_workers, lds_bytes, s)
    if (esz16 && tb16) AT_MX(uint16_t, uint16_t);
    if (esz16) AT_MX(uint16_t, int32_t);
    if (tb16) AT_MX(int32_t, uint16_t);
    AT_MX(int32_t, int32_t);
#undef AT_MX
}

template <typename TE, typename TB>
static int occupancy_mixed(uint32_t lds_bytes)
{
    if (set_lds(k_search_mixed<TE, TB>, lds_bytes) != hipSuccess) return 0;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_search_mixed<TE, TB>, kGlobalBlock,
                                                     lds_bytes) != hipSuccess)
        return 0;
    return per_cu * num_cus();
}

int max_groups_mixed(uint32_t lds_bytes, int tb16, int esz16)
{
    if (esz16 && tb16) return occupancy_mixed<uint16_t, uint16_t>(lds_bytes);
    if (esz16) return occupancy_mixed<uint16_t, int32_t>(lds_bytes);
    if (tb16) return occupancy_mixed<int32_t, uint16_t>(lds_bytes);
    return occupancy_mixed<int32_t, int32_t>(lds_bytes);
}

// Workgroups of the global schedule one CU holds, per (entry width, tabu width,
// block size, LDS bytes), asked of the runtime once per device and key.
static std::mutex g_occ_mu;
static std::map<std::tuple<int, int, int, int, uint32_t>, int> g_occ;

template <typename TE, typename TB>
static int occupancy_global(int block, uint32_t lds_bytes)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    const auto key = std::make_tuple(dev, (int)sizeof(TE), (int)sizeof(TB), block, lds_bytes);
    {
        std::lock_guard<std::mutex> lk(g_occ_mu);
        auto it = g_occ.find(key);
        if (it != g_occ.end()) return it->second * num_cus();
    }
    if (set_lds(k_search_global<TE, TB>, lds_bytes) != hipSuccess) return 0;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_search_global<TE, TB>, block,
                                                     lds_bytes) != hipSuccess)
        return 0;
    std::lock_guard<std::mutex> lk(g_occ_mu);
    g_occ[key] = per_cu;
    return per_cu * num_cus();
}

int max_groups_global(int block, uint32_t lds_bytes, int tb16, int esz16)
{
    if (esz16 && tb16) return occupancy_global<uint16_t, uint16_t>(block, lds_bytes);
    if (esz16) return occupancy_global<uint16_t, int32_t>(block, lds_bytes);
    if (tb16) return occupancy_global<int32_t, uint16_t>(block, lds_bytes);
    return occupancy_global<int32_t, int32_t>(block, lds_bytes);
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
