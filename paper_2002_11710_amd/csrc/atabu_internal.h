// atabu_internal.h -- data layouts shared by the library's kernels and its host
// code (never by the oracle).
//
// Device representation of an instance (built once per instance by the
// prepare kernel):
//   * The search only ever needs a flight from some location a vehicle LEAVES
//     (a mission's delivery or a base) to some location it ENTERS (a mission's
//     pickup or a base).  The prepare kernel therefore renumbers the exit
//     locations 0..R-1 and the entry locations 0..C-1 in increasing location
//     order and stores the R x C block of the travel matrix, row stride Cs,
//     as uint16 when every travel time fits (else int32).  Mission m keeps
//     mrow[m] = (exit row of its delivery) * Cs and mcol[m] = entry column of
//     its pickup; vehicle v keeps vrow[v], vcol[v] for its base.  Each
//     mission's loaded leg (pickup -> delivery) is the same in every solution,
//     so only their sum svc_sum is kept.
//   * The stride Cs makes rows land on different LDS banks: Cs = 2 mod 4 for
//     16-bit entries (odd in dwords), odd for 32-bit entries.
//
// Solve state (per solve, in LDS for the LDS-resident schedules):
//   seq[i]   mission at flat position i (routes concatenated by vehicle)
//   off[v]   first flat position of vehicle v, off[V] = M
//   rt[i]    vehicle of flat position i
//   pof[m], rof[m]  flat position / vehicle of mission m
//   tabu[v*M + m] = 1 + last iteration at which m may not enter v (0 = never)
// Per-iteration arrays (rebuilt from the state every iteration), 16-byte
// records so that one LDS broadcast read brings a whole column to a wavefront:
//   posA[i] = {mrow, mcol of the mission at i, xr, yc}
//             xr = exit row offset of its predecessor (or the base),
//             yc = entry column of its successor (or the base)
//   posB[i] = {outv, link, mission | vehicle << 16, rank}
//             outv = T[xr][p] + T[d][yc], link = T[xr][yc], rank = rank of the
//             mission id among the positions of its column chunk
//   gap[G]  = {ga, gb, gc, gr}: G = i + rt[i] is the gap before position i and
//             G = off[v+1] + v the gap before vehicle v's return; ga = exit row
//             offset on its left, gb = entry column on its right, gc = T[ga][gb],
//             gr = its vehicle
//   gend[G] = first gap of the next vehicle's route (where G's route ends)
//   prank[c*chunk + k] = position (within chunk c) of the mission of rank k
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace at {

constexpr int kWave = 64;
constexpr uint64_t kKeyNone = ~0ull;
constexpr int32_t kDeltaBias = 1 << 30;
constexpr int32_t kMaxTravel = 1 << 23;       // travel times must be below this (97 days)
constexpr int kMaxLocs = 65535;
constexpr int kMaxMissions = 65535;
constexpr int kMaxVehicles = 65535;
constexpr int kMaxGroups = 256;               // workgroups of one cooperative solve
// Exchange slots sit one per 128-byte line: workgroups that publish into one
// line and workgroups polling it contend (measured on gfx950: an exchange among
// 46 workgroups takes 1.6 us with contiguous slots, 1.0 us with one per line).
constexpr int kSlotStride = 16;
constexpr int kMaxClasses = 16;               // concurrent one-workgroup-per-job launches
constexpr int kMaxMultiJobs = 8;              // multi-workgroup solves sharing one launch

struct InstDev {
    // filled by the host
    int32_t L, M, V;
    int32_t pad0;
    const int32_t *T, *p, *d, *b;     // caller's device arrays
    int32_t *exit_loc, *enter_loc;    // workspace, L each
    int32_t *mrow, *mcol, *vrow, *vcol;
    void *tc;                         // workspace, capacity tc_cap bytes
    void *tct;                        // transposed block (C rows, stride Rs) or null
    void *tcr;                        // the block again with 16-byte aligned rows (stride Cg), or null
    int64_t tc_cap;
    int32_t scan0, fill0;             // first chunk of this instance in the scan / fill launches
    int32_t scan_bad;                 // a travel time outside [0, 2^23) (scan launch)
    // filled by the prepare kernels
    int32_t status;
    int32_t R, C, Cs, esz;            // esz = 2 or 4 bytes per compact entry
    int32_t Rs;                       // row stride of the transposed block
    int32_t Cg;                       // row stride of the aligned copy
    int32_t maxT;
    int64_t svc_sum;
    // the constrained model (null / 0 when off; filled by the host)
    const int32_t *T2, *vtype, *w, *heli;
    int32_t flimit, horizon;          // flimit <= 0: no flight limit
};

// An instance uses the constrained model when any of its fields is set.
__host__ __device__ inline bool constrained(const InstDev &d)
{
    return d.T2 || d.vtype || d.w || d.heli || d.flimit > 0;
}

struct JobScal {
    int64_t best_obj, final_obj;
    int32_t iters_done, best_iter, status, stopped;
};

// Saved search state (for chunked execution and the HBM-resident schedule).
struct SolveState {
    int32_t *seq, *off, *tabu;        // M, V+1, M*V (tabu in the 1 + until encoding)
    int64_t cur, best;
    int32_t t, best_iter, stopped, valid;
};

// HBM-resident state of one solve (the global schedule): the route arrays
// are double-buffered so that every workgroup can write the next iteration's
// routes while others still read the current ones.
struct GlobalBufs {
    // routes and the records built from them, double-buffered: an iteration reads
    // one parity and writes the next iteration's routes and records to the other
    uint16_t *seq[2], *rt[2], *pof[2], *rof[2];
    int32_t *off[2];
    int4 *posA[2], *posB[2], *gap[2];
    int2 *posC[2];                    // per position: exit row of its delivery, of its predecessor
    // tabu state as a ring of the entries set in the last ring_slots iterations,
    // two per iteration ({vehicle, mission, first iteration it is allowed again, 0};
    // an unused entry has 0 there): every entry set earlier has expired, so a
    // move is tabu exactly when the ring holds its (vehicle, mission) with a
    // value above the iteration
    int4 *ring;
    int32_t ring_slots;               // min(tenure + 1, max_iters), at least 1
    int32_t cur;                      // which parity holds the current routes
    // exchange of the solve's workgroups (reset before every launch): per-workgroup
    // slots of each barrier, 2 x kMaxGroups of them kSlotStride apart (buffer b & 1
    // for barrier b, bit 63 = bit 1 of b, the rest an encoded key), an abort flag
    // and the greedy objective
    uint64_t *slots;
    alignas(128) uint32_t abort;      // set by a workgroup whose wait ran out
    uint32_t pad2;
    int64_t init_obj;                 // greedy objective, published by workgroup 0
};

struct JobDev {
    const InstDev *inst;
    int32_t variant, tenure, max_iters, aspiration, trace;
    int32_t t_begin, t_end;           // iterations run by this launch
    int32_t resume, save;             // load / store `st`
    int32_t tb16;                     // tabu entries stored as uint16 in LDS
    int32_t chunk;                    // partner positions per swap work unit
    int32_t rchunk;                   // gaps per relocate work unit
    int32_t form;                     // AT_FORM_BEST or AT_FORM_SWEEP (wave schedule)
    int32_t gk;                       // global schedule: missions staged per block
    int32_t g0, ng;                   // global / multi schedules: the solve's workgroups in the launch
    int32_t sched;                    // AT_SCHED_* the solve runs on
    int32_t mx;                       // multi schedule: the solve's argmin slot set in Xchg
    uint64_t seed;
    int32_t *out_off, *out_seq, *out_of;
    int32_t *fin_off, *fin_seq;       // routes after the last iteration (may be null)
    uint32_t *tr_move;
    int32_t *tr_delta;
    int64_t *tr_obj;
    uint8_t *tr_flags;
    JobScal *scal;
    SolveState *st;
    GlobalBufs *gb;                   // global schedule only
};

// Device-side scheduling state of a call (the global schedule keeps its own in
// each solve's GlobalBufs).
struct Xchg {
    // per-workgroup argmin slots of the multi-workgroup schedule, one set per solve of
    // a launch, double-buffered by iteration parity; bit 63 carries the iteration's tag
    // (bit 1 of the iteration)
    uint64_t slots[kMaxMultiJobs][2][kMaxGroups * kSlotStride];   // workgroup w at w * kSlotStride
    uint32_t queues[kMaxClasses];     // next job of each one-workgroup-per-job launch
};

struct Lay {
    uint32_t tc, mrow, mcol, vrow, vcol, off, seq, rt, rof, pof;
    uint32_t posA, posB, gap, gend, prank, tabu, red, total;
};

__host__ __device__ inline uint32_t al16(uint32_t x) { return (x + 15u) & ~15u; }

__host__ __device__ inline Lay lds_layout(int M, int V, int R, int Cs, int esz, int tbsz)
{
    Lay l;
    uint32_t o = 0;
    uint32_t uM = (uint32_t)M, uV = (uint32_t)V, NG = uM + uV;
#define AT_TAKE(field, bytes) do { l.field = o; o = al16(o + (uint32_t)(bytes)); } while (0)
    AT_TAKE(tc, (uint64_t)R * (uint64_t)Cs * (uint64_t)esz);
    AT_TAKE(mrow, 4 * uM);
    AT_TAKE(mcol, 4 * uM);
    AT_TAKE(vrow, 4 * uV);
    AT_TAKE(vcol, 4 * uV);
    AT_TAKE(off, 4 * (uV + 1));
    AT_TAKE(seq, 2 * uM);
    AT_TAKE(rt, 2 * uM);
    AT_TAKE(rof, 2 * uM);
    AT_TAKE(pof, 2 * uM);
    AT_TAKE(posA, 16 * uM);
    AT_TAKE(posB, 16 * uM);
    AT_TAKE(gap, 16 * NG);
    AT_TAKE(gend, 2 * NG);
    AT_TAKE(prank, uM);
    AT_TAKE(tabu, (uint64_t)tbsz * uM * uV);
    AT_TAKE(red, 1024);
#undef AT_TAKE
    l.total = o;
    return l;
}

// Compact-matrix stride for C entry columns of esz bytes.
__host__ __device__ inline int compact_stride(int C, int esz)
{
    if (C < 1) C = 1;
    if (esz == 2) {
        int s = C;
        while ((s & 3) != 2) ++s;
        return s;
    }
    return C | 1;
}

// Upper bound of the exit rows / entry columns of an instance.
__host__ __device__ inline int64_t compact_bound(int L, int M, int V)
{
    int64_t r = (int64_t)M + V;
    return r < L ? r : L;
}

// Bytes of the HBM state of one solve on the global schedule (GlobalBufs arrays).
__host__ __device__ inline uint64_t global_state_bytes(int M, int V, int ring_slots)
{
    const uint64_t uM = (uint64_t)M, uV = (uint64_t)V, NG = uM + uV;
    auto a = [](uint64_t x) { return (x + 255u) & ~(uint64_t)255u; };
    return 8 * a(2 * uM) + 2 * a(4 * (uV + 1)) + 2 * (2 * a(16 * uM) + a(16 * NG) + a(8 * uM))
         + a(32 * (uint64_t)ring_slots) + a(2ull * kMaxGroups * kSlotStride * 8);
}

__host__ __device__ inline int64_t n_slots(int64_t M, int64_t V) { return M * (M + V) + M * (M - 1) / 2; }

// ---- launchers (defined in the .hip files) ----
hipError_t launch_travel(int32_t n, const double *lat, const double *lon, double speed,
                         int32_t *out, hipStream_t s);
// Eq (1) on the host (false if a time does not fit int32)
bool host_travel(int32_t n, const double *lat, const double *lon, double speed, int32_t *out);
// chunks of the travel scan of one instance (returned) and of its block fill (out)
int64_t prepare_chunks(const InstDev &h, int64_t *fill_chunks);
hipError_t launch_prepare(InstDev *insts, int32_t n, int64_t scan_chunks, int64_t fill_chunks, hipStream_t s);
hipError_t launch_search_wg(const JobDev *jobs, int32_t n_jobs, uint32_t *queue, int grid, int block,
                            uint32_t lds_bytes, int tb16, int esz16, hipStream_t s);
hipError_t launch_search_wg_wave(const JobDev *jobs, int32_t n_jobs, uint32_t *queue, int grid,
                                 int waves_per_group, uint32_t lds_per_solve, int tb16, int esz16,
                                 hipStream_t s);
// The multi-workgroup solves jobs[0..n_jobs) in one cooperative launch, each on its
// range [g0, g0 + ng) of the n_groups workgroups, with its own slot set (mx).
hipError_t launch_search_multi(const JobDev *jobs, int n_jobs, Xchg *xs, int n_groups, int block,
                               uint32_t lds_bytes, int tb16, int esz16, hipStream_t s);
hipError_t launch_search_global(const JobDev *jobs, int n_jobs, int n_groups, int block,
                                uint32_t lds_bytes, int tb16, int esz16, hipStream_t s);
int max_groups_global(int block, uint32_t lds_bytes, int tb16, int esz16);
// One grid for both kinds (block kGlobalBlock), cooperative: n_ggroups
// workgroups for the global jobs `gjobs` (each on its range), n_workers taking
// the jobs of `wjobs` from queue[0]: one-workgroup jobs, and global jobs run on
// a single workgroup (sched says which).  Resets every global job's exchange
// state first.
hipError_t launch_search_mixed(const JobDev *gjobs, int n_gjobs, int n_ggroups, const JobDev *wjobs, int n_wjobs,
                               uint32_t *queue, int n_workers, uint32_t lds_bytes, int tb16, int esz16,
                               hipStream_t s);
int max_groups_mixed(uint32_t lds_bytes, int tb16, int esz16);
// Missions staged per block by the global schedule's eval, at most.
constexpr int kGlobalKMax = 64;
static_assert(kGlobalKMax <= kWave, "a block's missions fit one wavefront");
// Threads per workgroup of the global schedule, at most.
constexpr int kGlobalBlock = 512;

// Staged lengths (elements) of the travel vectors of the global schedule's
// eval: a column of the block (R exit rows) and a row (C entry columns), each
// in whole 16-byte chunks.  They are also the row strides of the transposed
// block and of the aligned copy, whose rows are therefore 16-byte aligned.
__host__ __device__ inline int staged_rows(int R, int esz) { const int q = 16 / esz; return (R + q - 1) / q * q; }
__host__ __device__ inline int staged_cols(int C, int esz) { const int q = 16 / esz; return (C + q - 1) / q * q; }

// Per-block tables of the global schedule's eval: 4 source pointers, two int4
// records and a vehicle slot per mission, and the vehicle count.
__host__ __device__ inline uint32_t global_table_bytes(int K)
{
    return (uint32_t)(32 * K + 32 * K + ((4 * K + 8 + 15) & ~15));
}

// LDS bytes of the global schedule's mission-major eval: the per-block tables,
// K missions' four travel vectors and tabu columns, one tabu bit row (M bits)
// per vehicle of the block (at most K), then 2 KiB of reduction slots.
__host__ __device__ inline uint32_t global_lds_bytes(int K, int R, int C, int M, int V, int esz, int tbsz)
{
    const uint64_t Re = (uint64_t)staged_rows(R, esz), Ce = (uint64_t)staged_cols(C, esz);
    const uint64_t vec = (uint64_t)K * (2 * Re + 2 * Ce) * (uint64_t)esz;
    const uint64_t tk = (uint64_t)K * (uint64_t)V * (uint64_t)tbsz;
    const uint64_t rb = (uint64_t)K * (((uint64_t)M + 31) / 32) * 4;
    const uint64_t tot = global_table_bytes(K) + ((vec + 15) & ~15ull) + ((tk + 15) & ~15ull)
                       + ((rb + 15) & ~15ull) + 2048;
    return tot > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)tot;
}
hipError_t launch_debug_keys(const JobDev *job, const int32_t *off, const int32_t *seq,
                             const int32_t *tabu_until, int32_t t, int64_t cur, int64_t best,
                             uint64_t *keys, int block, uint32_t lds_bytes, int esz16,
                             hipStream_t s);
int max_groups_multi(int block, uint32_t lds_bytes, int tb16, int esz16);
// wave schedule: LDS bytes of one solve, launcher, key dump
uint32_t wave_lds_bytes(int M, int V, int R, int Cs, int esz, bool two);
constexpr int kWaveMaxMissions = 1024;
constexpr int kWaveMaxVehicles = 256;
hipError_t launch_search_wave(const JobDev *jobs, int32_t n_jobs, uint32_t *queue, int grid,
                              int waves_per_group, uint32_t lds_per_solve, int esz16, hipStream_t s);
hipError_t launch_debug_keys_wave(const JobDev *job, const int32_t *off, const int32_t *seq,
                                  const int32_t *tabu_until, int32_t t, int64_t cur, int64_t best,
                                  uint64_t *keys, uint32_t lds_bytes, int esz16, hipStream_t s);
uint32_t max_lds_bytes();
int num_cus();
hipError_t fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s);
hipError_t fill_u64(uint64_t *p, uint64_t v, size_t n, hipStream_t s);

// The pair (m1 < m2) of swap number sp, the swaps numbered row by row (row m1
// starts at m1*M - m1(m1+1)/2).  The row is the floor of the smaller root of
// the row-start quadratic, (A - sqrt(A^2 - 8 sp)) / 2 with A = 2M - 1: in double
// precision the square's argument is exact (below 2^53) and the computed root
// is off by a few units in the last place of a value below 2^17 (far below
// 2^-30), so the floor is off by at most one, next to a row boundary, and one
// test each way corrects it.
__device__ __forceinline__ void swap_pair(uint32_t sp, int M, int &m1, int &m2)
{
    const double A = 2.0 * (double)M - 1.0;
    int a = (int)floor((A - sqrt(A * A - 8.0 * (double)sp)) * 0.5);
    a = max(0, min(a, M - 2));
    auto rowstart = [&](int64_t x) { return x * M - x * (x + 1) / 2; };
    if (a + 1 <= M - 2 && rowstart(a + 1) <= (int64_t)sp) ++a;
    else if (a > 0 && rowstart(a) > (int64_t)sp) --a;
    m1 = a;
    m2 = (int)(a + 1 + ((int64_t)sp - rowstart(a)));
}

// ---------------------------------------------------------------------------
// Wavefront minimum on the VALU's data-parallel primitives (DPP): each step is
// one v_min_u32 whose second operand comes from another lane of the row (quad
// swaps, the half-row and row mirrors) or, for rows 1 and 3 and then rows 2
// and 3, from the last lane of the row before (row broadcasts 15 and 31), so
// lane 63 ends with the minimum of all 64 lanes, read out as a wave-uniform
// value.  Lanes a step does not write keep their value (the old operand is the
// identity).  The 64-bit form takes the minimum of the high words, then of the
// low words among the lanes that hold it.  Every lane of the wavefront must be
// active.
// ---------------------------------------------------------------------------
// The index of the calling thread's wavefront in its workgroup, as a scalar.
// Every lane computes the same tid / 64, but the compiler cannot tell: what is
// derived from it (a wavefront's work units, their bounds, loop counters) would
// be held per lane, its loops run with vector counters and exec-mask updates,
// and a lane index taken from it needs a readfirstlane at every use.
__device__ __forceinline__ int wave_id(int tid)
{
    return __builtin_amdgcn_readfirstlane(tid / kWave);
}

// A value every lane of the wavefront holds alike (an instance's sizes, a job
// index read from LDS), as a scalar.  Loads through generic pointers (the
// instance a job points to) and from LDS count as per-lane for the compiler,
// with the same cost for what is derived from them as above.
__device__ __forceinline__ int uniform(int x)
{
    return __builtin_amdgcn_readfirstlane(x);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_min_step(uint32_t x)
{
    const uint32_t y = (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFFu, (int)x, CTRL, ROWS, 0xF, false);
    return x < y ? x : y;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x)
{
    x = dpp_min_step<0xB1, 0xF>(x);    // quad_perm [1,0,3,2]
    x = dpp_min_step<0x4E, 0xF>(x);    // quad_perm [2,3,0,1]
    x = dpp_min_step<0x141, 0xF>(x);   // row_half_mirror
    x = dpp_min_step<0x140, 0xF>(x);   // row_mirror
    x = dpp_min_step<0x142, 0xA>(x);   // row_bcast:15 into rows 1 and 3
    x = dpp_min_step<0x143, 0xC>(x);   // row_bcast:31 into rows 2 and 3
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t k)
{
    const uint32_t hi = wave_min_u32((uint32_t)(k >> 32));
    const uint32_t lo = wave_min_u32((uint32_t)(k >> 32) == hi ? (uint32_t)k : 0xFFFFFFFFu);
    return ((uint64_t)hi << 32) | lo;
}

}  // namespace at
