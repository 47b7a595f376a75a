// prepare.hip -- per-instance checks and the compact exit x entry travel block.
//
// Three launches, each covering every instance of the call:
//   k_scan_travel  (many workgroups per instance, 4096 entries each): every
//                  travel time inside [0, 2^23), and the largest one;
//   k_prepare      (one workgroup per instance): check every mission (pickup,
//                  delivery inside [0, L), pickup != delivery) and vehicle base;
//                  mark the exit locations (deliveries, bases) and entry
//                  locations (pickups, bases) in LDS bitmaps and rank them by a
//                  prefix sum of popcounts, so both are numbered in increasing
//                  location order; store each mission's (delivery row * Cs,
//                  pickup column), each vehicle's (base row * Cs, base column),
//                  the entry width, the strides and the sum of the loaded legs;
//   k_fill_blocks  (many workgroups per instance): copy the R x C block
//                  T[exit_loc[r]][enter_loc[c]] with row stride Cs, as uint16
//                  when every travel time is below 2^16, and, for solves that
//                  may take the HBM-resident schedule, the same block
//                  transposed (stride Rs) and with 16-byte aligned rows (stride Cg).
// A workgroup of the two many-workgroup kernels finds its instance from the
// per-instance first-chunk indices scan0 / fill0 the host fills in.
#include "atabu_internal.h"
#include "atabu.h"

namespace at {

constexpr int kPrepThreads = 256;
constexpr int kChunk = 4096;                       // entries per workgroup of scan and fill
constexpr int kMaxWords = (kMaxLocs + 31) / 32;   // 2048

__device__ __forceinline__ int rank_of(const uint32_t *bm, const uint32_t *pf, int loc)
{
    const int w = loc >> 5;
    const uint32_t below = bm[w] & ((1u << (loc & 31)) - 1u);
    return (int)pf[w] + __popc(below);
}

// instance whose chunk range [first(i), first(i + 1)) holds chunk b
template <typename F>
__device__ __forceinline__ int owner(int n, int64_t b, F first)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first(mid) <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(kPrepThreads) k_scan_travel(InstDev *insts, int n)
{
    const int64_t b = blockIdx.x;
    const int i = owner(n, b, [&](int k) { return (int64_t)insts[k].scan0; });
    InstDev &I = insts[i];
    const int64_t nn = (int64_t)I.L * I.L;
    const int64_t k0 = (b - I.scan0) * kChunk;
    int lmax = 0, bad = 0;
    for (int64_t k = k0 + threadIdx.x; k < min(nn, k0 + kChunk); k += blockDim.x) {
        const int x = I.T[k];
        bad |= (x < 0 || x >= kMaxTravel) ? 1 : 0;
        lmax = x > lmax ? x : lmax;
    }
    if (__any(bad) && (threadIdx.x & (kWave - 1)) == 0) atomicOr(&I.scan_bad, 1);
    for (int o = 32; o > 0; o >>= 1) lmax = max(lmax, __shfl_xor(lmax, o, 64));
    if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(&I.maxT, lmax);
}

__global__ void __launch_bounds__(kPrepThreads) k_prepare(InstDev *insts)
{
    __shared__ uint32_t bmx[kMaxWords], bme[kMaxWords], pfx[kMaxWords], pfe[kMaxWords];
    __shared__ uint32_t part_x[kPrepThreads], part_e[kPrepThreads];
    __shared__ int s_bad;
    __shared__ unsigned long long s_svc;

    InstDev &I = insts[blockIdx.x];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int L = I.L, M = I.M, V = I.V;
    const int nw = (L + 31) >> 5;
    const int32_t *__restrict__ T = I.T;

    for (int w = tid; w < nw; w += nthr) { bmx[w] = 0; bme[w] = 0; }
    if (tid == 0) { s_bad = 0; s_svc = 0; }
    __syncthreads();

    int64_t svc = 0;
    for (int m = tid; m < M; m += nthr) {
        const int p = I.p[m], d = I.d[m];
        if (p < 0 || p >= L || d < 0 || d >= L || p == d) { atomicOr(&s_bad, 1); continue; }
        atomicOr(&bme[p >> 5], 1u << (p & 31));
        atomicOr(&bmx[d >> 5], 1u << (d & 31));
    }
    for (int v = tid; v < V; v += nthr) {
        const int b = I.b[v];
        if (b < 0 || b >= L) { atomicOr(&s_bad, 1); continue; }
        atomicOr(&bme[b >> 5], 1u << (b & 31));
        atomicOr(&bmx[b >> 5], 1u << (b & 31));
    }
    __syncthreads();
    if (s_bad || I.scan_bad) {
        if (tid == 0) I.status = s_bad ? AT_EINVAL : AT_ERANGE;
        return;
    }
    for (int m = tid; m < M; m += nthr) svc += T[(int64_t)I.p[m] * L + I.d[m]];
    atomicAdd(&s_svc, (unsigned long long)svc);

    // exclusive prefix of popcounts over the bitmap words
    const int per = (nw + nthr - 1) / nthr;
    const int w0 = tid * per, w1 = min(nw, w0 + per);
    uint32_t sx = 0, se = 0;
    for (int w = w0; w < w1; ++w) { sx += __popc(bmx[w]); se += __popc(bme[w]); }
    part_x[tid] = sx;
    part_e[tid] = se;
    __syncthreads();
    if (tid == 0) {
        uint32_t ax = 0, ae = 0;
        for (int k = 0; k < nthr; ++k) {
            const uint32_t a = part_x[k], b = part_e[k];
            part_x[k] = ax; part_e[k] = ae;
            ax += a; ae += b;
        }
        I.R = (int32_t)ax;
        I.C = (int32_t)ae;
    }
    __syncthreads();
    sx = part_x[tid];
    se = part_e[tid];
    for (int w = w0; w < w1; ++w) {
        pfx[w] = sx; pfe[w] = se;
        sx += __popc(bmx[w]); se += __popc(bme[w]);
    }
    __syncthreads();

    const int R = I.R, C = I.C;
    const int esz = I.maxT <= 65535 ? 2 : 4;
    const int Cs = compact_stride(C, esz);
    const int Rs = staged_rows(R, esz);
    const int Cg = staged_cols(C, esz);
    if ((int64_t)R * Cs * esz > I.tc_cap ||
        (I.tct && ((int64_t)C * Rs * esz > I.tc_cap || (int64_t)R * Cg * esz > I.tc_cap))) {
        if (tid == 0) I.status = AT_ENOMEM;
        return;
    }
    // location lists in increasing order
    for (int w = tid; w < nw; w += nthr) {
        uint32_t bits = bmx[w];
        int r = (int)pfx[w];
        while (bits) { const int b = __ffs(bits) - 1; I.exit_loc[r++] = w * 32 + b; bits &= bits - 1u; }
        bits = bme[w];
        r = (int)pfe[w];
        while (bits) { const int b = __ffs(bits) - 1; I.enter_loc[r++] = w * 32 + b; bits &= bits - 1u; }
    }
    for (int m = tid; m < M; m += nthr) {
        I.mrow[m] = rank_of(bmx, pfx, I.d[m]) * Cs;
        I.mcol[m] = rank_of(bme, pfe, I.p[m]);
    }
    for (int v = tid; v < V; v += nthr) {
        I.vrow[v] = rank_of(bmx, pfx, I.b[v]) * Cs;
        I.vcol[v] = rank_of(bme, pfe, I.b[v]);
    }
    __syncthreads();
    if (tid == 0) {
        I.Cs = Cs;
        I.Rs = Rs;
        I.Cg = Cg;
        I.esz = esz;
        I.svc_sum = (int64_t)s_svc;
        I.status = AT_OK;
    }
}

template <typename TE>
__device__ __forceinline__ void fill_chunk(const InstDev &I, int64_t k0)
{
    const int L = I.L, R = I.R, C = I.C, Cs = I.Cs, Rs = I.Rs, Cg = I.Cg;
    const int32_t *__restrict__ T = I.T;
    const int64_t n1 = (int64_t)R * Cs, n2 = I.tct ? (int64_t)C * Rs : 0, n3 = I.tcr ? (int64_t)R * Cg : 0;
    TE *tc = (TE *)I.tc, *tct = (TE *)I.tct, *tcr = (TE *)I.tcr;
    for (int64_t k = k0 + threadIdx.x; k < k0 + kChunk; k += blockDim.x) {
        if (k < n1) {
            const int r = (int)(k / Cs), c = (int)(k - (int64_t)r * Cs);
            tc[k] = c < C ? (TE)T[(int64_t)I.exit_loc[r] * L + I.enter_loc[c]] : (TE)0;
        }
        if (k < n2) {
            // the same block transposed (entry-major)
            const int c = (int)(k / Rs), r = (int)(k - (int64_t)c * Rs);
            tct[k] = r < R ? (TE)T[(int64_t)I.exit_loc[r] * L + I.enter_loc[c]] : (TE)0;
        }
        if (k < n3) {
            // and row-major with 16-byte aligned rows
            const int r = (int)(k / Cg), c = (int)(k - (int64_t)r * Cg);
            tcr[k] = c < C ? (TE)T[(int64_t)I.exit_loc[r] * L + I.enter_loc[c]] : (TE)0;
        }
    }
}

__global__ void __launch_bounds__(kPrepThreads) k_fill_blocks(InstDev *insts, int n)
{
    const int64_t b = blockIdx.x;
    const int i = owner(n, b, [&](int k) { return (int64_t)insts[k].fill0; });
    const InstDev &I = insts[i];
    if (I.status != AT_OK) return;
    const int64_t k0 = (b - I.fill0) * kChunk;
    if (I.esz == 2) fill_chunk<uint16_t>(I, k0);
    else fill_chunk<int32_t>(I, k0);
}

int64_t prepare_chunks(const InstDev &h, int64_t *fill_chunks)
{
    const int64_t B = compact_bound(h.L, h.M, h.V);
    if (fill_chunks) *fill_chunks = (B * (B + 8) + kChunk - 1) / kChunk;
    return ((int64_t)h.L * h.L + kChunk - 1) / kChunk;
}

hipError_t launch_prepare(InstDev *insts, int32_t n, int64_t scan_chunks, int64_t fill_chunks, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (scan_chunks > 0)
        hipLaunchKernelGGL(k_scan_travel, dim3((unsigned)scan_chunks), dim3(kPrepThreads), 0, s, insts, (int)n);
    hipLaunchKernelGGL(k_prepare, dim3((unsigned)n), dim3(kPrepThreads), 0, s, insts);
    if (fill_chunks > 0)
        hipLaunchKernelGGL(k_fill_blocks, dim3((unsigned)fill_chunks), dim3(kPrepThreads), 0, s, insts, (int)n);
    return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n)
{
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        p[k] = v;
}

__global__ void k_fill_u64(uint64_t *p, uint64_t v, size_t n)
{
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        p[k] = v;
}

hipError_t fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t fill_u64(uint64_t *p, uint64_t v, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

}  // namespace at
