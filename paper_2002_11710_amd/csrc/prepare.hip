// prepare.hip -- per-instance checks and the compact exit x entry travel block.
//
// One workgroup per instance:
//   1. check every mission (pickup, delivery inside [0, L), pickup != delivery)
//      and vehicle base, and every travel time inside [0, 2^23);
//   2. mark the exit locations (deliveries, bases) and entry locations
//      (pickups, bases) in LDS bitmaps and rank them by a prefix sum of
//      popcounts, so both are numbered in increasing location order;
//   3. copy the R x C block T[exit_loc[r]][enter_loc[c]] into the workspace with
//      row stride Cs, as uint16 when every travel time is below 2^16;
//   4. store each mission's (delivery row * Cs, pickup column) and each
//      vehicle's (base row * Cs, base column), and the sum of the loaded legs.
#include "atabu_internal.h"
#include "atabu.h"

namespace at {

constexpr int kPrepThreads = 256;
constexpr int kMaxWords = (kMaxLocs + 31) / 32;   // 2048

__device__ __forceinline__ int rank_of(const uint32_t *bm, const uint32_t *pf, int loc)
{
    const int w = loc >> 5;
    const uint32_t below = bm[w] & ((1u << (loc & 31)) - 1u);
    return (int)pf[w] + __popc(below);
}

__global__ void __launch_bounds__(kPrepThreads) k_prepare(InstDev *insts)
{
    __shared__ uint32_t bmx[kMaxWords], bme[kMaxWords], pfx[kMaxWords], pfe[kMaxWords];
    __shared__ uint32_t part_x[kPrepThreads], part_e[kPrepThreads];
    __shared__ int s_bad, s_max;
    __shared__ unsigned long long s_svc;

    InstDev &I = insts[blockIdx.x];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int L = I.L, M = I.M, V = I.V;
    const int nw = (L + 31) >> 5;
    const int32_t *__restrict__ T = I.T;

    for (int w = tid; w < nw; w += nthr) { bmx[w] = 0; bme[w] = 0; }
    if (tid == 0) { s_bad = 0; s_max = 0; s_svc = 0; }
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
    int lmax = 0;
    const int64_t nn = (int64_t)L * L;
    for (int64_t k = tid; k < nn; k += nthr) {
        const int x = T[k];
        if (x < 0 || x >= kMaxTravel) { atomicOr(&s_bad, 2); break; }
        lmax = x > lmax ? x : lmax;
    }
    atomicMax(&s_max, lmax);
    __syncthreads();
    if (s_bad) {
        if (tid == 0) I.status = (s_bad & 1) ? AT_EINVAL : AT_ERANGE;
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
    const int esz = s_max <= 65535 ? 2 : 4;
    const int Cs = compact_stride(C, esz);
    const int Rs = staged_rows(R, esz);
    if ((int64_t)R * Cs * esz > I.tc_cap || (I.tct && (int64_t)C * Rs * esz > I.tc_cap)) {
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
    __syncthreads();
    const int64_t total = (int64_t)R * Cs;
    if (esz == 2) {
        uint16_t *tc = (uint16_t *)I.tc;
        for (int64_t k = tid; k < total; k += nthr) {
            const int r = (int)(k / Cs), c = (int)(k - (int64_t)r * Cs);
            tc[k] = c < C ? (uint16_t)T[(int64_t)I.exit_loc[r] * L + I.enter_loc[c]] : (uint16_t)0;
        }
    } else {
        int32_t *tc = (int32_t *)I.tc;
        for (int64_t k = tid; k < total; k += nthr) {
            const int r = (int)(k / Cs), c = (int)(k - (int64_t)r * Cs);
            tc[k] = c < C ? T[(int64_t)I.exit_loc[r] * L + I.enter_loc[c]] : 0;
        }
    }
    if (I.tct) {
        // the same block transposed (entry-major), for the HBM-resident schedule
        const int64_t tt = (int64_t)C * Rs;
        if (esz == 2) {
            uint16_t *tct = (uint16_t *)I.tct;
            for (int64_t k = tid; k < tt; k += nthr) {
                const int c = (int)(k / Rs), r = (int)(k - (int64_t)c * Rs);
                tct[k] = r < R ? (uint16_t)T[(int64_t)I.exit_loc[r] * L + I.enter_loc[c]] : (uint16_t)0;
            }
        } else {
            int32_t *tct = (int32_t *)I.tct;
            for (int64_t k = tid; k < tt; k += nthr) {
                const int c = (int)(k / Rs), r = (int)(k - (int64_t)c * Rs);
                tct[k] = r < R ? T[(int64_t)I.exit_loc[r] * L + I.enter_loc[c]] : 0;
            }
        }
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
        I.esz = esz;
        I.maxT = s_max;
        I.svc_sum = (int64_t)s_svc;
        I.status = AT_OK;
    }
}

hipError_t launch_prepare(InstDev *insts, int32_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_prepare, dim3((unsigned)n), dim3(kPrepThreads), 0, s, insts);
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
