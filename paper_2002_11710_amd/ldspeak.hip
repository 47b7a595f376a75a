// ldspeak.hip -- LDS read bandwidth and bank count of the GPU the library runs
// on, and its rate of random 2-byte gathers, for the rooflines the move-delta
// kernels are measured against.
//
// Every thread of a full grid reads 32-bit words of a 64 KiB LDS buffer in a
// loop: lane i of a wavefront starts at word (i * stride) mod 1024, and a
// thread's 8 reads of an iteration lie 2047 words apart (more than a paired
// read reaches and no multiple of 64 words, so each is its own ds_read_b32,
// and its offset is an immediate of the instruction: one address add per iteration, one
// accumulate per read, so the vector ALU never limits the LDS).  With stride 1
// the 64 lanes touch 64 consecutive words: no bank conflicts, so the bytes
// read over the kernel's time are the LDS read peak.  Larger strides make
// lanes share banks; the time against the stride gives the number of banks
// (the smallest stride beyond which the time stops growing).  One thread also
// reads the shader clock and the 100 MHz wall clock around its loop, which
// gives the clock the kernel ran at.  Every iteration moves each thread's reads
// by 17 words (mod 1024), so no read can be lifted out of the loop; the lane
// pattern, and with it the banks the lanes hit, stays the same.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kWords = 16384;           // 64 KiB
constexpr int kUnroll = 8;              // reads per iteration, kSpread words apart
constexpr int kSpread = 2047;

__global__ void __launch_bounds__(1024) k_lds_read(int iters, int stride, uint32_t *sink, uint64_t *clocks)
{
    __shared__ uint32_t buf[kWords];
    for (int k = threadIdx.x; k < kWords; k += blockDim.x) buf[k] = (uint32_t)k * 2654435761u;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int base = (wave * 64 * stride + lane * stride) & 1023;
    uint32_t acc = 0;
    const uint64_t c0 = clock64(), w0 = wall_clock64();
    for (int i = 0; i < iters; ++i) {
        // p + 7 * kSpread <= 2046 + 14329 < kWords: every read stays inside the buffer
        const uint32_t *q = buf + base + ((i * 17) & 1023);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) acc += q[u * kSpread];
    }
    const uint64_t c1 = clock64(), w1 = wall_clock64();
    if (acc == 0x12345678u) sink[blockIdx.x] = acc;   // keeps the reads alive
    if (blockIdx.x == 0 && threadIdx.x == 0) { clocks[0] = c1 - c0; clocks[1] = w1 - w0; }
}

// Random 2-byte gathers, the access pattern of the move-delta kernels' travel
// reads: every thread reads 16-bit entries of a 64 KiB LDS buffer at 8 offsets
// drawn per thread in the buffer's first half (a 32-bit linear congruential
// generator seeded by the thread's global index), all moved by the same step
// every iteration (so no read can be lifted out of the loop, and each stays in
// the buffer without masking: one address add and one accumulate per read).
// The lanes of a wavefront hit the banks as independent uniform draws do.
__global__ void __launch_bounds__(1024) k_lds_gather(int iters, uint32_t *sink, uint64_t *clocks)
{
    __shared__ uint16_t buf[2 * kWords];
    for (int k = threadIdx.x; k < 2 * kWords; k += blockDim.x) buf[k] = (uint16_t)((uint32_t)k * 40503u);
    __syncthreads();
    const char *bytes = (const char *)buf;
    uint32_t x = (blockIdx.x * blockDim.x + threadIdx.x) * 2654435761u + 12345u, a[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        x = x * 1664525u + 1013904223u;
        a[u] = (x >> 18) << 1;           // byte offset of one of the first kWords entries
    }
    uint32_t acc = 0;
    const uint64_t c0 = clock64(), w0 = wall_clock64();
    for (int i = 0; i < iters; ++i) {
        // offset + step <= 2 (kWords - 1) + 2 (kWords - 1) < 4 kWords bytes: inside the buffer
        const uint32_t sh = (((uint32_t)i * 4099u) & (kWords - 1)) << 1;
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) acc += *(const uint16_t *)(bytes + a[u] + sh);
    }
    const uint64_t c1 = clock64(), w1 = wall_clock64();
    if (acc == 0x12345678u) sink[blockIdx.x] = acc;
    if (blockIdx.x == 0 && threadIdx.x == 0) { clocks[0] = c1 - c0; clocks[1] = w1 - w0; }
}

}  // namespace

extern "C" {

// Run the gather loop on `blocks` workgroups of 1024 threads, `iters` x 8
// reads per thread.  Writes the kernel time (ms, HIP events), and the shader
// clocks and 100 MHz ticks one thread counted.  Returns 0, or the HIP error.
int ldspeak_gather_run(int blocks, int iters, double *ms, uint64_t *shader_clocks, uint64_t *wall_ticks)
{
    uint32_t *sink = nullptr;
    uint64_t *clk = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipMalloc((void **)&sink, sizeof(uint32_t) * (size_t)blocks);
    if (e == hipSuccess) e = hipMalloc((void **)&clk, 2 * sizeof(uint64_t));
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_lds_gather, dim3(blocks), dim3(1024), 0, 0, 1, sink, clk);   // warm-up
        (void)hipEventRecord(a, 0);
        hipLaunchKernelGGL(k_lds_gather, dim3(blocks), dim3(1024), 0, 0, iters, sink, clk);
        (void)hipEventRecord(b, 0);
        e = hipEventSynchronize(b);
    }
    if (e == hipSuccess) {
        float f = 0.f;
        e = hipEventElapsedTime(&f, a, b);
        *ms = f;
    }
    uint64_t h[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpy(h, clk, sizeof(h), hipMemcpyDeviceToHost);
    *shader_clocks = h[0];
    *wall_ticks = h[1];
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (sink) (void)hipFree(sink);
    if (clk) (void)hipFree(clk);
    return (int)e;
}

// Run the read loop on `blocks` workgroups of 1024 threads, `iters` x 16
// reads per thread, lane stride `stride` words.  Writes the kernel time (ms,
// HIP events), and the shader clocks and 100 MHz ticks one thread counted.
// Returns 0, or the HIP error.
int ldspeak_run(int blocks, int iters, int stride, double *ms, uint64_t *shader_clocks,
                uint64_t *wall_ticks)
{
    uint32_t *sink = nullptr;
    uint64_t *clk = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipMalloc((void **)&sink, sizeof(uint32_t) * (size_t)blocks);
    if (e == hipSuccess) e = hipMalloc((void **)&clk, 2 * sizeof(uint64_t));
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_lds_read, dim3(blocks), dim3(1024), 0, 0, 1, stride, sink, clk);   // warm-up
        (void)hipEventRecord(a, 0);
        hipLaunchKernelGGL(k_lds_read, dim3(blocks), dim3(1024), 0, 0, iters, stride, sink, clk);
        (void)hipEventRecord(b, 0);
        e = hipEventSynchronize(b);
    }
    if (e == hipSuccess) {
        float f = 0.f;
        e = hipEventElapsedTime(&f, a, b);
        *ms = f;
    }
    uint64_t h[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpy(h, clk, sizeof(h), hipMemcpyDeviceToHost);
    *shader_clocks = h[0];
    *wall_ticks = h[1];
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (sink) (void)hipFree(sink);
    if (clk) (void)hipFree(clk);
    return (int)e;
}

}  // extern "C"
