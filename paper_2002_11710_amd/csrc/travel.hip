// travel.hip -- Eq (1): travel time between two points from the haversine
// great-circle distance over the vehicle speed, in FP64, compiled without
// floating-point contraction so that every product and sum is rounded exactly
// as written:
//   s1 = sin((phi_j - phi_i) / 2), s2 = sin((psi_j - psi_i) / 2)
//   a  = s1*s1 + cos(phi_i)*cos(phi_j)*s2*s2
//   km = 2 * 6371 * asin(sqrt(min(1, a)))
//   T[i][j] = round_half_away(km * 3600 / speed)
// Latitudes phi and longitudes psi arrive in degrees.
//
// host_travel is the matrix the library's callers build (host libm, one pass
// over every ordered pair); k_travel computes the same expression on the
// device, one thread per ordered pair, with the device math library.
#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "atabu_internal.h"

namespace at {

static inline double haversine_seconds(double lat_i, double lon_i, double lat_j, double lon_j,
                                       double speed)
{
    const double rad = 3.14159265358979323846 / 180.0;
    const double phi_i = lat_i * rad, phi_j = lat_j * rad;
    const double psi_i = lon_i * rad, psi_j = lon_j * rad;
    const double s1 = std::sin((phi_j - phi_i) / 2.0);
    const double s2 = std::sin((psi_j - psi_i) / 2.0);
    const double a = s1 * s1 + std::cos(phi_i) * std::cos(phi_j) * s2 * s2;
    const double km = 2.0 * 6371.0 * std::asin(std::sqrt(std::fmin(1.0, a)));
    return km * 3600.0 / speed;
}

// Rows [r0, r1) of the matrix; false if a time does not fit int32.
static bool travel_rows(int32_t n, int32_t r0, int32_t r1, const double *lat, const double *lon,
                        double speed, int32_t *out)
{
    for (int32_t i = r0; i < r1; ++i)
        for (int32_t j = 0; j < n; ++j) {
            const double sec = haversine_seconds(lat[i], lon[i], lat[j], lon[j], speed);
            // llround of anything at or above 2^31 - 0.5 leaves int32
            if (!(sec < 2147483647.5)) return false;
            out[(int64_t)i * n + j] = (int32_t)std::llround(sec);
        }
    return true;
}

// Every entry is computed on its own, so splitting the rows over host threads
// (large matrices: the 10 000-mission workload has 4.8 million entries) gives
// the same matrix as one pass.
bool host_travel(int32_t n, const double *lat, const double *lon, double speed, int32_t *out)
{
    const int64_t nn = (int64_t)n * n;
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int nt = (int)std::min<int64_t>({(int64_t)std::min(hw, 16u), nn / 65536 + 1, (int64_t)n});
    if (nt <= 1) return travel_rows(n, 0, n, lat, lon, speed, out);
    std::vector<std::thread> pool;
    std::vector<char> ok((size_t)nt, 1);
    for (int k = 0; k < nt; ++k) {
        const int32_t r0 = (int32_t)((int64_t)n * k / nt), r1 = (int32_t)((int64_t)n * (k + 1) / nt);
        pool.emplace_back([=, &ok] { ok[(size_t)k] = travel_rows(n, r0, r1, lat, lon, speed, out) ? 1 : 0; });
    }
    for (auto &th : pool) th.join();
    return std::all_of(ok.begin(), ok.end(), [](char c) { return c != 0; });
}

__global__ void __launch_bounds__(256) k_travel(int32_t n, const double *__restrict__ lat,
                                               const double *__restrict__ lon, double speed,
                                               int32_t *__restrict__ out)
{
    const double rad = 3.14159265358979323846 / 180.0;
    const int64_t nn = (int64_t)n * n;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nn; k += stride) {
        const int32_t i = (int32_t)(k / n), j = (int32_t)(k - (int64_t)i * n);
        const double phi_i = lat[i] * rad, phi_j = lat[j] * rad;
        const double psi_i = lon[i] * rad, psi_j = lon[j] * rad;
        const double s1 = sin((phi_j - phi_i) / 2.0);
        const double s2 = sin((psi_j - psi_i) / 2.0);
        const double a = s1 * s1 + cos(phi_i) * cos(phi_j) * s2 * s2;
        const double km = 2.0 * 6371.0 * asin(sqrt(fmin(1.0, a)));
        const double sec = km * 3600.0 / speed;
        // a time that does not fit int32 saturates (and fails the solve's range check)
        out[k] = sec < 2147483647.5 ? (int32_t)llround(sec) : INT32_MAX;
    }
}

hipError_t launch_travel(int32_t n, const double *lat, const double *lon, double speed,
                         int32_t *out, hipStream_t s)
{
    const int64_t nn = (int64_t)n * n;
    int64_t blocks = (nn + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_travel, dim3((unsigned)blocks), dim3(256), 0, s, n, lat, lon, speed, out);
    return hipGetLastError();
}

}  // namespace at
