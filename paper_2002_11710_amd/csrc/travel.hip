// travel.hip -- Eq (1): travel time between two points from the haversine
// great-circle distance over the vehicle speed.  One thread per (i, j) pair,
// FP64 throughout, compiled without floating-point contraction so that every
// product and sum is rounded exactly as written:
//   s1 = sin((phi_j - phi_i) / 2), s2 = sin((psi_j - psi_i) / 2)
//   a  = s1*s1 + cos(phi_i)*cos(phi_j)*s2*s2
//   km = 2 * 6371 * asin(sqrt(min(1, a)))
//   T[i][j] = round_half_away(km * 3600 / speed)
// Latitudes phi and longitudes psi arrive in degrees.
#include "atabu_internal.h"

namespace at {

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
        out[k] = (int32_t)llround(sec);
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
