// noise.hip -- photon-count (shot) noise for synthetic transient captures.
//
// Sec. 4.5 (non-line-of-sight capture simulation, "Realistic hardware
// noise") adds noise to simulated captures so that they resemble measured
// ones; the paper's model uses measurements of real devices.  This kernel is
// the measurement-free stand-in: every bin value v becomes N / scale with
// N ~ Poisson(scale * v), i.e. the film is read as an expected photon count
// scale * v and one capture of it is drawn.
//
// Sampling.  N is a sum of m independent Poisson(lambda / m) variables with
// m = ceil(lambda / 256) (additivity of the Poisson law), each drawn by
// sequential inversion of its CDF in FP64: with u uniform in [0, 1),
// N_j = min{k : u < sum_{i<=k} e^-mu mu^i / i!}.  e^-256 is far above the
// FP64 underflow threshold, so every term of the recurrence is representable.
// For lambda > 2^16 (far beyond any film normalised to a peak count of a
// few thousand) the normal approximation
// N = max(0, round(lambda + sqrt(lambda) z)) is used, z from the Box-Muller
// transform.  Uniforms come from Philox4x32-10 with
// key = seed and counter = (bin index lo, hi, draw block, kNoiseStream), two
// 53-bit uniforms per block, so the result depends only on (seed, index,
// value, scale).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_math.h"
#include "internal.h"

namespace trhip {
namespace {

constexpr uint32_t kNoiseStream = 0x6e6f6973u;
constexpr double kPieceMean = 256.0;
constexpr double kNormalAbove = 65536.0;
// a Poisson(256) draw exceeds 256 + 40 sqrt(256) with probability < 1e-300
constexpr int kMaxSteps = 256 + 40 * 16 + 64;

__device__ __forceinline__ double unit53(uint32_t hi, uint32_t lo)
{
    return (double)(((uint64_t)(hi >> 5) << 26) | (uint64_t)(lo >> 6)) * 0x1p-53;
}

// Poisson(mu) by inversion, 0 < mu <= kPieceMean
__device__ __forceinline__ double poisson_inverse(double mu, double u)
{
    double p = exp(-mu);
    double cdf = p;
    int k = 0;
    while (u >= cdf && k < kMaxSteps) {
        ++k;
        p = p * mu / (double)k;
        cdf += p;
    }
    return (double)k;
}

__global__ void k_poisson(const float* __restrict__ film, float* __restrict__ out, uint64_t n, float scale,
                          uint32_t key0, uint32_t key1)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const float v = film[i];
        const double lambda = (double)scale * (double)v;
        double count = 0.0;
        const uint32_t lo = (uint32_t)i, hi = (uint32_t)(i >> 32);
        if (lambda > kNormalAbove) {
            const u32x4 r = philox4x32_10(u32x4{lo, hi, 0u, kNoiseStream}, key0, key1);
            const double u1 = 1.0 - unit53(r.a, r.b);  // (0, 1]
            const double u2 = unit53(r.c, r.d);
            const double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
            count = fmax(0.0, rint(lambda + sqrt(lambda) * z));
        } else if (lambda > 0.0) {
            const uint32_t m = (uint32_t)ceil(lambda / kPieceMean);
            const double mu = lambda / (double)m;
            for (uint32_t j = 0; j < m; j += 2) {
                const u32x4 r = philox4x32_10(u32x4{lo, hi, j / 2, kNoiseStream}, key0, key1);
                count += poisson_inverse(mu, unit53(r.a, r.b));
                if (j + 1 < m) count += poisson_inverse(mu, unit53(r.c, r.d));
            }
        }
        out[i] = (float)(count / (double)scale);
    }
}

}  // namespace

hipError_t launch_poisson(const float* film, float* out, uint64_t n, float scale, uint64_t seed, hipStream_t stream)
{
    const unsigned g = (unsigned)std::min<uint64_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(k_poisson, dim3(g), dim3(256), 0, stream, film, out, n, scale, (uint32_t)seed,
                       (uint32_t)(seed >> 32));
    return hipGetLastError();
}

}  // namespace trhip
