// probe.hip -- the renderer's FP32 and integer primitives evaluated one by
// one on the device, with the same device functions and the same compiler
// flags as the render kernels, so that a test can compare them bit for bit
// with an independent host implementation: the random numbers (Philox),
// the two transcendental approximations that decide sampled directions and
// free-flight distances, and the correctly rounded division and square root
// that every ray, hit point and bin index goes through.
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "internal.h"

namespace trhip {

namespace {

__global__ void k_probe(int op, const void* __restrict__ in, void* __restrict__ out, uint64_t n, uint64_t first)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        switch (op) {
        case kProbeSinCos2Pi: {
            const float u = (float)(uint32_t)(first + i) * 0x1p-24f;
            float s, c;
            sincos_2pi(u, s, c);
            reinterpret_cast<float2*>(out)[i] = make_float2(s, c);
            break;
        }
        case kProbeLog1m: {
            const float u = (float)(uint32_t)(first + i) * 0x1p-24f;
            reinterpret_cast<float*>(out)[i] = log_one_minus(u);
            break;
        }
        case kProbePhilox: {
            const uint32_t* w = reinterpret_cast<const uint32_t*>(in) + 6 * i;
            const u32x4 r = philox4x32_10(u32x4{w[0], w[1], w[2], w[3]}, w[4], w[5]);
            reinterpret_cast<uint4*>(out)[i] = make_uint4(r.a, r.b, r.c, r.d);
            break;
        }
        case kProbeDiv: {
            const float2 ab = reinterpret_cast<const float2*>(in)[i];
            reinterpret_cast<float*>(out)[i] = ab.x / ab.y;
            break;
        }
        default: {  // kProbeSqrt
            reinterpret_cast<float*>(out)[i] = sqrtf(reinterpret_cast<const float*>(in)[i]);
            break;
        }
        }
    }
}

}  // namespace

hipError_t launch_probe(int op, const void* in, void* out, uint64_t n, uint64_t first, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    const uint64_t blocks = (n + 255) / 256;
    const unsigned g = (unsigned)(blocks < 65536 ? blocks : 65536);
    hipLaunchKernelGGL(k_probe, dim3(g), dim3(256), 0, stream, op, in, out, n, first);
    return hipGetLastError();
}

}  // namespace trhip
