// SampleFree(n) (Alg. 3) with the Halton sequence, as the paper samples the
// state space (Sec. V-A): coordinate d of point i is the radical inverse of i
// in the d-th prime base (2, 3, 5, 7, 11, 13), mapped onto the sampling box.
// The mirrored digits and the base power are exact integers (i < 2^31 keeps
// both below 2^53), so phi is one correctly rounded FP64 division; the box
// mapping rounds after each operation (no contraction) and stores FP32.
#include <hip/hip_runtime.h>

#include "pump_internal.hpp"

namespace pump {

namespace {

__device__ __forceinline__ double radical_inverse(uint64_t i, uint64_t b) {
    uint64_t R = 0, B = 1;
    while (i > 0) {
        const uint64_t q = i / b;
        R = R * b + (i - q * b);
        B *= b;
        i = q;
    }
    return (double)R / (double)B;
}

struct HaltonBox {
    double lo[6], hi[6];
};

// thread t = point r * 6 + coordinate d
__global__ void k_halton(int64_t start, int32_t n, HaltonBox box, float* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * 6) return;
    const int d = (int)(t % 6);
    const int64_t r = t / 6;
    constexpr uint64_t kBase[6] = {2, 3, 5, 7, 11, 13};
    const double phi = radical_inverse((uint64_t)(start + r), kBase[d]);
    const double x = __dadd_rn(box.lo[d], __dmul_rn(__dadd_rn(box.hi[d], -box.lo[d]), phi));
    out[t] = (float)x;
}

}  // namespace

hipError_t launch_halton(hipStream_t s, int64_t start, int32_t n, const float* lo, const float* hi,
                         float* out) {
    if (n <= 0) return hipSuccess;
    HaltonBox box;
    for (int d = 0; d < 6; ++d) {
        box.lo[d] = (double)lo[d];
        box.hi[d] = (double)hi[d];
    }
    const int64_t threads = (int64_t)n * 6;
    k_halton<<<(unsigned)((threads + 255) / 256), 256, 0, s>>>(start, n, box, out);
    return hipGetLastError();
}

}  // namespace pump
