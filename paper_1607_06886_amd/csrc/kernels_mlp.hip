// Learned sampling proposal: BF16 MLP forward/backward on MFMA (FP32
// accumulation), mixture negative log-likelihood, Adam, mixture sampling.
#include <hip/hip_runtime.h>
#include <math.h>

#include "mlp_internal.hpp"

namespace pump {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
    // round to nearest even; NaN stays NaN
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------------------------
// C[M x N] = sum_k A[m][k] * B[n][k]  (both operands K-contiguous, BF16),
// FP32 accumulation on v_mfma_f32_16x16x32_bf16.  A block of 4 waves covers a
// 64 x 64 tile, each wave 32 x 32 (2 x 2 MFMA tiles); M, N, K are multiples
// of 32.  Lane l feeds row l % 16 and k = 8 (l / 16) .. +7 of each operand;
// it receives D[4 (l / 16) + r][l % 16], r = 0..3.
// ---------------------------------------------------------------------------
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_nt(const uint16_t* __restrict__ A, int lda,
                                                 const uint16_t* __restrict__ B, int ldb, int M,
                                                 int N, int K, EpiArgs ep) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m0 = blockIdx.y * 64 + (wave >> 1) * 32;
    const int n0 = blockIdx.x * 64 + (wave & 1) * 32;
    if (m0 >= M || n0 >= N) return;
    const int r = lane & 15, kq = (lane >> 4) * 8;
    f32x4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < K; k += 32) {
        bf16x8 a[2], b[2];
        for (int i = 0; i < 2; ++i) {
            const int row = m0 + 16 * i + r;
            a[i] = *reinterpret_cast<const bf16x8*>(A + (size_t)row * lda + k + kq);
        }
        for (int j = 0; j < 2; ++j) {
            const int row = n0 + 16 * j + r;
            b[j] = *reinterpret_cast<const bf16x8*>(B + (size_t)row * ldb + k + kq);
        }
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int rr = 0; rr < 4; ++rr) {
                const int m = m0 + 16 * i + 4 * (lane >> 4) + rr;
                const int n = n0 + 16 * j + (lane & 15);
                const float v = acc[i][j][rr];
                if (EPI == kEpiHidden) {
                    // z = v + b; h = relu(z) feeds the next layer (row- and column-major)
                    const float z = v + (n < ep.n_real ? ep.bias[n] : 0.0f);
                    const uint16_t h = f2bf(fmaxf(z, 0.0f));
                    ep.out_bf[(size_t)m * ep.ld_out + n] = h;
                    ep.out_bfT[(size_t)n * ep.ld_outT + m] = h;
                } else if (EPI == kEpiOutput) {
                    ep.out_f32[(size_t)m * ep.ld_out + n] = v + (n < ep.n_real ? ep.bias[n] : 0.0f);
                } else if (EPI == kEpiWgrad) {
                    if (m < ep.m_real && n < ep.n_real)
                        ep.out_f32[(size_t)m * ep.ld_out + n] = v;
                } else {  // kEpiDgrad: mask by the layer input's ReLU
                    const float keep = bf2f(ep.mask_bf[(size_t)m * ep.ld_mask + n]) > 0.0f ? 1.0f : 0.0f;
                    ep.out_f32[(size_t)m * ep.ld_out + n] = v * keep;
                }
            }
}

void launch_gemm_nt(hipStream_t s, int epi, const uint16_t* A, int lda, const uint16_t* B,
                    int ldb, int M, int N, int K, const EpiArgs& ep) {
    dim3 grid((N + 63) / 64, (M + 63) / 64);
    switch (epi) {
        case kEpiHidden: k_gemm_nt<kEpiHidden><<<grid, 256, 0, s>>>(A, lda, B, ldb, M, N, K, ep); break;
        case kEpiOutput: k_gemm_nt<kEpiOutput><<<grid, 256, 0, s>>>(A, lda, B, ldb, M, N, K, ep); break;
        case kEpiWgrad: k_gemm_nt<kEpiWgrad><<<grid, 256, 0, s>>>(A, lda, B, ldb, M, N, K, ep); break;
        default: k_gemm_nt<kEpiDgrad><<<grid, 256, 0, s>>>(A, lda, B, ldb, M, N, K, ep); break;
    }
}

// Condition rows (FP32, 396 wide) -> BF16 layer-1 input, padded to 416
// columns and Bp rows, plus its transpose.
__global__ void k_input_bf16(const float* __restrict__ X, int B, int Bp, int d_in, int d_pad,
                             uint16_t* __restrict__ H, uint16_t* __restrict__ HT) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Bp * d_pad) return;
    const int m = t / d_pad, k = t - m * d_pad;
    const float v = (m < B && k < d_in) ? X[(size_t)m * d_in + k] : 0.0f;
    const uint16_t h = f2bf(v);
    H[(size_t)m * d_pad + k] = h;
    HT[(size_t)k * Bp + m] = h;
}

void launch_input_bf16(hipStream_t s, const float* X, int B, int Bp, int d_in, int d_pad,
                       uint16_t* H, uint16_t* HT) {
    const int n = Bp * d_pad;
    k_input_bf16<<<(n + 255) / 256, 256, 0, s>>>(X, B, Bp, d_in, d_pad, H, HT);
}

// ---------------------------------------------------------------------------
// Mixture NLL and its gradient with respect to the 208 outputs, one row per
// thread.  Outputs: logits [16], means [16][6], log-std [16][6] clamped to
// [-4, 2].  G rows beyond the batch are zero; loss partial sums per block.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mixture_nll(const float* __restrict__ Y, int ldy,
                                                     const float* __restrict__ Z, int B, int Bp,
                                                     float* __restrict__ G, int ldg,
                                                     float* __restrict__ partial) {
    __shared__ float s_sum[256];
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    float loss = 0.0f;
    if (m < Bp) {
        float* g = G + (size_t)m * ldg;
        if (m >= B) {
            for (int j = 0; j < ldg; ++j) g[j] = 0.0f;
        } else {
            const float* y = Y + (size_t)m * ldy;
            float z[kDState];
            for (int d = 0; d < kDState; ++d) z[d] = Z[(size_t)m * kDState + d];
            float lmax = -INFINITY;
            for (int k = 0; k < kComp; ++k) lmax = fmaxf(lmax, y[k]);
            float se = 0.0f;
            for (int k = 0; k < kComp; ++k) se += expf(y[k] - lmax);
            const float lse_logit = lmax + logf(se);
            float a[kComp];
            float amax = -INFINITY;
            for (int k = 0; k < kComp; ++k) {
                float q = 0.0f, ssum = 0.0f;
                for (int d = 0; d < kDState; ++d) {
                    const float s = fminf(fmaxf(y[kComp * 7 + k * kDState + d], kLogStdMin), kLogStdMax);
                    const float rr = (z[d] - y[kComp + k * kDState + d]) * expf(-s);
                    q += rr * rr;
                    ssum += s;
                }
                a[k] = (y[k] - lse_logit) - 0.5f * q - ssum - 0.5f * kDState * 1.8378770664093453f;
                amax = fmaxf(amax, a[k]);
            }
            float sa = 0.0f;
            for (int k = 0; k < kComp; ++k) sa += expf(a[k] - amax);
            const float lse_a = amax + logf(sa);
            loss = -lse_a;
            const float invB = 1.0f / (float)B;
            for (int k = 0; k < kComp; ++k) {
                const float w = expf(a[k] - lse_a);
                const float pi = expf(y[k] - lse_logit);
                g[k] = (pi - w) * invB;
                for (int d = 0; d < kDState; ++d) {
                    const float raw = y[kComp * 7 + k * kDState + d];
                    const float s = fminf(fmaxf(raw, kLogStdMin), kLogStdMax);
                    const float inv = expf(-s);
                    const float rr = (z[d] - y[kComp + k * kDState + d]) * inv;
                    g[kComp + k * kDState + d] = -w * rr * inv * invB;
                    const bool inside = raw > kLogStdMin && raw < kLogStdMax;
                    g[kComp * 7 + k * kDState + d] = inside ? w * (1.0f - rr * rr) * invB : 0.0f;
                }
            }
            for (int j = kOut; j < ldg; ++j) g[j] = 0.0f;
        }
    }
    s_sum[threadIdx.x] = loss;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s_sum[threadIdx.x] += s_sum[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = s_sum[0];
}

__global__ void k_sum_partials(const float* __restrict__ partial, int n, int B,
                               float* __restrict__ loss) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += (double)partial[i];
    *loss = (float)(s / (double)B);
}

void launch_mixture_nll(hipStream_t s, const float* Y, int ldy, const float* Z, int B, int Bp,
                        float* G, int ldg, float* partial, float* loss) {
    const int blocks = (Bp + 255) / 256;
    k_mixture_nll<<<blocks, 256, 0, s>>>(Y, ldy, Z, B, Bp, G, ldg, partial);
    k_sum_partials<<<1, 64, 0, s>>>(partial, blocks, B, loss);
}

// FP32 gradient rows -> BF16 (row- and column-major) for the next products,
// and the bias gradient as column sums (sequential over rows: deterministic).
__global__ void k_grad_bf16(const float* __restrict__ G, int ldg, int Bp, int width,
                            uint16_t* __restrict__ GB, uint16_t* __restrict__ GBT) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Bp * width) return;
    const int m = t / width, n = t - m * width;
    const uint16_t h = f2bf(G[(size_t)m * ldg + n]);
    GB[(size_t)m * width + n] = h;
    GBT[(size_t)n * Bp + m] = h;
}

__global__ void k_colsum(const float* __restrict__ G, int ldg, int Bp, int n_real,
                         float* __restrict__ out) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_real) return;
    float s = 0.0f;
    for (int m = 0; m < Bp; ++m) s += G[(size_t)m * ldg + n];
    out[n] = s;
}

void launch_grad_prep(hipStream_t s, const float* G, int ldg, int Bp, int width, int n_real,
                      uint16_t* GB, uint16_t* GBT, float* bias_grad) {
    const int n = Bp * width;
    k_grad_bf16<<<(n + 255) / 256, 256, 0, s>>>(G, ldg, Bp, width, GB, GBT);
    k_colsum<<<(n_real + 255) / 256, 256, 0, s>>>(G, ldg, Bp, n_real, bias_grad);
}

// ---------------------------------------------------------------------------
// Adam (Kingma & Ba) on the FP32 master parameters, then the BF16 copies
// (row-major [out_p][in_p] and transposed [in_p][out_p], zero padded).
// ---------------------------------------------------------------------------
// (1 - beta) is passed rounded from its exact value: 1 - 0.999f in FP32 would be
// 1.3e-5 relatively off 0.001.
__global__ void k_adam(float* __restrict__ p, float* __restrict__ m1, float* __restrict__ m2,
                       const float* __restrict__ g, int n, float lr, float b1, float b2,
                       float omb1, float omb2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + omb1 * gi;
    const float b = b2 * m2[i] + omb2 * gi * gi;
    m1[i] = a;
    m2[i] = b;
    p[i] = p[i] - lr * (a / c1) / (sqrtf(b / c2) + eps);
}

void launch_adam(hipStream_t s, float* p, float* m1, float* m2, const float* g, int n, float lr,
                 int t) {
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 - pow(b1, t)), c2 = (float)(1.0 - pow(b2, t));
    k_adam<<<(n + 255) / 256, 256, 0, s>>>(p, m1, m2, g, n, lr, (float)b1, (float)b2,
                                           (float)(1.0 - b1), (float)(1.0 - b2), 1e-8f, c1, c2);
}

__global__ void k_refresh_bf16(const float* __restrict__ W, int out, int in, int out_p, int in_p,
                               uint16_t* __restrict__ Wb, uint16_t* __restrict__ WbT) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= out_p * in_p) return;
    const int n = t / in_p, k = t - n * in_p;
    const uint16_t h = (n < out && k < in) ? f2bf(W[(size_t)n * in + k]) : (uint16_t)0;
    Wb[(size_t)n * in_p + k] = h;
    WbT[(size_t)k * out_p + n] = h;
}

void launch_refresh_bf16(hipStream_t s, const float* W, int out, int in, int out_p, int in_p,
                         uint16_t* Wb, uint16_t* WbT) {
    const int n = out_p * in_p;
    k_refresh_bf16<<<(n + 255) / 256, 256, 0, s>>>(W, out, in, out_p, in_p, Wb, WbT);
}

// ---------------------------------------------------------------------------
// Condition vectors: start (6), goal centre (3) and half-size (3), then up to
// 64 boxes (lo xyz, hi xyz), zero padded.
// ---------------------------------------------------------------------------
__global__ void k_condition(const float* __restrict__ x_init, const float* __restrict__ goal,
                            const float* __restrict__ boxes, const int32_t* __restrict__ n_obs,
                            int q, int max_boxes_in, float* __restrict__ cond) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= q * kIn) return;
    const int i = t / kIn, j = t - i * kIn;
    float v = 0.0f;
    if (j < 6) {
        v = x_init[(size_t)i * 6 + j];
    } else if (j < 9) {
        v = 0.5f * (goal[(size_t)i * 6 + (j - 6)] + goal[(size_t)i * 6 + 3 + (j - 6)]);
    } else if (j < 12) {
        v = 0.5f * (goal[(size_t)i * 6 + 3 + (j - 9)] - goal[(size_t)i * 6 + (j - 9)]);
    } else {
        const int b = (j - 12) / 6, c = (j - 12) % 6;
        if (b < n_obs[i] && b < kMaxBoxes) v = boxes[((size_t)i * max_boxes_in + b) * 6 + c];
    }
    cond[(size_t)i * kIn + j] = v;
}

void launch_condition(hipStream_t s, const float* x_init, const float* goal, const float* boxes,
                      const int32_t* n_obs, int q, int max_boxes_in, float* cond) {
    const int n = q * kIn;
    k_condition<<<(n + 255) / 256, 256, 0, s>>>(x_init, goal, boxes, n_obs, q, max_boxes_in, cond);
}

// ---------------------------------------------------------------------------
// Mixture sampling: one draw per thread.  The component is chosen by the
// inverse CDF of softmax(logits) at u * total (FP64), the state is
// mu + sigma * eps, clamped to the state box.
// ---------------------------------------------------------------------------
__global__ void k_sample(const float* __restrict__ Y, int ldy, int q, int n,
                         const float* __restrict__ u, const float* __restrict__ eps,
                         float* __restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= q * n) return;
    const int i = t / n;
    const float* y = Y + (size_t)i * ldy;
    double mx = -INFINITY;
    for (int k = 0; k < kComp; ++k) mx = fmax(mx, (double)y[k]);
    double cdf[kComp];
    double acc = 0.0;
    for (int k = 0; k < kComp; ++k) {
        acc += exp((double)y[k] - mx);
        cdf[k] = acc;
    }
    const double target = (double)u[t] * acc;
    int k = 0;
    while (k < kComp - 1 && !(target < cdf[k])) ++k;
    const double lo[kDState] = {0.0, 0.0, 0.0, -0.5, -0.5, -0.5};
    const double hi[kDState] = {1.0, 1.0, 1.0, 0.5, 0.5, 0.5};
    for (int d = 0; d < kDState; ++d) {
        const double mu = (double)y[kComp + k * kDState + d];
        const double s = fmin(fmax((double)y[kComp * 7 + k * kDState + d], (double)kLogStdMin),
                              (double)kLogStdMax);
        double v = mu + exp(s) * (double)eps[(size_t)t * kDState + d];
        v = fmin(fmax(v, lo[d]), hi[d]);
        out[(size_t)t * kDState + d] = (float)v;
    }
}

void launch_sample(hipStream_t s, const float* Y, int ldy, int q, int n, const float* u,
                   const float* eps, float* out) {
    const int total = q * n;
    k_sample<<<(total + 255) / 256, 256, 0, s>>>(Y, ldy, q, n, u, eps, out);
}

}  // namespace pump
