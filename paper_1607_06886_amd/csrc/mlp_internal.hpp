// Internal declarations of the learned-proposal MLP.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pump {

constexpr int kComp = 16;               // mixture components
constexpr int kDState = 6;              // state dimension
constexpr int kMaxBoxes = 64;           // boxes in the condition vector
constexpr int kIn = 12 + 6 * kMaxBoxes; // 396 condition values
constexpr int kInPad = 416;             // padded to a multiple of 32
constexpr int kHidden = 256;
constexpr int kOut = kComp * (1 + 2 * kDState);  // 208 outputs
constexpr int kOutPad = 224;
constexpr int kLayers = 5;              // 4 hidden + output
constexpr float kLogStdMin = -4.0f, kLogStdMax = 2.0f;

enum { kEpiHidden = 0, kEpiOutput = 1, kEpiWgrad = 2, kEpiDgrad = 3 };

struct EpiArgs {
    const float* bias;      // [n_real]
    int n_real;             // columns with a bias / kept
    int m_real;             // rows kept (wgrad)
    uint16_t* out_bf;       // hidden: BF16 activations [M][ld_out]
    uint16_t* out_bfT;      // hidden: transpose [N][ld_outT]
    int ld_out, ld_outT;
    float* out_f32;         // output / wgrad / dgrad destination
    const uint16_t* mask_bf;  // dgrad: layer input activations (ReLU mask)
    int ld_mask;
};

void launch_gemm_nt(hipStream_t s, int epi, const uint16_t* A, int lda, const uint16_t* B,
                    int ldb, int M, int N, int K, const EpiArgs& ep);
void launch_input_bf16(hipStream_t s, const float* X, int B, int Bp, int d_in, int d_pad,
                       uint16_t* H, uint16_t* HT);
void launch_mixture_nll(hipStream_t s, const float* Y, int ldy, const float* Z, int B, int Bp,
                        float* G, int ldg, float* partial, float* loss);
void launch_grad_prep(hipStream_t s, const float* G, int ldg, int Bp, int width, int n_real,
                      uint16_t* GB, uint16_t* GBT, float* bias_grad);
void launch_adam(hipStream_t s, float* p, float* m1, float* m2, const float* g, int n, float lr,
                 int t);
void launch_refresh_bf16(hipStream_t s, const float* W, int out, int in, int out_p, int in_p,
                         uint16_t* Wb, uint16_t* WbT);
void launch_condition(hipStream_t s, const float* x_init, const float* goal, const float* boxes,
                      const int32_t* n_obs, int q, int max_boxes_in, float* cond);
void launch_sample(hipStream_t s, const float* Y, int ldy, int q, int n, const float* u,
                   const float* eps, float* out);

}  // namespace pump
