// C ABI of the learned sampling proposal (forward, training step, sampling).
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "mlp_internal.hpp"
#include "pump.h"

using namespace pump;

namespace {
const int kInReal[kLayers] = {kIn, kHidden, kHidden, kHidden, kHidden};
const int kInP[kLayers] = {kInPad, kHidden, kHidden, kHidden, kHidden};
const int kOutReal[kLayers] = {kHidden, kHidden, kHidden, kHidden, kOut};
const int kOutP[kLayers] = {kHidden, kHidden, kHidden, kHidden, kOutPad};
}  // namespace

// Staging for pump_mlp_sample_noalloc (draws in host memory): the uniforms,
// the normals and the drawn states pass through this array instead of
// buffers allocated per call.  One copy per GPU, held until the process
// ends: kNoallocFloats floats (8 MiB).  Host code never names the array
// itself: its device address comes from hipGetSymbolAddress, once per device
// (noalloc_staging below), since the host-side symbol is only a stand-in.
constexpr size_t kNoallocFloats = (size_t)2 << 20;
static __device__ __align__(256) float scratch[kNoallocFloats];

struct pump_mlp {
    hipStream_t stream = nullptr;
    int device = 0;                 // the device current at create
    float* staging = nullptr;       // that device's address of `scratch`
    bool own_stream = false;
    int max_batch = 0, maxBp = 0;
    int n_params = 0;
    int off_W[kLayers] = {0}, off_b[kLayers] = {0};
    float *params = nullptr, *m1 = nullptr, *m2 = nullptr, *grads = nullptr;
    uint16_t *Wb[kLayers] = {nullptr}, *WbT[kLayers] = {nullptr};
    uint16_t *H[kLayers] = {nullptr}, *HT[kLayers] = {nullptr};
    float *Y = nullptr, *G = nullptr, *G2 = nullptr;
    uint16_t *GB = nullptr, *GBT = nullptr;
    float *partial = nullptr, *loss = nullptr;
    float *xbuf = nullptr, *zbuf = nullptr, *ubuf = nullptr, *ebuf = nullptr, *obuf = nullptr;
    int t = 0;
    std::string err;
};

namespace {

int mfail(pump_mlp* m, int code, const std::string& msg) {
    if (m) m->err = msg;
    return code;
}

#define MCHK(call)                                                                     \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return mfail(m, PUMP_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

int round32(int b) { return (b + 31) / 32 * 32; }

void refresh_all(pump_mlp* m) {
    for (int l = 0; l < kLayers; ++l)
        launch_refresh_bf16(m->stream, m->params + m->off_W[l], kOutReal[l], kInReal[l], kOutP[l],
                            kInP[l], m->Wb[l], m->WbT[l]);
}

// Y = MLP(cond rows in m->xbuf or `X`), rows padded to Bp.
void forward(pump_mlp* m, const float* X, int B, int Bp) {
    launch_input_bf16(m->stream, X, B, Bp, kIn, kInPad, m->H[0], m->HT[0]);
    for (int l = 0; l < kLayers; ++l) {
        EpiArgs ep;
        memset(&ep, 0, sizeof(ep));
        ep.bias = m->params + m->off_b[l];
        ep.n_real = kOutReal[l];
        if (l < kLayers - 1) {
            ep.out_bf = m->H[l + 1];
            ep.ld_out = kOutP[l];
            ep.out_bfT = m->HT[l + 1];
            ep.ld_outT = Bp;
            launch_gemm_nt(m->stream, kEpiHidden, m->H[l], kInP[l], m->Wb[l], kInP[l], Bp, kOutP[l],
                           kInP[l], ep);
        } else {
            ep.out_f32 = m->Y;
            ep.ld_out = kOutPad;
            launch_gemm_nt(m->stream, kEpiOutput, m->H[l], kInP[l], m->Wb[l], kInP[l], Bp, kOutP[l],
                           kInP[l], ep);
        }
    }
}

// Gradients of the mean NLL into m->grads (and the loss into m->loss).
void backward(pump_mlp* m, const float* Z, int B, int Bp) {
    launch_mixture_nll(m->stream, m->Y, kOutPad, Z, B, Bp, m->G, kOutPad, m->partial, m->loss);
    float* G = m->G;
    float* G2 = m->G2;
    for (int l = kLayers - 1; l >= 0; --l) {
        const int width = kOutP[l];
        launch_grad_prep(m->stream, G, width, Bp, width, kOutReal[l], m->GB, m->GBT,
                         m->grads + m->off_b[l]);
        EpiArgs ep;
        memset(&ep, 0, sizeof(ep));
        ep.m_real = kOutReal[l];
        ep.n_real = kInReal[l];
        ep.out_f32 = m->grads + m->off_W[l];
        ep.ld_out = kInReal[l];
        launch_gemm_nt(m->stream, kEpiWgrad, m->GBT, Bp, m->HT[l], Bp, kOutP[l], kInP[l], Bp, ep);
        if (l > 0) {
            EpiArgs ed;
            memset(&ed, 0, sizeof(ed));
            ed.out_f32 = G2;
            ed.ld_out = kInP[l];
            ed.mask_bf = m->H[l];
            ed.ld_mask = kInP[l];
            launch_gemm_nt(m->stream, kEpiDgrad, m->GB, width, m->WbT[l], kOutP[l], Bp, kInP[l],
                           kOutP[l], ed);
            std::swap(G, G2);
        }
    }
}

// Device address of `scratch` on the current device, looked up on the first
// call per device and kept for the life of the process.
constexpr int kMaxDevices = 64;
std::mutex g_staging_mu;
float* g_staging[kMaxDevices] = {};

hipError_t noalloc_staging(int dev, float** out) {
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_staging_mu);
    if (!g_staging[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_staging[dev] = static_cast<float*>(p);
    }
    *out = g_staging[dev];
    return hipSuccess;
}

const float* stage(pump_mlp* m, const float* src, float* buf, size_t n, int mem, hipError_t* e) {
    *e = hipSuccess;
    if (mem == PUMP_MEM_DEVICE) return src;
    *e = hipMemcpyAsync(buf, src, n * sizeof(float), hipMemcpyHostToDevice, m->stream);
    return buf;
}

}  // namespace

extern "C" {

int pump_mlp_create(int32_t max_batch, void* hip_stream, pump_mlp** out) {
    if (!out) return PUMP_E_ARG;
    *out = nullptr;
    if (max_batch < 1 || max_batch > (1 << 20)) return PUMP_E_ARG;
    pump_mlp* m = new pump_mlp();
    if (hip_stream) {
        m->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreate(&m->stream) != hipSuccess) { delete m; return PUMP_E_HIP; }
        m->own_stream = true;
    }
    m->max_batch = max_batch;
    m->maxBp = round32(max_batch);
    // this device's staging address for pump_mlp_sample_noalloc (the
    // device current now is the one whose memory the context uses)
    if (hipGetDevice(&m->device) != hipSuccess ||
        noalloc_staging(m->device, &m->staging) != hipSuccess) {
        if (m->own_stream) (void)hipStreamDestroy(m->stream);
        delete m;
        return PUMP_E_HIP;
    }
    int off = 0;
    for (int l = 0; l < kLayers; ++l) {
        m->off_W[l] = off;
        off += kOutReal[l] * kInReal[l];
        m->off_b[l] = off;
        off += kOutReal[l];
    }
    m->n_params = off;
    const size_t Bp = (size_t)m->maxBp;
    bool ok = true;
    auto A = [&](hipError_t e) { ok = ok && e == hipSuccess; };
    auto alloc = [&](void** p, size_t bytes) { A(hipMalloc(p, bytes ? bytes : 16)); };
    alloc((void**)&m->params, (size_t)off * 4);
    alloc((void**)&m->m1, (size_t)off * 4);
    alloc((void**)&m->m2, (size_t)off * 4);
    alloc((void**)&m->grads, (size_t)off * 4);
    for (int l = 0; l < kLayers; ++l) {
        alloc((void**)&m->Wb[l], (size_t)kOutP[l] * kInP[l] * 2);
        alloc((void**)&m->WbT[l], (size_t)kOutP[l] * kInP[l] * 2);
        alloc((void**)&m->H[l], Bp * kInP[l] * 2);
        alloc((void**)&m->HT[l], Bp * kInP[l] * 2);
    }
    alloc((void**)&m->Y, Bp * kOutPad * 4);
    alloc((void**)&m->G, Bp * kInPad * 4);
    alloc((void**)&m->G2, Bp * kInPad * 4);
    alloc((void**)&m->GB, Bp * kHidden * 2);
    alloc((void**)&m->GBT, Bp * kHidden * 2);
    alloc((void**)&m->partial, (Bp / 256 + 2) * 4);
    alloc((void**)&m->loss, 16);
    alloc((void**)&m->xbuf, Bp * kIn * 4);
    alloc((void**)&m->zbuf, Bp * kDState * 4);
    alloc((void**)&m->ubuf, Bp * 4);
    alloc((void**)&m->ebuf, Bp * kDState * 4);
    alloc((void**)&m->obuf, Bp * kDState * 4);
    if (!ok) {
        pump_mlp_destroy(m);
        return PUMP_E_HIP;
    }
    *out = m;
    return PUMP_OK;
}

int pump_mlp_destroy(pump_mlp* m) {
    if (!m) return PUMP_OK;
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    void* ptrs[] = {m->params, m->m1, m->m2, m->grads, m->Y, m->G, m->G2, m->GB, m->GBT,
                    m->partial, m->loss, m->xbuf, m->zbuf, m->ubuf, m->ebuf, m->obuf};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    for (int l = 0; l < kLayers; ++l) {
        void* q[] = {m->Wb[l], m->WbT[l], m->H[l], m->HT[l]};
        for (void* p : q)
            if (p) (void)hipFree(p);
    }
    if (m->own_stream && m->stream) (void)hipStreamDestroy(m->stream);
    delete m;
    return PUMP_OK;
}

int pump_mlp_num_params(void) {
    int n = 0;
    for (int l = 0; l < kLayers; ++l) n += kOutReal[l] * kInReal[l] + kOutReal[l];
    return n;
}

int pump_mlp_set_params(pump_mlp* m, const float* params, int64_t n) {
    if (!m || !params) return PUMP_E_ARG;
    if (n != m->n_params) return mfail(m, PUMP_E_ARG, "parameter count mismatch");
    MCHK(hipMemcpyAsync(m->params, params, (size_t)n * 4, hipMemcpyHostToDevice, m->stream));
    MCHK(hipMemsetAsync(m->m1, 0, (size_t)n * 4, m->stream));
    MCHK(hipMemsetAsync(m->m2, 0, (size_t)n * 4, m->stream));
    refresh_all(m);
    m->t = 0;
    MCHK(hipStreamSynchronize(m->stream));
    return PUMP_OK;
}

int pump_mlp_get_params(pump_mlp* m, float* params, int64_t n) {
    if (!m || !params) return PUMP_E_ARG;
    if (n != m->n_params) return mfail(m, PUMP_E_ARG, "parameter count mismatch");
    MCHK(hipMemcpyAsync(params, m->params, (size_t)n * 4, hipMemcpyDeviceToHost, m->stream));
    MCHK(hipStreamSynchronize(m->stream));
    return PUMP_OK;
}

int pump_mlp_get_state(pump_mlp* m, float* params, float* m1, float* m2, int64_t n, int32_t* t) {
    if (!m || !params || !m1 || !m2 || !t) return PUMP_E_ARG;
    if (n != m->n_params) return mfail(m, PUMP_E_ARG, "parameter count mismatch");
    MCHK(hipMemcpyAsync(params, m->params, (size_t)n * 4, hipMemcpyDeviceToHost, m->stream));
    MCHK(hipMemcpyAsync(m1, m->m1, (size_t)n * 4, hipMemcpyDeviceToHost, m->stream));
    MCHK(hipMemcpyAsync(m2, m->m2, (size_t)n * 4, hipMemcpyDeviceToHost, m->stream));
    MCHK(hipStreamSynchronize(m->stream));
    *t = m->t;
    return PUMP_OK;
}

int pump_mlp_set_state(pump_mlp* m, const float* params, const float* m1, const float* m2,
                       int64_t n, int32_t t) {
    if (!m || !params || !m1 || !m2) return PUMP_E_ARG;
    if (n != m->n_params) return mfail(m, PUMP_E_ARG, "parameter count mismatch");
    if (t < 0) return mfail(m, PUMP_E_ARG, "negative step count");
    MCHK(hipMemcpyAsync(m->params, params, (size_t)n * 4, hipMemcpyHostToDevice, m->stream));
    MCHK(hipMemcpyAsync(m->m1, m1, (size_t)n * 4, hipMemcpyHostToDevice, m->stream));
    MCHK(hipMemcpyAsync(m->m2, m2, (size_t)n * 4, hipMemcpyHostToDevice, m->stream));
    refresh_all(m);
    m->t = t;
    MCHK(hipStreamSynchronize(m->stream));
    return PUMP_OK;
}

int pump_mlp_adam_step(pump_mlp* m, const float* grads, int64_t n, float lr, int32_t mem) {
    if (!m || !grads) return PUMP_E_ARG;
    if (n != m->n_params) return mfail(m, PUMP_E_ARG, "parameter count mismatch");
    if (!(lr > 0.0f)) return mfail(m, PUMP_E_ARG, "learning rate must be positive");
    if (mem == PUMP_MEM_DEVICE) {
        MCHK(hipMemcpyAsync(m->grads, grads, (size_t)n * 4, hipMemcpyDeviceToDevice, m->stream));
    } else {
        MCHK(hipMemcpyAsync(m->grads, grads, (size_t)n * 4, hipMemcpyHostToDevice, m->stream));
    }
    m->t += 1;
    launch_adam(m->stream, m->params, m->m1, m->m2, m->grads, m->n_params, lr, m->t);
    refresh_all(m);
    MCHK(hipStreamSynchronize(m->stream));
    MCHK(hipGetLastError());
    return PUMP_OK;
}

int pump_mlp_forward(pump_mlp* m, const float* cond, int32_t B, float* out, int32_t mem) {
    if (!m || !cond || !out) return PUMP_E_ARG;
    if (B < 1 || B > m->max_batch) return mfail(m, PUMP_E_ARG, "batch out of range");
    hipError_t e;
    const float* X = stage(m, cond, m->xbuf, (size_t)B * kIn, mem, &e);
    MCHK(e);
    forward(m, X, B, round32(B));
    MCHK(hipMemcpy2DAsync(out, kOut * 4, m->Y, kOutPad * 4, kOut * 4, B,
                          mem == PUMP_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                          m->stream));
    MCHK(hipStreamSynchronize(m->stream));
    MCHK(hipGetLastError());
    return PUMP_OK;
}

int pump_mlp_loss_grad(pump_mlp* m, const float* cond, const float* target, int32_t B,
                       float* loss, float* grads, int32_t mem) {
    if (!m || !cond || !target) return PUMP_E_ARG;
    if (B < 1 || B > m->max_batch) return mfail(m, PUMP_E_ARG, "batch out of range");
    hipError_t e;
    const float* X = stage(m, cond, m->xbuf, (size_t)B * kIn, mem, &e);
    MCHK(e);
    const float* Z = stage(m, target, m->zbuf, (size_t)B * kDState, mem, &e);
    MCHK(e);
    const int Bp = round32(B);
    forward(m, X, B, Bp);
    backward(m, Z, B, Bp);
    if (loss) MCHK(hipMemcpyAsync(loss, m->loss, 4, hipMemcpyDeviceToHost, m->stream));
    if (grads)
        MCHK(hipMemcpyAsync(grads, m->grads, (size_t)m->n_params * 4,
                            mem == PUMP_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                            m->stream));
    MCHK(hipStreamSynchronize(m->stream));
    MCHK(hipGetLastError());
    return PUMP_OK;
}

int pump_mlp_train_step(pump_mlp* m, const float* cond, const float* target, int32_t B, float lr,
                        float* loss, int32_t mem) {
    if (!m || !cond || !target) return PUMP_E_ARG;
    if (B < 1 || B > m->max_batch) return mfail(m, PUMP_E_ARG, "batch out of range");
    if (!(lr > 0.0f)) return mfail(m, PUMP_E_ARG, "learning rate must be positive");
    hipError_t e;
    const float* X = stage(m, cond, m->xbuf, (size_t)B * kIn, mem, &e);
    MCHK(e);
    const float* Z = stage(m, target, m->zbuf, (size_t)B * kDState, mem, &e);
    MCHK(e);
    const int Bp = round32(B);
    forward(m, X, B, Bp);
    backward(m, Z, B, Bp);
    m->t += 1;
    launch_adam(m->stream, m->params, m->m1, m->m2, m->grads, m->n_params, lr, m->t);
    refresh_all(m);
    if (loss) {
        MCHK(hipMemcpyAsync(loss, m->loss, 4, hipMemcpyDeviceToHost, m->stream));
        MCHK(hipStreamSynchronize(m->stream));
    }
    MCHK(hipGetLastError());
    return PUMP_OK;
}

int pump_mlp_condition(pump_mlp* m, const float* x_init, const float* goal, const float* boxes,
                       const int32_t* n_obs, int32_t q, int32_t max_boxes_in, float* cond) {
    if (!m || !x_init || !goal || !boxes || !n_obs || !cond) return PUMP_E_ARG;
    if (q < 1 || max_boxes_in < 1) return mfail(m, PUMP_E_ARG, "bad sizes");
    launch_condition(m->stream, x_init, goal, boxes, n_obs, q, max_boxes_in, cond);
    MCHK(hipStreamSynchronize(m->stream));
    MCHK(hipGetLastError());
    return PUMP_OK;
}

int pump_mlp_sample(pump_mlp* m, const float* cond, int32_t q, const float* u, const float* eps,
                    int32_t n, float* out, int32_t mem) {
    if (!m || !cond || !u || !eps || !out) return PUMP_E_ARG;
    if (q < 1 || q > m->max_batch || n < 1) return mfail(m, PUMP_E_ARG, "bad sizes");
    hipError_t e;
    const float* X = stage(m, cond, m->xbuf, (size_t)q * kIn, mem, &e);
    MCHK(e);
    forward(m, X, q, round32(q));
    const float* U = u;
    const float* EPS = eps;
    float* O = out;
    std::vector<float> dummy;
    float *du = nullptr, *de = nullptr, *dout = nullptr;
    if (mem != PUMP_MEM_DEVICE) {
        const size_t total = (size_t)q * n;
        MCHK(hipMalloc((void**)&du, total * 4));
        MCHK(hipMalloc((void**)&de, total * kDState * 4));
        MCHK(hipMalloc((void**)&dout, total * kDState * 4));
        MCHK(hipMemcpyAsync(du, u, total * 4, hipMemcpyHostToDevice, m->stream));
        MCHK(hipMemcpyAsync(de, eps, total * kDState * 4, hipMemcpyHostToDevice, m->stream));
        U = du;
        EPS = de;
        O = dout;
    }
    launch_sample(m->stream, m->Y, kOutPad, q, n, U, EPS, O);
    if (mem != PUMP_MEM_DEVICE) {
        const size_t total = (size_t)q * n;
        MCHK(hipMemcpyAsync(out, dout, total * kDState * 4, hipMemcpyDeviceToHost, m->stream));
    }
    MCHK(hipStreamSynchronize(m->stream));
    if (du) (void)hipFree(du);
    if (de) (void)hipFree(de);
    if (dout) (void)hipFree(dout);
    MCHK(hipGetLastError());
    return PUMP_OK;
}

int pump_mlp_sample_noalloc(pump_mlp* m, const float* cond, int32_t q, const float* u,
                            const float* eps, int32_t n, float* out, int32_t mem) {
    if (!m || !cond || !u || !eps || !out) return PUMP_E_ARG;
    if (q < 1 || q > m->max_batch || n < 1) return mfail(m, PUMP_E_ARG, "bad sizes");
    const size_t total = (size_t)q * (size_t)n;
    if (mem != PUMP_MEM_DEVICE && total * (1 + 2 * kDState) > kNoallocFloats)
        return mfail(m, PUMP_E_CAPACITY,
                     "q * n = " + std::to_string(total) + " draws exceed the no-alloc staging (" +
                         std::to_string(kNoallocFloats / (1 + 2 * kDState)) + " draws)");
    if (!m->staging) return mfail(m, PUMP_E_STATE, "no staging address for this device");
    hipError_t e;
    const float* X = stage(m, cond, m->xbuf, (size_t)q * kIn, mem, &e);
    MCHK(e);
    forward(m, X, q, round32(q));
    const float* U = u;
    const float* EPS = eps;
    float* O = out;
    if (mem != PUMP_MEM_DEVICE) {
        // the uniforms, the normals and the draws in the staging array:
        // every word the kernel reads is copied in first, every word it
        // writes is copied out, so nothing needs clearing
        float* su = m->staging;
        float* se = su + total;
        float* so = se + total * kDState;
        MCHK(hipMemcpyAsync(su, u, total * 4, hipMemcpyHostToDevice, m->stream));
        MCHK(hipMemcpyAsync(se, eps, total * kDState * 4, hipMemcpyHostToDevice, m->stream));
        U = su;
        EPS = se;
        O = so;
    }
    launch_sample(m->stream, m->Y, kOutPad, q, n, U, EPS, O);
    if (mem != PUMP_MEM_DEVICE)
        MCHK(hipMemcpyAsync(out, O, total * kDState * 4, hipMemcpyDeviceToHost, m->stream));
    MCHK(hipStreamSynchronize(m->stream));
    MCHK(hipGetLastError());
    return PUMP_OK;
}

const char* pump_mlp_last_error(const pump_mlp* m) { return m ? m->err.c_str() : ""; }

}  // extern "C"
