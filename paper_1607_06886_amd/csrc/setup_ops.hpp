// Per-query setup operations: the particle deviation table and BuildGraph
// (Alg. 3), shared by the single-query kernels and the batched engine.
#pragma once

#include "device_math.hpp"
#include "pump_internal.hpp"

namespace pump {


// ---------------------------------------------------------------------------
// Particle deviation table (Sec. III-B particles; eq. (2) closed loop).
// Per (axis a, particle j) the recurrence
//   dx_{s+1} = A_cl dx_s + L (xi[s][2a][j], xi[s][2a+1][j])^T,  dx_0 = 0
// runs in FP64 and the position part D[s][a][j] is stored in FP32.  The
// steps are cut into chunks of kDevChunk so that many lanes work at once:
// (1) every (chunk, a, j) runs its chunk from a zero state, giving the
// chunk's own response E_k; (2) every (a, j) chains the chunk start states,
// X_{k+1} = A_cl^C X_k + E_k; (3) every (chunk, a, j) reruns its chunk from
// X_k and stores D.  The state at a chunk start differs from the sequential
// recurrence only by FP64 rounding.
// Scratch: E and X0, each [K][3][N] double2 with K = ceil(S / kDevChunk).
// ---------------------------------------------------------------------------
constexpr int kDevChunk = 16;

struct DevCoef {
    double a00, a01, a10, a11, l00, l10, l11;
};

__device__ __forceinline__ void dev_run_chunk(const float* __restrict__ noise, int N, int S, int a,
                                              int j, int k, const DevCoef& m, double& p,
                                              double& v, float* __restrict__ D) {
    const int s0 = k * kDevChunk;
    float w0[kDevChunk], w1[kDevChunk];
#pragma unroll
    for (int u = 0; u < kDevChunk; ++u) {
        const int s = s0 + u < S ? s0 + u : S - 1;
        w0[u] = noise[((size_t)s * 6 + 2 * a) * N + j];
        w1[u] = noise[((size_t)s * 6 + 2 * a + 1) * N + j];
    }
#pragma unroll
    for (int u = 0; u < kDevChunk; ++u) {
        if (s0 + u >= S) break;
        const double pn = m.a00 * p + m.a01 * v + m.l00 * (double)w0[u];
        const double vn = m.a10 * p + m.a11 * v + (m.l10 * (double)w0[u] + m.l11 * (double)w1[u]);
        p = pn;
        v = vn;
        if (D) D[((size_t)(s0 + u + 1) * 3 + a) * N + j] = (float)p;
    }
}

// (1) chunk responses; thread t = (k * 3 + a) * N + j
__device__ __forceinline__ void dev_local_dev(const float* __restrict__ noise, double* __restrict__ E,
                                              int N, int S, const DevCoef& m) {
    const int K = (S + kDevChunk - 1) / kDevChunk;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= K * 3 * N) return;
    const int j = t % N, a = (t / N) % 3, k = t / (3 * N);
    double p = 0.0, v = 0.0;
    dev_run_chunk(noise, N, S, a, j, k, m, p, v, nullptr);
    E[2 * (size_t)t] = p;
    E[2 * (size_t)t + 1] = v;
}

// (2) chunk start states; thread col = a * N + j
__device__ __forceinline__ void dev_carry_dev(const double* __restrict__ E, double* __restrict__ X0,
                                              int N, int S, const DevCoef& m) {
    const int K = (S + kDevChunk - 1) / kDevChunk;
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= 3 * N) return;
    // Phi = A_cl^C
    double f00 = 1.0, f01 = 0.0, f10 = 0.0, f11 = 1.0;
    for (int u = 0; u < kDevChunk; ++u) {
        const double g00 = m.a00 * f00 + m.a01 * f10, g01 = m.a00 * f01 + m.a01 * f11;
        const double g10 = m.a10 * f00 + m.a11 * f10, g11 = m.a10 * f01 + m.a11 * f11;
        f00 = g00; f01 = g01; f10 = g10; f11 = g11;
    }
    double p = 0.0, v = 0.0;
    for (int k = 0; k < K; ++k) {
        const size_t t = (size_t)k * 3 * N + col;
        X0[2 * t] = p;
        X0[2 * t + 1] = v;
        const double pn = f00 * p + f01 * v + E[2 * t];
        const double vn = f10 * p + f11 * v + E[2 * t + 1];
        p = pn;
        v = vn;
    }
}

// (3) the table; thread t = (k * 3 + a) * N + j
__device__ __forceinline__ void dev_final_dev(const float* __restrict__ noise, const double* __restrict__ X0,
                                              float* __restrict__ D, int N, int S, const DevCoef& m) {
    const int K = (S + kDevChunk - 1) / kDevChunk;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= K * 3 * N) return;
    const int j = t % N, a = (t / N) % 3, k = t / (3 * N);
    if (k == 0) D[(size_t)a * N + j] = 0.0f;
    double p = X0[2 * (size_t)t], v = X0[2 * (size_t)t + 1];
    dev_run_chunk(noise, N, S, a, j, k, m, p, v, D);
}

// ---------------------------------------------------------------------------
// The deviation table under LQG tracking.  Per (axis a, particle j) the
// joint state z = (dp, dv, p_hat, v_hat) follows z' = m z + e xi with
// xi = (noise[s][2a][j], noise[s][2a+1][j], noise_meas[s][a][j]), z_0 = 0;
// D stores dp.  Same three chunked passes as above with a 4-state carry
// (Phi = m^C).  Scratch: E and X0, each [K][3][N] of 4 doubles.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void lqg_run_chunk(const float* __restrict__ noise,
                                              const float* __restrict__ meas, int N, int S, int a,
                                              int j, int k, const LqgCoef& q, double z[4],
                                              float* __restrict__ D) {
    const int s0 = k * kDevChunk;
    float w0[kDevChunk], w1[kDevChunk], w2[kDevChunk];
#pragma unroll
    for (int u = 0; u < kDevChunk; ++u) {
        const int s = s0 + u < S ? s0 + u : S - 1;
        w0[u] = noise[((size_t)s * 6 + 2 * a) * N + j];
        w1[u] = noise[((size_t)s * 6 + 2 * a + 1) * N + j];
        w2[u] = meas[((size_t)s * 3 + a) * N + j];
    }
#pragma unroll
    for (int u = 0; u < kDevChunk; ++u) {
        if (s0 + u >= S) break;
        lqg_step(q, z, (double)w0[u], (double)w1[u], (double)w2[u]);
        if (D) D[((size_t)(s0 + u + 1) * 3 + a) * N + j] = (float)z[0];
    }
}

// (1) chunk responses; thread t = (k * 3 + a) * N + j
__device__ __forceinline__ void lqg_local_dev(const float* __restrict__ noise,
                                              const float* __restrict__ meas,
                                              double* __restrict__ E, int N, int S,
                                              const LqgCoef& q) {
    const int K = (S + kDevChunk - 1) / kDevChunk;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= K * 3 * N) return;
    const int j = t % N, a = (t / N) % 3, k = t / (3 * N);
    double z[4] = {0.0, 0.0, 0.0, 0.0};
    lqg_run_chunk(noise, meas, N, S, a, j, k, q, z, nullptr);
#pragma unroll
    for (int i = 0; i < 4; ++i) E[4 * (size_t)t + i] = z[i];
}

// (2) chunk start states; thread col = a * N + j
__device__ __forceinline__ void lqg_carry_dev(const double* __restrict__ E,
                                              double* __restrict__ X0, int N, int S,
                                              const LqgCoef& q) {
    const int K = (S + kDevChunk - 1) / kDevChunk;
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= 3 * N) return;
    double f[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) f[i] = (i % 5 == 0) ? 1.0 : 0.0;
    for (int u = 0; u < kDevChunk; ++u) {
        double g[16];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                g[4 * i + c] = q.m[4 * i] * f[c] + q.m[4 * i + 1] * f[4 + c] +
                               q.m[4 * i + 2] * f[8 + c] + q.m[4 * i + 3] * f[12 + c];
#pragma unroll
        for (int i = 0; i < 16; ++i) f[i] = g[i];
    }
    double z[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < K; ++k) {
        const size_t t = (size_t)k * 3 * N + col;
        double zn[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            X0[4 * t + i] = z[i];
            zn[i] = f[4 * i] * z[0] + f[4 * i + 1] * z[1] + f[4 * i + 2] * z[2] +
                    f[4 * i + 3] * z[3] + E[4 * t + i];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) z[i] = zn[i];
    }
}

// (3) the table; thread t = (k * 3 + a) * N + j
__device__ __forceinline__ void lqg_final_dev(const float* __restrict__ noise,
                                              const float* __restrict__ meas,
                                              const double* __restrict__ X0,
                                              float* __restrict__ D, int N, int S,
                                              const LqgCoef& q) {
    const int K = (S + kDevChunk - 1) / kDevChunk;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= K * 3 * N) return;
    const int j = t % N, a = (t / N) % 3, k = t / (3 * N);
    if (k == 0) D[(size_t)a * N + j] = 0.0f;
    double z[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) z[i] = X0[4 * (size_t)t + i];
    lqg_run_chunk(noise, meas, N, S, a, j, k, q, z, D);
}

// Bounding box of the particle cloud at each step: cloud[s] = (min_j D[s][a][j], max_j ...).
__device__ __forceinline__ void cloud_dev(const float* __restrict__ D, float* __restrict__ cloud, int N) {
    __shared__ float smin[3][256], smax[3][256];
    int s = blockIdx.x, t = threadIdx.x;
    for (int a = 0; a < 3; ++a) {
        float mn = INFINITY, mx = -INFINITY;
        for (int j = t; j < N; j += blockDim.x) {
            float d = D[((size_t)s * 3 + a) * N + j];
            mn = fminf(mn, d);
            mx = fmaxf(mx, d);
        }
        smin[a][t] = mn;
        smax[a][t] = mx;
    }
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (t < w)
            for (int a = 0; a < 3; ++a) {
                smin[a][t] = fminf(smin[a][t], smin[a][t + w]);
                smax[a][t] = fmaxf(smax[a][t], smax[a][t + w]);
            }
        __syncthreads();
    }
    if (t < 3) {
        cloud[(size_t)s * 6 + t] = smin[t][0];
        cloud[(size_t)s * 6 + 3 + t] = smax[t][0];
    }
}

__device__ __forceinline__ void gcloud_dev(const float* __restrict__ cloud, float* __restrict__ g, int S1) {
    __shared__ float sm[6][256];
    const int t = threadIdx.x;
    float v[6];
    for (int k = 0; k < 6; ++k) v[k] = k < 3 ? INFINITY : -INFINITY;
    for (int s = t; s < S1; s += blockDim.x)
        for (int k = 0; k < 6; ++k) {
            float c = cloud[(size_t)s * 6 + k];
            v[k] = k < 3 ? fminf(v[k], c) : fmaxf(v[k], c);
        }
    for (int k = 0; k < 6; ++k) sm[k][t] = v[k];
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (t < w)
            for (int k = 0; k < 6; ++k)
                sm[k][t] = k < 3 ? fminf(sm[k][t], sm[k][t + w]) : fmaxf(sm[k][t], sm[k][t + w]);
        __syncthreads();
    }
    if (t < 6) g[t] = sm[t][0];
}

// ---------------------------------------------------------------------------
// Node validity (sample not in a closed obstacle box) and goal membership
// (position in the closed goal box).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void mark_valid_dev(const float* __restrict__ X, int n, const float* __restrict__ obs,
                             int n_obs, float g0, float g1, float g2, float g3, float g4, float g5,
                             uint8_t* __restrict__ valid, uint8_t* __restrict__ goal,
                             int32_t* __restrict__ bad) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n_obs) {
        // obstacle sanity: finite, ordered, inside [-16, 16]
        const float* b = obs + (size_t)v * 6;
        bool okb = true;
        for (int k = 0; k < 3; ++k)
            okb &= (b[k] <= b[3 + k]) & (fabsf(b[k]) <= 16.0f) & (fabsf(b[3 + k]) <= 16.0f);
        if (!okb) atomicOr(bad, 1);
    }
    if (v >= n) return;
    float p0 = X[(size_t)v * 6], p1 = X[(size_t)v * 6 + 1], p2 = X[(size_t)v * 6 + 2];
    if (!(fabsf(p0) <= 16.0f && fabsf(p1) <= 16.0f && fabsf(p2) <= 16.0f)) atomicOr(bad, 1);
    bool in = false;
    for (int o = 0; o < n_obs; ++o) {
        const float* b = obs + (size_t)o * 6;
        in |= (p0 >= b[0]) & (p0 <= b[3]) & (p1 >= b[1]) & (p1 <= b[4]) & (p2 >= b[2]) & (p2 <= b[5]);
    }
    if (v == 0 && in) atomicOr(bad, 2);
    valid[v] = in ? 0 : 1;
    bool g = (p0 >= g0) & (p0 <= g3) & (p1 >= g1) & (p1 <= g4) & (p2 >= g2) & (p2 <= g5);
    goal[v] = (!in && g) ? 1 : 0;
}

// ---------------------------------------------------------------------------
// BuildGraph (Alg. 3).  Edge v -> u iff both nodes are valid, u != v,
// c*(v,u) < r_n, tau* > 1e-6 and the nominal trajectory meets no obstacle
// (continuous, exact; closed boxes).  Pass 1 evaluates every ordered pair and
// records the result as a bit matrix and per-row counts; after a scan of the
// counts, pass 2 writes each row's neighbours in ascending order with their
// (tau*, c*).
// ---------------------------------------------------------------------------
// One block (256 threads) per source row v.  The row is scanned in chunks of
// 4096 targets: every thread applies the exact rejection test to 16 targets
// and appends the survivors to a list in LDS.  The survivors are then steered
// densely (one per thread); a near pair whose trajectory's bounding box meets
// some obstacle boxes contributes one (pair, box) entry per such box to an
// LDS queue, and the queue is processed densely too (one exact trajectory-box
// test per thread), so lanes do not idle while a few pairs test many boxes.
// Bits of edges are set in the row's LDS bitmask, which is written out with
// the row's degree at the end.
constexpr int kMarkChunk = 4096;
constexpr int kMarkQueue = 2048;

__device__ __forceinline__ void graph_mark_dev(const float* __restrict__ X,
                                                    const uint8_t* __restrict__ valid, int n,
                                                    const float* __restrict__ obs, int n_obs,
                                                    double r_steer, double r_conn,
                                                    uint32_t* __restrict__ ebits,
                                                    int32_t* __restrict__ deg, int words) {
    __shared__ float s_obs[kMaxObs * 6];
    __shared__ int s_list[kMarkChunk];
    __shared__ double s_tau[256];
    __shared__ int s_blk[256];
    __shared__ uint32_t s_q[kMarkQueue];
    __shared__ int s_w[4];
    __shared__ int s_cnt;
    extern __shared__ uint32_t s_row[];          // words u32
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int t = tid; t < n_obs * 6; t += blockDim.x) s_obs[t] = obs[t];
    for (int t = tid; t < words; t += blockDim.x) s_row[t] = 0u;
    const int v = blockIdx.x;
    float xv[6];
    for (int k = 0; k < 6; ++k) xv[k] = X[(size_t)v * 6 + k];
    const bool vv = valid[v] != 0;
    __syncthreads();
    if (vv) {
        for (int c0 = 0; c0 < n; c0 += kMarkChunk) {
            if (tid == 0) s_cnt = 0;
            __syncthreads();
            for (int u = c0 + tid; u < c0 + kMarkChunk && u < n; u += blockDim.x) {
                if (u == v || !valid[u]) continue;
                float xu[6];
                for (int k = 0; k < 6; ++k) xu[k] = X[(size_t)u * 6 + k];
                if (!surely_not_near(boundary_sums(xv, xu), r_steer, r_conn))
                    s_list[atomicAdd(&s_cnt, 1)] = u;
            }
            __syncthreads();
            const int cnt = s_cnt;
            for (int base = 0; base < cnt; base += 256) {
                const int i = base + tid;
                int u = -1;
                bool near = false;
                double tau = 0.0;
                unsigned long long ov[kMaxObs / 64] = {0ull, 0ull, 0ull, 0ull};
                int n_ov = 0;
                if (i < cnt) {
                    u = s_list[i];
                    float xu[6];
                    for (int k = 0; k < 6; ++k) xu[k] = X[(size_t)u * 6 + k];
                    double c;
                    steer64(xv, xu, r_steer, tau, c);
                    near = c < r_conn && tau > kTauMin;
                    if (near && n_obs > 0) {
                        Cubic cs[3];
                        hermite(xv, xu, tau, cs);
                        double mn[3], mx[3];
                        for (int a = 0; a < 3; ++a) cubic_range(cs[a], tau, mn[a], mx[a]);
                        for (int o = 0; o < n_obs; ++o) {
                            const float* bx = s_obs + o * 6;
                            bool disjoint = false;
                            for (int a = 0; a < 3; ++a)
                                disjoint |= (mx[a] < (double)bx[a]) | (mn[a] > (double)bx[3 + a]);
                            if (!disjoint) {
                                ov[o >> 6] |= 1ull << (o & 63);
                                ++n_ov;
                            }
                        }
                    }
                }
                s_tau[tid] = tau;
                s_blk[tid] = 0;
                // exclusive scan of the per-thread test counts
                int x = n_ov;
                for (int o = 1; o < 64; o <<= 1) {
                    const int y = __shfl_up(x, o, 64);
                    if (lane >= o) x += y;
                }
                if (lane == 63) s_w[wave] = x;
                __syncthreads();
                int off = x - n_ov, total = 0;
                for (int w = 0; w < 4; ++w) {
                    if (w < wave) off += s_w[w];
                    total += s_w[w];
                }
                for (int seg = 0; seg < total; seg += kMarkQueue) {
                    if (n_ov > 0 && off < seg + kMarkQueue && off + n_ov > seg) {
                        int k = off;
                        for (int wd = 0; wd < kMaxObs / 64; ++wd) {
                            unsigned long long m = ov[wd];
                            while (m) {
                                const int o = wd * 64 + __ffsll((long long)m) - 1;
                                m &= m - 1ull;
                                if (k >= seg && k < seg + kMarkQueue)
                                    s_q[k - seg] = ((uint32_t)tid << 8) | (uint32_t)o;
                                ++k;
                            }
                        }
                    }
                    __syncthreads();
                    const int m = total - seg < kMarkQueue ? total - seg : kMarkQueue;
                    for (int e = tid; e < m; e += blockDim.x) {
                        const uint32_t ent = s_q[e];
                        const int slot = (int)(ent >> 8), o = (int)(ent & 255u);
                        if (s_blk[slot]) continue;   // already known to collide
                        const int uu = s_list[base + slot];
                        float xu[6];
                        for (int k = 0; k < 6; ++k) xu[k] = X[(size_t)uu * 6 + k];
                        Cubic cs[3];
                        const double tt = s_tau[slot];
                        hermite(xv, xu, tt, cs);
                        if (trajectory_hits_box(cs, tt, s_obs + o * 6)) s_blk[slot] = 1;
                    }
                    __syncthreads();
                }
                if (near && !s_blk[tid]) atomicOr(&s_row[u >> 5], 1u << (u & 31));
                __syncthreads();
            }
        }
    }
    int d = 0;
    for (int t = tid; t < words; t += blockDim.x) {
        const uint32_t w = s_row[t];
        ebits[(size_t)v * words + t] = w;
        d += __popc(w);
    }
    // block sum of the degree
    for (int o = 32; o > 0; o >>= 1) d += __shfl_down(d, o, 64);
    __shared__ int s_deg[4];
    if ((tid & 63) == 0) s_deg[tid >> 6] = d;
    __syncthreads();
    if (tid == 0) deg[v] = s_deg[0] + s_deg[1] + s_deg[2] + s_deg[3];
}

__device__ __forceinline__ void graph_fill_dev(int n, const uint32_t* __restrict__ ebits,
                                                    const int32_t* __restrict__ row_ptr,
                                                    int32_t* __restrict__ col,
                                                    int32_t* __restrict__ esrc, int words) {
    const int v = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (v >= n) return;
    int pos = row_ptr[v];
    for (int base = 0; base < n; base += 64) {
        uint32_t w = ebits[(size_t)v * words + base / 32 + (lane >> 5)];
        bool e = (w >> (lane & 31)) & 1u;
        unsigned long long b = __ballot(e);
        if (e) {
            unsigned long long below = lane ? (b & ((1ull << lane) - 1ull)) : 0ull;
            int at = pos + (int)__popcll(below);
            col[at] = base + lane;
            esrc[at] = v;
        }
        pos += (int)__popcll(b);
    }
}

// Edge controls, one lane per edge: the same FP64 steering as pass 1, so the
// cached (tau*, c*) are bit-identical to the values that admitted the edge.
__device__ __forceinline__ void edge_steer_dev(const float* __restrict__ X, int n,
                                                    double r_steer,
                                                    const int32_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ col,
                                                    const int32_t* __restrict__ esrc,
                                                    double* __restrict__ etau,
                                                    double* __restrict__ ecost) {
    const int E = row_ptr[n];
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < E; e += gridDim.x * blockDim.x) {
        const float* xv = X + (size_t)esrc[e] * 6;
        const float* xu = X + (size_t)col[e] * 6;
        double tau, c;
        steer64(xv, xu, r_steer, tau, c);
        etau[e] = tau;
        ecost[e] = c;
    }
}


}  // namespace pump
