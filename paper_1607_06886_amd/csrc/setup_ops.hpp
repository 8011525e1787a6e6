// Per-query setup operations: the particle deviation table and BuildGraph
// (Alg. 3), shared by the single-query kernels and the batched engine.
#pragma once

#include "box_bins.hpp"
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
// (continuous, exact; closed boxes).  The result is a bit matrix (row v,
// bit u) and per-row counts; after a scan of the counts, pass 2 writes each
// row's neighbours in ascending order with their (tau*, c*).
//
// Pass 1 runs as stages, each its own kernel so that the register-heavy
// exact box test does not hold down the occupancy of the others:
//   near    one workgroup per row: every target through the exact Near
//           rejection test into an LDS list, then the survivors steered
//           densely (tau*, c*); near connections -> the near list;
//   boxes   per near connection, its nominal position range against every
//           box and, where they meet, the quick trajectory-box test; a hit
//           blocks it, an unsure case goes to the exact queue; connections
//           not blocked set their bit;
//   exact   per queued (connection, box), one wave: the piecewise test with
//           64 pieces across the lanes and, if still unsure, the exact
//           trajectory-box test; a hit clears the bit;
//   degree  popcount of each row.
// A connection's bit ends set iff no box blocks it, the decision of the exact
// test on every box its range meets.
// ---------------------------------------------------------------------------
constexpr int kNearChunk = 4096;   // targets per LDS survivor list
// workgroup of the near stage: 256 threads let five workgroups share a CU
// (registers and the 32 KB of lists); on the 20,000-sample indoor query this
// measured faster than 128, 512 or 1024 threads and than 2048- or
// 8192-target chunks
constexpr int kNearThreads = 256;

// Append `ok` items of a wave to a list: one atomic per wave (all 64 lanes
// call it).  Returns the slot of this lane's item.
__device__ __forceinline__ int wave_append(bool ok, int32_t* counter) {
    const unsigned long long m = __ballot(ok);
    const int lane = threadIdx.x & 63;
    int base = 0;
    if (lane == 0 && m) base = atomicAdd(counter, (int)__popcll(m));
    base = __shfl(base, 0, 64);
    return base + (int)__popcll(m & (lane ? ((1ull << lane) - 1ull) : 0ull));
}

__device__ __forceinline__ void gw_push_near(const GraphWork& gw, bool ok, int src, int dst,
                                             double tau) {
    const int slot = wave_append(ok, gw.counts + 0);
    if (ok && slot < gw.near_cap) {
        gw.near_src[slot] = src;
        gw.near_dst[slot] = dst;
        gw.near_tau[slot] = tau;
    }
}

// The same for a whole workgroup (all threads call it): one global atomic
// per workgroup and call, since every near connection of every row bumps the
// same counter.  s_w: [blockDim.x / 64 + 1] ints of LDS.
__device__ __forceinline__ void gw_push_near_block(const GraphWork& gw, bool ok, int src, int dst,
                                                   double tau, int* s_w) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const unsigned long long m = __ballot(ok);
    if (lane == 0) s_w[w] = (int)__popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int k = 0; k < nw; ++k) {
            const int c = s_w[k];
            s_w[k] = tot;
            tot += c;
        }
        s_w[nw] = tot ? atomicAdd(gw.counts + 0, tot) : 0;
    }
    __syncthreads();
    const int slot = s_w[nw] + s_w[w] + (int)__popcll(m & (lane ? ((1ull << lane) - 1ull) : 0ull));
    if (ok && slot < gw.near_cap) {
        gw.near_src[slot] = src;
        gw.near_dst[slot] = dst;
        gw.near_tau[slot] = tau;
    }
    __syncthreads();   // s_w is reused
}

// near: row v (whole workgroup, blockDim a multiple of 64, at most 1024;
// s_list holds 2 * kNearChunk ints, s_cnt 3 + 17).  Per chunk of targets,
// three passes, each over a list compacted by the one before it so that no
// wave carries lanes the pass has no work for (a few per cent of the targets
// pass the FP32 bound, so a wave of 64 targets taken in place would nearly
// always run the FP64 test, and the root solve, for one or two lanes):
//   1. the FP32 first look at the Bernstein bound over every target;
//   2. the FP64 rejection test over the targets it could not settle;
//   3. the root solve (tau*, c*) over the targets that test keeps, those
//      whose solve takes steer64's one-root branch listed first and the
//      others from the end of the list, so that a wave runs one branch.
__device__ __forceinline__ void gw_near_row(const float* __restrict__ X,
                                            const uint8_t* __restrict__ valid, int n, int v,
                                            double r_steer, double r_conn, const GraphWork& gw,
                                            int* s_list, int* s_cnt) {
    if (!valid[v]) return;
    int* s_l1 = s_list;                 // pass 1 -> 2
    int* s_l2 = s_list + kNearChunk;    // pass 2 -> 3
    float xv[6];
    for (int k = 0; k < 6; ++k) xv[k] = X[(size_t)v * 6 + k];
    const float r32 = (float)r_steer, R32 = (float)r_conn;
    for (int c0 = 0; c0 < n; c0 += kNearChunk) {
        if (threadIdx.x == 0) {
            s_cnt[0] = 0;
            s_cnt[1] = 0;
            s_cnt[2] = 0;
        }
        __syncthreads();
        for (int u = c0 + threadIdx.x; u < c0 + kNearChunk && u < n; u += blockDim.x) {
            if (u == v || !valid[u]) continue;
            const float2* xu2 = reinterpret_cast<const float2*>(X + (size_t)u * 6);
            const float2 p01 = xu2[0], p2v0 = xu2[1], v12 = xu2[2];
            const float xu[6] = {p01.x, p01.y, p2v0.x, p2v0.y, v12.x, v12.y};
            if (!surely_not_near32(xv, xu, r32, R32)) s_l1[atomicAdd(&s_cnt[0], 1)] = u;
        }
        __syncthreads();
        const int cnt1 = s_cnt[0];
        for (int i = threadIdx.x; i < cnt1; i += blockDim.x) {
            const int u = s_l1[i];
            const BSums bs = boundary_sums(xv, X + (size_t)u * 6);
            if (!surely_not_near(bs, r_steer, r_conn)) {
                if (steer_one_root(bs, r_steer))
                    s_l2[atomicAdd(&s_cnt[1], 1)] = u;
                else
                    s_l2[kNearChunk - 1 - atomicAdd(&s_cnt[2], 1)] = u;
            }
        }
        __syncthreads();
        const int n_one = s_cnt[1], n_many = s_cnt[2];
        const int cnt2 = n_one + n_many;
        for (int base = 0; base < cnt2; base += blockDim.x) {
            const int i = base + threadIdx.x;
            bool ok = false;
            int u = 0;
            double tau = 0.0;
            if (i < cnt2) {
                u = s_l2[i < n_one ? i : kNearChunk - n_many + (i - n_one)];
                double c;
                steer64(xv, X + (size_t)u * 6, r_steer, tau, c);
                ok = c < r_conn && tau > kTauMin;
            }
            gw_push_near_block(gw, ok, v, u, tau, s_cnt + 3);
        }
        __syncthreads();
    }
}

// near for the column of node 0: thread p is the pair (p + 1) -> 0 (all
// lanes of a wave call it)
__device__ __forceinline__ void gw_near_col0(const float* __restrict__ X,
                                             const uint8_t* __restrict__ valid, int n, int p,
                                             double r_steer, double r_conn, const GraphWork& gw) {
    const int src = p + 1;
    bool ok = false;
    double tau = 0.0;
    if (src < n && valid[0] && valid[src] &&
        !surely_not_near32(X + (size_t)src * 6, X, (float)r_steer, (float)r_conn) &&
        !surely_not_near(boundary_sums(X + (size_t)src * 6, X), r_steer, r_conn)) {
        double c;
        steer64(X + (size_t)src * 6, X, r_steer, tau, c);
        ok = c < r_conn && tau > kTauMin;
    }
    gw_push_near(gw, ok, src, 0, tau);
}

// The quick test's 8 pieces of one connection against the boxes its range
// meets (bit set ov, n_ov boxes), each piece's hull computed once for all of
// them.  A hull that misses a box clears that piece for that box (as in
// trajectory_box_pieces).  A piece whose hull lies inside a box's slabs on
// two axes, by kHullMargin, while its end values on the third axis enclose a
// value inside that slab by the same margin, proves a hit: the third
// coordinate passes through its slab while the other two stay in theirs (a
// thin wall crossed inside its extent is settled this way).  Returns true on
// a proved hit; otherwise ov / n_ov keep the boxes that some piece's hull
// meets without a proof (left to the quick test) and the others are missed.
__device__ __forceinline__ bool pieces_vs_boxes(const Cubic* cs, double tau, const float* s_obs,
                                                unsigned long long* ov, int& n_ov) {
    constexpr int kP = 8;
    const double inv = 1.0 / (double)kP;
    const double h3 = (inv * tau) * (1.0 / 3.0);
    double pa[3], da[3];
    for (int a = 0; a < 3; ++a) {
        pa[a] = cs[a].c0;
        da[a] = cs[a].c1;
    }
    unsigned long long unres[kMaxObsWords] = {0ull, 0ull, 0ull, 0ull};
    for (int k = 1; k <= kP; ++k) {
        const double t = k == kP ? tau : tau * (inv * (double)k);
        double pb[3], db[3];
        eval_pd(cs, t, pb, db);
        double lo[3], hi[3], emin[3], emax[3];
        for (int a = 0; a < 3; ++a) {
            const double b1 = pa[a] + h3 * da[a], b2 = pb[a] - h3 * db[a];
            emin[a] = fmin(pa[a], pb[a]);
            emax[a] = fmax(pa[a], pb[a]);
            lo[a] = fmin(emin[a], fmin(b1, b2)) - kHullMargin;
            hi[a] = fmax(emax[a], fmax(b1, b2)) + kHullMargin;
        }
        for (int w = 0; w < kMaxObsWords; ++w) {
            unsigned long long m = ov[w];
            while (m) {
                const int o = w * 64 + __ffsll((long long)m) - 1;
                const unsigned long long bit = m & (~m + 1ull);
                m &= m - 1ull;
                const float* bx = s_obs + o * 6;
                bool sep = false, in[3], cr[3];
                for (int a = 0; a < 3; ++a) {
                    const double blo = (double)bx[a], bhi = (double)bx[3 + a];
                    sep |= (hi[a] < blo) | (lo[a] > bhi);
                    in[a] = (lo[a] >= blo) & (hi[a] <= bhi);
                    const double ilo = blo + kHullMargin, ihi = bhi - kHullMargin;
                    cr[a] = (ilo <= ihi) & (emin[a] <= ihi) & (emax[a] >= ilo);
                }
                if (sep) continue;
                if ((in[0] & in[1] & cr[2]) | (in[0] & cr[1] & in[2]) | (cr[0] & in[1] & in[2]))
                    return true;
                unres[w] |= bit;
            }
        }
        for (int a = 0; a < 3; ++a) {
            pa[a] = pb[a];
            da[a] = db[a];
        }
    }
    n_ov = 0;
    for (int w = 0; w < kMaxObsWords; ++w) {
        ov[w] = unres[w];
        n_ov += __popcll(unres[w]);
    }
    return false;
}

// boxes over one list of connections (src, dst, tau, optional cached range).
// Exact-queue entries name the connection by `tag` (>= 0: index into the
// roadmap list, < 0: -1 - index into the near list).  check_valid: skip
// connections with an invalid end (the cached roadmap list).
//
// Lane i of a wave takes connection i of the wave's 64 and finds the boxes
// its range meets (candidates from the workspace partition `bins`, then the
// range test), then runs pieces_vs_boxes over them.  The (connection, box)
// pairs that leaves open are spread over all 64 lanes through an LDS queue
// per wave, so a connection with many of them does not hold its wave: each
// pair gets the quick test, a hit blocks the connection, an unsure pair goes
// to the exact queue; connections not blocked set their bit.  Whole
// workgroup of kBoxThreads; s_q/s_src/s_dst/s_tau/s_blk are per-wave LDS
// arrays (kBoxQueue, 64, 64, 64, 64 entries per wave).
constexpr int kBoxThreads = 256;
constexpr int kBoxQueue = 256;

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void gw_boxes(const float* __restrict__ X,
                                         const uint8_t* __restrict__ valid,
                                         const int32_t* __restrict__ src_a,
                                         const int32_t* __restrict__ dst_a,
                                         const double* __restrict__ tau_a,
                                         const double* __restrict__ bbox, int count, bool near_list,
                                         bool check_valid, const float* s_obs, int n_obs,
                                         const BoxBins* bins,
                                         const GraphWork& gw, uint32_t* __restrict__ ebits,
                                         int words, int gid, int stride, uint32_t* s_q,
                                         int* s_src, int* s_dst, double* s_tau, int* s_blk) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t* q = s_q + w * kBoxQueue;
    int* qs = s_src + w * 64;
    int* qd = s_dst + w * 64;
    double* qt = s_tau + w * 64;
    int* blk = s_blk + w * 64;
    // all lanes of a wave iterate together (stride is a multiple of 64)
    for (int base = gid - lane; base < count; base += stride) {
        const int i = base + lane;
        bool keep = i < count;
        int src = 0, dst = 0;
        double tau = 0.0;
        if (keep) {
            src = src_a[i];
            dst = dst_a[i];
            tau = tau_a[i];
            keep = !check_valid || (valid[src] && valid[dst]);
        }
        unsigned long long ov[kMaxObsWords] = {0ull, 0ull, 0ull, 0ull};
        int n_ov = 0;
        bool proved = false;
        if (keep) {
            if (n_obs > 0) {
                double mn[3], mx[3];
                Cubic cs[3];
                if (bbox) {
                    for (int a = 0; a < 3; ++a) {
                        mn[a] = bbox[(size_t)i * 6 + a];
                        mx[a] = bbox[(size_t)i * 6 + 3 + a];
                    }
                } else {
                    hermite(X + (size_t)src * 6, X + (size_t)dst * 6, tau, cs);
                    for (int a = 0; a < 3; ++a) cubic_range(cs[a], tau, mn[a], mx[a]);
                }
                // the range rounded outwards to FP32: a box it misses in FP32
                // the FP64 range misses too; the few it then meets that the
                // FP64 range would not go to the piece and exact tests, which
                // decide them the same way
                float mnf[3], mxf[3];
                for (int a = 0; a < 3; ++a) {
                    mnf[a] = __double2float_rd(mn[a]);
                    mxf[a] = __double2float_ru(mx[a]);
                }
                unsigned long long cand[kMaxObsWords];
                box_bins_query(bins, mnf, mxf, cand);
                for (int w = 0; w < kMaxObsWords; ++w) {
                    unsigned long long m = cand[w];
                    while (m) {
                        const int o = w * 64 + __ffsll((long long)m) - 1;
                        m &= m - 1ull;
                        const float* bx = s_obs + o * 6;
                        const bool disjoint = (mxf[0] < bx[0]) | (mnf[0] > bx[3]) |
                                              (mxf[1] < bx[1]) | (mnf[1] > bx[4]) |
                                              (mxf[2] < bx[2]) | (mnf[2] > bx[5]);
                        if (!disjoint) {
                            ov[w] |= 1ull << (o & 63);
                            ++n_ov;
                        }
                    }
                }
                if (n_ov > 0) {
                    if (bbox) hermite(X + (size_t)src * 6, X + (size_t)dst * 6, tau, cs);
                    proved = pieces_vs_boxes(cs, tau, s_obs, ov, n_ov);
                    if (proved) n_ov = 0;
                }
            }
        }
        qs[lane] = src;
        qd[lane] = dst;
        qt[lane] = tau;
        blk[lane] = proved ? 1 : 0;
        // this lane's first pair within the wave's list
        int x = n_ov;
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        const int total = __shfl(x, 63, 64);
        const int first = x - n_ov;
        const int tag_base = near_list ? -1 - base : base;   // tag of lane 0's connection
        for (int seg = 0; seg < total; seg += kBoxQueue) {
            // this lane's pairs that fall in [seg, seg + kBoxQueue)
            if (n_ov > 0 && first < seg + kBoxQueue && first + n_ov > seg) {
                int k = first;
                for (int wd = 0; wd < kMaxObs / 64; ++wd) {
                    unsigned long long m = ov[wd];
                    while (m) {
                        const int o = wd * 64 + __ffsll((long long)m) - 1;
                        m &= m - 1ull;
                        if (k >= seg && k < seg + kBoxQueue) q[k - seg] = ((uint32_t)lane << 8) | (uint32_t)o;
                        ++k;
                    }
                }
            }
            wave_lds_sync();
            const int m_seg = min(total - seg, kBoxQueue);
            for (int j0 = 0; j0 < m_seg; j0 += 64) {
                const int j = j0 + lane;
                bool unsure = false;
                int who = 0, o = 0;
                if (j < m_seg) {
                    who = (int)(q[j] >> 8);
                    o = (int)(q[j] & 255u);
                    const int cs_src = qs[who], cs_dst = qd[who];
                    const double ct = qt[who];
                    Cubic cs[3];
                    hermite(X + (size_t)cs_src * 6, X + (size_t)cs_dst * 6, ct, cs);
                    const int r = trajectory_box_quick(cs, ct, s_obs + o * 6);
                    if (r == kBoxHit) blk[who] = 1;
                    unsure = r == kBoxUnsure;
                }
                const int slot = wave_append(unsure, gw.counts + 1);
                if (unsure && slot < gw.xq_cap) {
                    gw.xq_edge[slot] = near_list ? tag_base - who : tag_base + who;
                    gw.xq_box[slot] = o;
                }
            }
            wave_lds_sync();
        }
        wave_lds_sync();
        if (keep && !blk[lane]) atomicOr(&ebits[(size_t)src * words + (dst >> 5)], 1u << (dst & 31));
        wave_lds_sync();
    }
}

// exact: queued (connection, box) pairs; a hit clears the connection's bit
__device__ __forceinline__ void gw_exact(const float* __restrict__ X, const float* __restrict__ obs,
                                         const GraphWork& gw, const int32_t* __restrict__ rm_src,
                                         const int32_t* __restrict__ rm_dst,
                                         const double* __restrict__ rm_tau,
                                         uint32_t* __restrict__ ebits, int words, int gid,
                                         int stride) {
    // One wave per queued (connection, box); lane k takes piece k of 64 (the
    // piecewise test of trajectory_box_pieces, its pieces side by side), and
    // only if no piece proves a hit and some piece stays unsure does the wave
    // solve for the slab crossings (all lanes in step on the same inputs).
    constexpr int kPieces = 64;
    const int lane = threadIdx.x & 63;
    const int N = min(gw.counts[1], gw.xq_cap);
    for (int i = gid >> 6; i < N; i += stride >> 6) {
        const int tag = gw.xq_edge[i];
        int src, dst;
        double tau;
        if (tag >= 0) {
            src = rm_src[tag]; dst = rm_dst[tag]; tau = rm_tau[tag];
        } else {
            src = gw.near_src[-1 - tag]; dst = gw.near_dst[-1 - tag]; tau = gw.near_tau[-1 - tag];
        }
        Cubic cs[3];
        hermite(X + (size_t)src * 6, X + (size_t)dst * 6, tau, cs);
        const float* box = obs + (size_t)gw.xq_box[i] * 6;
        const double inv = 1.0 / (double)kPieces;
        const double h = inv * tau;
        const double h3 = h * (1.0 / 3.0), q3 = 0.25 * h3;
        const double ta = tau * (inv * (double)lane);
        const double tb = lane == kPieces - 1 ? tau : tau * (inv * (double)(lane + 1));
        double pa[3], da[3], pb[3], db[3];
        eval_pd(cs, ta, pa, da);
        eval_pd(cs, tb, pb, db);
        bool hit = lane < kPieces - 1 && point_in_box(pb, box);
        bool unsure = false;
        if (!hit && !piece_clear(pa, da, pb, db, h3, box)) {
            double qa[3] = {pa[0], pa[1], pa[2]}, qd[3] = {da[0], da[1], da[2]};
            for (int j = 1; j <= 4 && !hit; ++j) {
                double qb[3], qe[3];
                if (j == 4) {
                    for (int a = 0; a < 3; ++a) { qb[a] = pb[a]; qe[a] = db[a]; }
                } else {
                    eval_pd(cs, ta + 0.25 * (double)j * h, qb, qe);
                    hit = point_in_box(qb, box);
                }
                unsure |= !piece_clear(qa, qd, qb, qe, q3, box);
                for (int a = 0; a < 3; ++a) { qa[a] = qb[a]; qd[a] = qe[a]; }
            }
        }
        bool blocked = __ballot(hit) != 0ull;
        if (!blocked && __ballot(unsure) != 0ull) blocked = trajectory_hits_box_exact(cs, tau, box);
        if (blocked && lane == 0)
            atomicAnd(&ebits[(size_t)src * words + (dst >> 5)], ~(1u << (dst & 31)));
    }
}

// degree: out-degree of each row of the bit matrix (one wave per row)
__device__ __forceinline__ void row_deg_dev(const uint32_t* __restrict__ ebits, int n_nodes, int words,
                                            int32_t* __restrict__ deg, int v) {
    const int lane = threadIdx.x & 63;
    if (v >= n_nodes) return;
    int d = 0;
    for (int w = lane; w < words; w += 64) d += __popc(ebits[(size_t)v * words + w]);
    for (int o = 32; o > 0; o >>= 1) d += __shfl_down(d, o, 64);
    if (lane == 0) deg[v] = d;
}

__device__ __forceinline__ void graph_fill_dev(int n, const uint32_t* __restrict__ ebits,
                                                    const int32_t* __restrict__ row_ptr,
                                                    int32_t* __restrict__ col,
                                                    int32_t* __restrict__ esrc, int words) {
    // one wave per row, one 32-bit word of the row per lane and pass: the
    // lanes' bit counts scanned across the wave give each lane its first
    // slot, and the lane writes its word's columns in ascending order
    const int v = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (v >= n) return;
    int pos = row_ptr[v];
    for (int w0 = 0; w0 < words; w0 += 64) {
        const int w = w0 + lane;
        uint32_t bits = w < words ? ebits[(size_t)v * words + w] : 0u;
        const int c = __popc(bits);
        int x = c;
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        int at = pos + x - c;
        while (bits) {
            const int b = __ffs((int)bits) - 1;
            bits &= bits - 1u;
            col[at] = w * 32 + b;
            esrc[at] = v;
            ++at;
        }
        pos += __shfl(x, 63, 64);
    }
}

// Pass 2 from the near list, without steering again.  The near list holds
// each connection's tau* from pass 1 and every graph edge is one of its
// entries whose bit survived the box and exact stages, so:
//   word_start_dev: the CSR slot of the first edge of each 32-bit word of
//     each row (one wave per row, the words' bit counts scanned);
//   near_to_slot_dev: each surviving near entry's slot (its word's start
//     plus the bits below it in the word) receives its tau* -- in ecost,
//     since etau still holds the near list;
//   edge_cost_dev (after graph_fill_dev): tau* to etau and c* = cost_of(tau*)
//     to ecost, the very expression steer64 returns, so (tau*, c*) equal
//     what a second steering would give, bit for bit.
__device__ __forceinline__ void word_start_dev(int n, const uint32_t* __restrict__ ebits,
                                               const int32_t* __restrict__ row_ptr,
                                               int32_t* __restrict__ wstart, int words) {
    const int v = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (v >= n) return;
    int pos = row_ptr[v];
    for (int w0 = 0; w0 < words; w0 += 64) {
        const int w = w0 + lane;
        const int c = w < words ? __popc(ebits[(size_t)v * words + w]) : 0;
        int x = c;
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (w < words) wstart[(size_t)v * words + w] = pos + x - c;
        pos += __shfl(x, 63, 64);
    }
}

__device__ __forceinline__ void near_to_slot_dev(const GraphWork& gw, const uint32_t* __restrict__ ebits,
                                                 const int32_t* __restrict__ wstart, int words,
                                                 double* __restrict__ slot_tau) {
    const int count = min(gw.counts[0], gw.near_cap);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        const int v = gw.near_src[i], u = gw.near_dst[i];
        const size_t wi = (size_t)v * words + (u >> 5);
        const uint32_t word = ebits[wi];
        const uint32_t bit = 1u << (u & 31);
        if (word & bit) slot_tau[wstart[wi] + __popc(word & (bit - 1u))] = gw.near_tau[i];
    }
}

__device__ __forceinline__ void edge_cost_dev(const float* __restrict__ X, int n, double r_steer,
                                              const int32_t* __restrict__ row_ptr,
                                              const int32_t* __restrict__ col,
                                              const int32_t* __restrict__ esrc,
                                              double* __restrict__ etau, double* __restrict__ ecost) {
    const int E = row_ptr[n];
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < E; e += gridDim.x * blockDim.x) {
        const double tau = ecost[e];
        const BSums s = boundary_sums(X + (size_t)esrc[e] * 6, X + (size_t)col[e] * 6);
        etau[e] = tau;
        ecost[e] = cost_of(tau, s, r_steer);
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
