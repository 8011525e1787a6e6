// Per-query setup kernels: the particle deviation table and BuildGraph (Alg. 3).
#include "device_math.hpp"
#include "pump_internal.hpp"

namespace pump {

// ---------------------------------------------------------------------------
// Particle deviation table (Sec. III-B particles; eq. (2) closed loop).
// One thread per (axis a, particle j) runs the recurrence
//   dx_{s+1} = A_cl dx_s + L (xi[s][2a][j], xi[s][2a+1][j])^T,  dx_0 = 0
// in FP64 and stores the position part D[s][a][j] in FP32.
// ---------------------------------------------------------------------------
__global__ void k_deviation(const float* __restrict__ noise, float* __restrict__ D, int N,
                            int S, double a00, double a01, double a10, double a11, double l00,
                            double l10, double l11) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * N) return;
    int a = t / N, j = t - a * N;
    double p = 0.0, v = 0.0;
    D[(size_t)a * N + j] = 0.0f;
    for (int s = 0; s < S; ++s) {
        double w0 = (double)noise[((size_t)s * 6 + 2 * a) * N + j];
        double w1 = (double)noise[((size_t)s * 6 + 2 * a + 1) * N + j];
        double pn = a00 * p + a01 * v + l00 * w0;
        double vn = a10 * p + a11 * v + (l10 * w0 + l11 * w1);
        p = pn;
        v = vn;
        D[((size_t)(s + 1) * 3 + a) * N + j] = (float)p;
    }
}

// Bounding box of the particle cloud at each step: cloud[s] = (min_j D[s][a][j], max_j ...).
__global__ void k_cloud(const float* __restrict__ D, float* __restrict__ cloud, int N) {
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

__global__ void k_gcloud(const float* __restrict__ cloud, float* __restrict__ g, int S1) {
    int t = threadIdx.x;
    if (t >= 6) return;
    float v = cloud[t];
    for (int s = 1; s < S1; ++s) {
        float c = cloud[(size_t)s * 6 + t];
        v = t < 3 ? fminf(v, c) : fmaxf(v, c);
    }
    g[t] = v;
}

void launch_deviation_table(hipStream_t s, const float* noise, float* D, float* cloud,
                            float* gcloud, int N, int S_max, const double* Acl,
                            const double* L) {
    int threads = 3 * N;
    k_deviation<<<(threads + 255) / 256, 256, 0, s>>>(noise, D, N, S_max, Acl[0], Acl[1],
                                                      Acl[2], Acl[3], L[0], L[2], L[3]);
    k_cloud<<<S_max + 1, 256, 0, s>>>(D, cloud, N);
    k_gcloud<<<1, 64, 0, s>>>(cloud, gcloud, S_max + 1);
}

// ---------------------------------------------------------------------------
// Node validity (sample not in a closed obstacle box) and goal membership
// (position in the closed goal box).
// ---------------------------------------------------------------------------
__global__ void k_mark_valid(const float* __restrict__ X, int n, const float* __restrict__ obs,
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

void launch_mark_valid(hipStream_t s, const float* X, int n_nodes, const float* obs, int n_obs,
                       const float* gb, uint8_t* valid, uint8_t* goal, int32_t* bad) {
    int n = n_nodes > n_obs ? n_nodes : n_obs;
    k_mark_valid<<<(n + 255) / 256, 256, 0, s>>>(X, n_nodes, obs, n_obs, gb[0], gb[1], gb[2],
                                                 gb[3], gb[4], gb[5], valid, goal, bad);
}

// ---------------------------------------------------------------------------
// BuildGraph (Alg. 3).  Edge v -> u iff both nodes are valid, u != v,
// c*(v,u) < r_n, tau* > 1e-6 and the nominal trajectory meets no obstacle
// (continuous, exact; closed boxes).  Pass 1 evaluates every ordered pair and
// records the result as a bit matrix and per-row counts; after a scan of the
// counts, pass 2 writes each row's neighbours in ascending order with their
// (tau*, c*).
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool edge_free(const float* xv, const float* xu, double tau,
                                          const float* s_obs, int n_obs) {
    Cubic cs[3];
    hermite(xv, xu, tau, cs);
    double mn[3], mx[3];
    for (int a = 0; a < 3; ++a) cubic_range(cs[a], tau, mn[a], mx[a]);
    for (int o = 0; o < n_obs; ++o) {
        const float* b = s_obs + o * 6;
        bool disjoint = false;
        for (int a = 0; a < 3; ++a)
            disjoint |= (mx[a] < (double)b[a]) | (mn[a] > (double)b[3 + a]);
        if (disjoint) continue;
        if (trajectory_hits_box(cs, tau, b)) return false;
    }
    return true;
}

__global__ __launch_bounds__(256) void k_graph_mark(const float* __restrict__ X,
                                                    const uint8_t* __restrict__ valid, int n,
                                                    const float* __restrict__ obs, int n_obs,
                                                    double r_steer, double r_conn,
                                                    uint32_t* __restrict__ ebits,
                                                    int32_t* __restrict__ deg, int words) {
    __shared__ float s_obs[kMaxObs * 6];
    for (int t = threadIdx.x; t < n_obs * 6; t += blockDim.x) s_obs[t] = obs[t];
    __syncthreads();
    const int v = blockIdx.y;
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    float xv[6], xu[6];
    for (int k = 0; k < 6; ++k) xv[k] = X[(size_t)v * 6 + k];
    bool e = false;
    if (u < n && u != v && valid[u] && valid[v]) {
        for (int k = 0; k < 6; ++k) xu[k] = X[(size_t)u * 6 + k];
        double tau, c;
        steer64(xv, xu, r_steer, tau, c);
        if (c < r_conn && tau > kTauMin) e = edge_free(xv, xu, tau, s_obs, n_obs);
    }
    unsigned long long b = __ballot(e);
    if (lane == 0) {
        const int base = (u - lane) / 32;            // u - lane is a multiple of 64
        if (base < words) {
            ebits[(size_t)v * words + base] = (uint32_t)b;
            ebits[(size_t)v * words + base + 1] = (uint32_t)(b >> 32);
        }
        if (b) atomicAdd(&deg[v], (int)__popcll(b));
    }
}

__global__ __launch_bounds__(256) void k_graph_fill(const float* __restrict__ X, int n,
                                                    double r_steer,
                                                    const uint32_t* __restrict__ ebits,
                                                    const int32_t* __restrict__ row_ptr,
                                                    int32_t* __restrict__ col,
                                                    double* __restrict__ etau,
                                                    double* __restrict__ ecost, int words) {
    const int v = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (v >= n) return;
    float xv[6];
    for (int k = 0; k < 6; ++k) xv[k] = X[(size_t)v * 6 + k];
    int pos = row_ptr[v];
    for (int base = 0; base < n; base += 64) {
        uint32_t w = ebits[(size_t)v * words + base / 32 + (lane >> 5)];
        bool e = (w >> (lane & 31)) & 1u;
        unsigned long long b = __ballot(e);
        if (e) {
            int u = base + lane;
            unsigned long long below = lane ? (b & ((1ull << lane) - 1ull)) : 0ull;
            int at = pos + (int)__popcll(below);
            float xu[6];
            for (int k = 0; k < 6; ++k) xu[k] = X[(size_t)u * 6 + k];
            double tau, c;
            steer64(xv, xu, r_steer, tau, c);
            col[at] = u;
            etau[at] = tau;
            ecost[at] = c;
        }
        pos += (int)__popcll(b);
    }
}

void launch_graph_mark(hipStream_t s, const float* X, const uint8_t* valid, int n_nodes,
                       const float* obs, int n_obs, double r_steer, double r_conn,
                       uint32_t* ebits, int32_t* deg, int words) {
    dim3 grid((n_nodes + 255) / 256, n_nodes);
    k_graph_mark<<<grid, 256, 0, s>>>(X, valid, n_nodes, obs, n_obs, r_steer, r_conn, ebits, deg,
                                      words);
}

void launch_graph_fill(hipStream_t s, const float* X, int n_nodes, double r_steer,
                       const uint32_t* ebits, const int32_t* row_ptr, int32_t* col,
                       double* etau, double* ecost, int words) {
    k_graph_fill<<<(n_nodes + 3) / 4, 256, 0, s>>>(X, n_nodes, r_steer, ebits, row_ptr, col,
                                                   etau, ecost, words);
}

}  // namespace pump
