// Per-query operations of PlanSelection (Alg. 5), shared by the single-query
// kernels and the batched engine.
#pragma once

#include "device_math.hpp"
#include "pump_internal.hpp"

namespace pump {

// P_goal = plans still in P(v) for goal nodes v (Alg. 4 return), in id order
// (whole block; blockDim.x a multiple of 64, at most 1024).  a.n_plans < 0:
// the plan count is read from the control block (Explore still in flight on
// the stream when the host enqueued this).
__device__ __forceinline__ void goal_collect_block(const SelectArgs& a) {
    const int n_plans = a.n_plans >= 0 ? a.n_plans : a.ctl->n_plans;
    __shared__ int s_w[16];
    __shared__ int s_base;
    const int nw = blockDim.x >> 6;
    if (threadIdx.x == 0) s_base = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int b0 = 0; b0 < n_plans; b0 += blockDim.x) {
        const int p = b0 + threadIdx.x;
        const bool f = p < n_plans && a.p_state[p] != kRemoved && a.goal[a.p_head[p]];
        const unsigned long long m = __ballot(f);
        if (lane == 0) s_w[wave] = __popcll(m);
        __syncthreads();
        int off = s_base;
        for (int w = 0; w < wave; ++w) off += s_w[w];
        const int pos = off + (int)__popcll(m & (lane ? ((1ull << lane) - 1ull) : 0ull));
        if (f && pos < kMaxGoal) a.goal_ids[pos] = p;
        __syncthreads();
        if (threadIdx.x == 0) {
            int t = 0;
            for (int w = 0; w < nw; ++w) t += s_w[w];
            s_base += t;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) a.ctl->n_goal = s_base;
}

// Pareto front of P_goal (d dominates p iff p.cost > d.cost and
// p.pop >= d.pop), sorted by pop ascending, cost descending, then node
// sequence.  Paths are reconstructed from the parent links.
__device__ __forceinline__ int path_of(const SelectArgs& a, int p, int* out, int cap) {
    int n = 0;
    for (int q = p; q >= 0 && n < cap; q = a.p_parent[q]) out[n++] = a.p_head[q];
    for (int i = 0; i < n / 2; ++i) { int t = out[i]; out[i] = out[n - 1 - i]; out[n - 1 - i] = t; }
    return n;
}

__device__ __forceinline__ bool front_less(const SelectArgs& a, int fa, int fb) {
    const int pa = a.front_ids[fa], pb = a.front_ids[fb];
    if (a.p_pop[pa] != a.p_pop[pb]) return a.p_pop[pa] < a.p_pop[pb];
    if (a.p_cost[pa] != a.p_cost[pb]) return a.p_cost[pa] > a.p_cost[pb];
    const int stride = a.S_max + 1;
    const int* xa = a.paths + (size_t)fa * stride;
    const int* xb = a.paths + (size_t)fb * stride;
    const int la = a.path_len[fa], lb = a.path_len[fb];
    for (int i = 0; i < la && i < lb; ++i)
        if (xa[i] != xb[i]) return xa[i] < xb[i];
    return la < lb;
}

// Whole block; `max_front` bounds the front kept (kMaxFront or less).
// The dominance test takes the goal plans' (cost, pop) in LDS tiles; the
// front's paths are rebuilt by a thread each, ordered by one thread on an
// index array, and rebuilt once more in that order (no path is moved).
constexpr int kFrontTile = 256;

__device__ __forceinline__ void front_block(const SelectArgs& a, int max_front) {
    __shared__ int s_flag[kMaxFront];
    __shared__ int s_ord[kMaxFront];
    __shared__ double s_c[kFrontTile];
    __shared__ int s_k[kFrontTile];
    __shared__ int s_n;
    const int G = a.ctl->n_goal < kMaxGoal ? a.ctl->n_goal : kMaxGoal;
    if (threadIdx.x == 0) s_n = 0;
    for (int g0 = 0; g0 < G; g0 += blockDim.x) {   // (the same trip count in every thread)
        const int g = g0 + threadIdx.x;
        const bool have = g < G;
        double c = 0.0;
        int k = 0;
        if (have) {
            const int p = a.goal_ids[g];
            c = a.p_cost[p];
            k = a.p_pop[p];
        }
        bool dom = false;
        for (int h0 = 0; h0 < G; h0 += kFrontTile) {
            __syncthreads();
            for (int t = threadIdx.x; t < kFrontTile && h0 + t < G; t += blockDim.x) {
                const int d = a.goal_ids[h0 + t];
                s_c[t] = a.p_cost[d];
                s_k[t] = a.p_pop[d];
            }
            __syncthreads();
            const int hn = min(kFrontTile, G - h0);
            if (have)
                for (int h = 0; h < hn && !dom; ++h) dom = (c > s_c[h]) && (k >= s_k[h]);
        }
        if (have && !dom) {
            const int slot = atomicAdd(&s_n, 1);
            if (slot < max_front) s_flag[slot] = g;
        }
    }
    __syncthreads();
    const int n = s_n < max_front ? s_n : max_front;
    if (threadIdx.x == 0) {
        if (s_n > max_front) a.ctl->err = 2;
        // deterministic order of discovery: sort slots by goal index
        for (int i = 1; i < n; ++i) {
            const int v = s_flag[i];
            int j = i - 1;
            while (j >= 0 && s_flag[j] > v) { s_flag[j + 1] = s_flag[j]; --j; }
            s_flag[j + 1] = v;
        }
    }
    __syncthreads();
    const int stride = a.S_max + 1;
    for (int f = threadIdx.x; f < n; f += blockDim.x) {
        a.front_ids[f] = a.goal_ids[s_flag[f]];
        a.path_len[f] = path_of(a, a.front_ids[f], a.paths + (size_t)f * stride, stride);
        s_ord[f] = f;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // insertion sort of the front's indices (pop, then cost, then path)
        for (int i = 1; i < n; ++i) {
            const int v = s_ord[i];
            int j = i - 1;
            while (j >= 0 && front_less(a, v, s_ord[j])) { s_ord[j + 1] = s_ord[j]; --j; }
            s_ord[j + 1] = v;
        }
    }
    __syncthreads();
    int id[(kMaxFront + 63) / 64];   // this thread's entries in the sorted order
    for (int f = threadIdx.x, r = 0; f < n; f += blockDim.x, ++r) id[r] = a.front_ids[s_ord[f]];
    __syncthreads();
    for (int f = threadIdx.x, r = 0; f < n; f += blockDim.x, ++r) {
        a.front_ids[f] = id[r];
        a.path_len[f] = path_of(a, id[r], a.paths + (size_t)f * stride, stride);
    }
    if (threadIdx.x == 0) a.ctl->n_front = n;
}

// Nominal tracking waypoints of path f (step 0 = the first node's position):
// each connection (u, v) contributes K_e = max(1, ceil(tau*/dt)) waypoints at
// t_k = k tau*/K_e.
__device__ __forceinline__ void waypoints_one(const SelectArgs& a, int f) {
    const int stride = a.S_max + 1;
    const int* nodes = a.paths + (size_t)f * stride;
    const int len = a.path_len[f];
    double* wp = a.wp + (size_t)f * stride * 3;
    const float* x0 = a.X + (size_t)nodes[0] * 6;
    for (int ax = 0; ax < 3; ++ax) wp[ax] = (double)x0[ax];
    int s = 0;
    bool ok = true;
    for (int l = 1; l < len && ok; ++l) {
        const float* xu = a.X + (size_t)nodes[l - 1] * 6;
        const float* xv = a.X + (size_t)nodes[l] * 6;
        double tau, c;
        steer64(xu, xv, a.r_steer, tau, c);
        const int K = max(1, (int)ceil(tau / a.dt));
        if (s + K > a.S_max) { ok = false; break; }
        Cubic cs[3];
        hermite(xu, xv, tau, cs);
        for (int k = 1; k <= K; ++k) {
            const double t = ((double)k * tau) / (double)K;
            for (int ax = 0; ax < 3; ++ax) wp[(size_t)(s + k) * 3 + ax] = cs[ax].at(t);
        }
        s += K;
    }
    a.wp_len[f] = ok ? s : -1;
}

// The same for one path by a whole wave (all 64 lanes call it): lane l takes
// the path's edges l + 1, l + 65, ...; the edges' waypoint counts are scanned
// across the wave for their offsets, so the root solves run side by side.
// Every waypoint is computed as in waypoints_one (same steer, same cubic,
// same t_k), so the table is identical; a path past S_max gets wp_len -1.
__device__ __forceinline__ void waypoints_wave(const SelectArgs& a, int f) {
    const int lane = threadIdx.x & 63;
    const int stride = a.S_max + 1;
    const int* nodes = a.paths + (size_t)f * stride;
    const int len = a.path_len[f];
    double* wp = a.wp + (size_t)f * stride * 3;
    if (lane == 0) {
        const float* x0 = a.X + (size_t)nodes[0] * 6;
        for (int ax = 0; ax < 3; ++ax) wp[ax] = (double)x0[ax];
    }
    int s0 = 0;                            // waypoints before this chunk of edges
    for (int l0 = 1; l0 < len; l0 += 64) {
        const int l = l0 + lane;
        double tau = 0.0;
        int K = 0;
        if (l < len) {
            double c;
            steer64(a.X + (size_t)nodes[l - 1] * 6, a.X + (size_t)nodes[l] * 6, a.r_steer, tau, c);
            K = max(1, (int)ceil(tau / a.dt));
        }
        int x = K;                         // inclusive scan of K over the lanes
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        const int s = s0 + x - K;          // this edge's first step - 1
        if (l < len) {
            Cubic cs[3];
            hermite(a.X + (size_t)nodes[l - 1] * 6, a.X + (size_t)nodes[l] * 6, tau, cs);
            for (int k = 1; k <= K && s + k <= a.S_max; ++k) {
                const double t = ((double)k * tau) / (double)K;
                for (int ax = 0; ax < 3; ++ax) wp[(size_t)(s + k) * 3 + ax] = cs[ax].at(t);
            }
        }
        s0 += __shfl(x, 63, 64);
    }
    if (lane == 0) a.wp_len[f] = s0 <= a.S_max ? s0 : -1;
}

// Alg. 5's choice among the risk-sorted front (cp_hat ascending): a
// bisection for the riskiest plan whose certification count stays within
// alpha, premised on MC growing along that order.  `good` (1-based) is the
// plan the search stands on -- it starts on the safest plan, not yet
// evaluated -- and plans from `bad` on are ruled out.  Each probe takes the
// middle of the open range: a count within alpha moves `good` up to it, one
// above alpha moves `bad` down to it.  Once nothing lies strictly between the
// two, `good` is checked once more (it may never have been probed).  Returns
// its 0-based index, or -1 when that check fails (infeasible) or nf < 1.
__device__ __forceinline__ int certified_pick(const int* mc_counts, int nf, int M, double alpha) {
    if (nf < 1) return -1;
    auto within = [&](int k) { return (double)mc_counts[k - 1] / (double)M <= alpha; };
    int good = 1, bad = nf + 1;
    while (bad - good > 1) {
        const int mid = (good + bad) >> 1;
        if (within(mid)) good = mid; else bad = mid;
    }
    return within(good) ? good - 1 : -1;
}

// Does the segment prev -> cur meet one of the closed obstacle boxes
// o0, o0 + ostep, ...?  Slab clipping in FP64 after a bounding-box reject.
__device__ __forceinline__ bool segment_hits_boxes(const double prev[3], const double cur[3],
                                                   const float* s_obs, int n_obs, int o0,
                                                   int ostep) {
    double smin[3], smax[3];
    for (int ax = 0; ax < 3; ++ax) {
        smin[ax] = fmin(prev[ax], cur[ax]);
        smax[ax] = fmax(prev[ax], cur[ax]);
    }
    bool hit = false;
    for (int o = o0; o < n_obs && !hit; o += ostep) {
        const float* b = s_obs + o * 6;
        // a segment whose bounding box misses the box misses the box
        if ((smax[0] < (double)b[0]) | (smin[0] > (double)b[3]) | (smax[1] < (double)b[1]) |
            (smin[1] > (double)b[4]) | (smax[2] < (double)b[2]) | (smin[2] > (double)b[5]))
            continue;
        double t0 = 0.0, t1 = 1.0;
        bool miss = false;
        for (int ax = 0; ax < 3; ++ax) {
            const double d = cur[ax] - prev[ax];
            const double lo = (double)b[ax], hi = (double)b[3 + ax];
            if (d == 0.0) {
                miss |= (prev[ax] < lo) | (prev[ax] > hi);
            } else {
                const double ta = (lo - prev[ax]) / d, tb = (hi - prev[ax]) / d;
                t0 = fmax(t0, fmin(ta, tb));
                t1 = fmin(t1, fmax(ta, tb));
            }
        }
        hit = !miss && (t0 <= t1);
    }
    return hit;
}

// MC(p) for one certification particle m over nominal waypoints wp[0..S]
// (step 0 = the start): its deviation follows the closed-loop recurrence from
// zero with its own noise; its workspace path is the polyline through the
// waypoint positions plus deviations; it collides iff a segment meets a
// closed obstacle box (slab clipping, FP64).
__device__ __forceinline__ bool mc_particle_lqr(const SelectArgs& a, const double* wp, int S,
                                                int m, const float* s_obs, int o0, int ostep) {
    double dp[3] = {0.0, 0.0, 0.0}, dv[3] = {0.0, 0.0, 0.0};
    double prev[3] = {wp[0], wp[1], wp[2]};
    const double a00 = a.Acl[0], a01 = a.Acl[1], a10 = a.Acl[2], a11 = a.Acl[3];
    const double l00 = a.L[0], l10 = a.L[2], l11 = a.L[3];
    bool hit = false;
    for (int s = 0; s < S && !hit; ++s) {
        double cur[3];
        for (int ax = 0; ax < 3; ++ax) {
            const double w0 = (double)a.noise_mc[((size_t)s * 6 + 2 * ax) * a.M + m];
            const double w1 = (double)a.noise_mc[((size_t)s * 6 + 2 * ax + 1) * a.M + m];
            const double pn = a00 * dp[ax] + a01 * dv[ax] + l00 * w0;
            const double vn = a10 * dp[ax] + a11 * dv[ax] + (l10 * w0 + l11 * w1);
            dp[ax] = pn;
            dv[ax] = vn;
            cur[ax] = wp[(size_t)(s + 1) * 3 + ax] + pn;
        }
        hit = segment_hits_boxes(prev, cur, s_obs, a.n_obs, o0, ostep);
        prev[0] = cur[0]; prev[1] = cur[1]; prev[2] = cur[2];
    }
    return hit;
}

// The same under LQG tracking: per axis the particle carries (dp, dv, p_hat,
// v_hat), driven by its two process normals and its measurement normal.
__device__ __forceinline__ bool mc_particle_lqg(const SelectArgs& a, const double* wp, int S,
                                                int m, const float* s_obs, int o0, int ostep) {
    double z[3][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
    double prev[3] = {wp[0], wp[1], wp[2]};
    bool hit = false;
    for (int s = 0; s < S && !hit; ++s) {
        double cur[3];
        for (int ax = 0; ax < 3; ++ax) {
            const double w0 = (double)a.noise_mc[((size_t)s * 6 + 2 * ax) * a.M + m];
            const double w1 = (double)a.noise_mc[((size_t)s * 6 + 2 * ax + 1) * a.M + m];
            const double w2 = (double)a.noise_mc_meas[((size_t)s * 3 + ax) * a.M + m];
            lqg_step(a.lqg, z[ax], w0, w1, w2);
            cur[ax] = wp[(size_t)(s + 1) * 3 + ax] + z[ax][0];
        }
        hit = segment_hits_boxes(prev, cur, s_obs, a.n_obs, o0, ostep);
        prev[0] = cur[0]; prev[1] = cur[1]; prev[2] = cur[2];
    }
    return hit;
}

__device__ __forceinline__ bool mc_particle_wp(const SelectArgs& a, const double* wp, int S, int m,
                                               const float* s_obs, int o0, int ostep) {
    if (m >= a.M || S < 0) return false;
    return a.estimator ? mc_particle_lqg(a, wp, S, m, s_obs, o0, ostep)
                       : mc_particle_lqr(a, wp, S, m, s_obs, o0, ostep);
}

// MC(p) over waypoints wp[0..S] for the 64 particles m_base .. m_base + 63,
// one workgroup of kMcThreads: wave w tests the boxes w, w + 4, ... (each
// wave follows all 64 particles through the same recurrence), the per-wave
// hits are ORed in LDS and their count added to *count.  s_obs holds the
// boxes, s_hit 64 flags.
constexpr int kMcThreads = 256;
constexpr int kMcParticles = 64;

__device__ __forceinline__ void mc_block_count(const SelectArgs& a, const double* wp, int S,
                                               int m_base, const float* s_obs, int* s_hit,
                                               int* count) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x < kMcParticles) s_hit[threadIdx.x] = 0;
    __syncthreads();
    if (mc_particle_wp(a, wp, S, m_base + lane, s_obs, w, kMcThreads / 64)) s_hit[lane] = 1;
    __syncthreads();
    if (w == 0) {
        const unsigned long long b = __ballot(s_hit[lane] != 0);
        if (lane == 0 && b) atomicAdd(count, (int)__popcll(b));
    }
}

}  // namespace pump
