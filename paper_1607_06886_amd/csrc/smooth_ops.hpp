// Smooth(p*, alpha), the last step of PlanSelection (Alg. 5), shared by the
// single-query kernels and the batched engine.
//
// The selected plan p* (its concatenated edge cubics, duration T_p) is
// blended with the optimal connection q from x_init to p*.head (duration
// tau_q): with weight beta, duration T = (1 - beta) T_p + beta tau_q and
// position P(s) = (1 - beta) p(s T_p) + beta q(s tau_q) over normalised time
// s in [0, 1], which keeps both boundary states.  The blend's tracking grid
// has K = max(1, ceil(T / dt)) waypoints at s = k / K, and it is certified by
// MC over them with the certification particles of MC(p).  beta = 1 is tried
// first, then kSmoothLevels bisection steps on [0, 1] keep the certified side
// low; the blend at the final low end replaces p* if its cost
// T + r_u int |P''|^2 ds / T^3 is lower.
//
// On the GPU the bisection is evaluated three levels at a time: a round
// certifies the 7 midpoints of the next three levels of the current interval
// (plus beta = 1 in the first round) at once, then one thread replays the
// three decisions.  The weights are dyadic, so every side computes the same
// weights exactly, and the decisions equal those of the sequential search.
#pragma once

#include "device_math.hpp"
#include "pump_internal.hpp"
#include "select_ops.hpp"

namespace pump {

// Weight of candidate c in round r (-1: not evaluated).
__device__ __forceinline__ double smooth_beta(const SmoothState& st, int r, int c) {
    if (st.done || st.E < 1) return -1.0;
    if (r == 0) return c == 0 ? 1.0 : (double)c / 8.0;
    if (c == 0) return -1.0;
    return st.lo + (st.hi - st.lo) * ((double)c / 8.0);
}

// Position of the blend at normalised time s.
__device__ __forceinline__ void smooth_pos(const SmoothState& st, const SmoothBuf& b, double beta,
                                           double s, double out[3]) {
    const double t = s * st.T_p;
    // edge holding plan time t: the last e with e_t0[e] <= t, within [0, E-1]
    int lo = 0, hi = st.E;   // invariant: e_t0[lo] <= t (or lo = 0), answer < hi
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (b.e_t0[mid] <= t) lo = mid; else hi = mid;
    }
    const double loc = t - b.e_t0[lo];
    const double tq = s * st.tau_q;
    const double* c = b.e_coef + (size_t)lo * 12;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double p = c[4 * a] + loc * (c[4 * a + 1] + loc * (c[4 * a + 2] + loc * c[4 * a + 3]));
        const double* q = st.qc + 4 * a;
        const double r = q[0] + tq * (q[1] + tq * (q[2] + tq * q[3]));
        out[a] = (1.0 - beta) * p + beta * r;
    }
}

__device__ __forceinline__ int smooth_steps(const SmoothState& st, double beta, double dt) {
    const double T = (1.0 - beta) * st.T_p + beta * st.tau_q;
    return max(1, (int)ceil(T / dt));
}

// Edge cubics of p*, the optimal connection and the search state (one block).
__device__ __forceinline__ void smooth_prep_block(const SelectArgs& a, int f_best, double plan_cost,
                                                  const SmoothBuf& b) {
    SmoothState& st = *b.st;
    const int stride = a.S_max + 1;
    const int len = f_best >= 0 ? a.path_len[f_best] : 0;
    const int E = len > 1 ? len - 1 : 0;
    const int* nodes = a.paths + (size_t)(f_best >= 0 ? f_best : 0) * stride;
    for (int e = threadIdx.x; e < E; e += blockDim.x) {
        const float* xu = a.X + (size_t)nodes[e] * 6;
        const float* xv = a.X + (size_t)nodes[e + 1] * 6;
        double tau, c;
        steer64(xu, xv, a.r_steer, tau, c);
        Cubic cs[3];
        hermite(xu, xv, tau, cs);
        double* o = b.e_coef + (size_t)e * 12;
        for (int ax = 0; ax < 3; ++ax) {
            o[4 * ax] = cs[ax].c0; o[4 * ax + 1] = cs[ax].c1;
            o[4 * ax + 2] = cs[ax].c2; o[4 * ax + 3] = cs[ax].c3;
        }
        b.e_t0[e + 1] = tau;   // durations; summed below
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    st.E = E;
    st.f_best = f_best;
    st.plan_cost = plan_cost;
    st.lo = 0.0;
    st.hi = 1.0;
    st.lo_cnt = 0;
    st.lo_K = 0;
    st.done = E < 1;
    st.beta = 0.0;
    b.e_t0[0] = 0.0;
    double T = 0.0;
    for (int e = 0; e < E; ++e) {
        T = T + b.e_t0[e + 1];
        b.e_t0[e + 1] = T;
    }
    st.T_p = T;
    if (E >= 1) {
        const float* x0 = a.X + (size_t)nodes[0] * 6;
        const float* xh = a.X + (size_t)nodes[E] * 6;
        double tau, c;
        steer64(x0, xh, a.r_steer, tau, c);
        Cubic cs[3];
        hermite(x0, xh, tau, cs);
        st.tau_q = tau;
        for (int ax = 0; ax < 3; ++ax) {
            st.qc[4 * ax] = cs[ax].c0; st.qc[4 * ax + 1] = cs[ax].c1;
            st.qc[4 * ax + 2] = cs[ax].c2; st.qc[4 * ax + 3] = cs[ax].c3;
        }
    } else {
        st.tau_q = 0.0;
    }
}

// Waypoints of candidate c in round r; thread k of the candidate writes
// waypoint k (k = 0 also records the step count and clears the count).
__device__ __forceinline__ void smooth_wp_one(const SelectArgs& a, const SmoothBuf& b, int r, int c,
                                              int k) {
    const SmoothState& st = *b.st;
    const double beta = smooth_beta(st, r, c);
    if (beta < 0.0) return;
    const int K = smooth_steps(st, beta, a.dt);
    if (k == 0) {
        b.st->K[c] = K > a.S_max ? -1 : K;
        b.st->cnt[c] = 0;
    }
    if (K > a.S_max || k > K) return;
    double p[3];
    smooth_pos(st, b, beta, (double)k / (double)K, p);
    double* o = b.wp + ((size_t)c * (a.S_max + 1) + k) * 3;
    o[0] = p[0]; o[1] = p[1]; o[2] = p[2];
}

// Replay of round r's three bisection levels (one thread).
__device__ __forceinline__ void smooth_resolve_one(const SelectArgs& a, double alpha,
                                                   const SmoothBuf& b, int r) {
    SmoothState& st = *b.st;
    if (st.done || st.E < 1) return;
    auto certified = [&](int c) {
        return st.K[c] >= 0 && !((double)st.cnt[c] / (double)a.M > alpha);
    };
    if (r == 0 && certified(0)) {
        st.lo = 1.0;
        st.lo_cnt = st.cnt[0];
        st.lo_K = st.K[0];
        st.done = 1;
        return;
    }
    const double lo0 = st.lo, w = st.hi - st.lo;
    for (int lvl = 0; lvl < 3; ++lvl) {
        const double m = 0.5 * (st.lo + st.hi);
        const int c = (int)((m - lo0) / w * 8.0);
        if (certified(c)) {
            st.lo = m;
            st.lo_cnt = st.cnt[c];
            st.lo_K = st.K[c];
        } else {
            st.hi = m;
        }
    }
    if (r == kSmoothRounds - 1) st.done = 1;
}

// Result: the blend at lo if lo > 0 and it is cheaper than p*, else p*
// (count and steps of p* given); its waypoints go to out_wp.  One block.
__device__ __forceinline__ void smooth_final_block(const SelectArgs& a, const SmoothBuf& b,
                                                   double r_steer, int plan_count, int plan_steps) {
    __shared__ double s_sum[256];
    SmoothState& st = *b.st;
    const double beta = st.lo;
    const bool cand = st.E >= 1 && beta > 0.0;
    double part = 0.0;
    if (cand) {
        const double T_p = st.T_p;
        for (int e = threadIdx.x; e < st.E; e += blockDim.x) {
            const double sa = b.e_t0[e] / T_p, sb = b.e_t0[e + 1] / T_p;
            const double sm = 0.5 * (sa + sb);
            const double* c = b.e_coef + (size_t)e * 12;
            double f[3];
            const double ss[3] = {sa, sm, sb};
            for (int i = 0; i < 3; ++i) {
                const double loc = ss[i] * T_p - b.e_t0[e];
                const double tq = ss[i] * st.tau_q;
                double acc = 0.0;
                for (int ax = 0; ax < 3; ++ax) {
                    const double pdd = 2.0 * c[4 * ax + 2] + 6.0 * c[4 * ax + 3] * loc;
                    const double qdd = 2.0 * st.qc[4 * ax + 2] + 6.0 * st.qc[4 * ax + 3] * tq;
                    const double v = (1.0 - beta) * T_p * T_p * pdd + beta * st.tau_q * st.tau_q * qdd;
                    acc += v * v;
                }
                f[i] = acc;
            }
            part += (sb - sa) / 6.0 * (f[0] + 4.0 * f[1] + f[2]);
        }
    }
    s_sum[threadIdx.x] = part;
    __syncthreads();
    __shared__ int s_take;
    if (threadIdx.x == 0) {
        double N = 0.0;
        for (int t = 0; t < (int)blockDim.x; ++t) N += s_sum[t];
        const double T = (1.0 - beta) * st.T_p + beta * st.tau_q;
        const double cost = cand ? T + r_steer * N / (T * T * T) : st.plan_cost;
        const int take = cand && cost < st.plan_cost;
        s_take = take;
        st.beta = take ? beta : 0.0;
        st.cost = take ? cost : st.plan_cost;
        st.count = take ? st.lo_cnt : plan_count;
        st.steps = take ? st.lo_K : plan_steps;
    }
    __syncthreads();
    const int stride = a.S_max + 1;
    if (s_take) {
        const int K = st.lo_K;
        for (int k = threadIdx.x; k <= K; k += blockDim.x) {
            double p[3];
            smooth_pos(st, b, beta, (double)k / (double)K, p);
            for (int ax = 0; ax < 3; ++ax) b.out_wp[(size_t)k * 3 + ax] = p[ax];
        }
    } else if (st.f_best >= 0 && plan_steps >= 0) {
        const double* w = a.wp + (size_t)st.f_best * stride * 3;
        for (int t = threadIdx.x; t < (plan_steps + 1) * 3; t += blockDim.x) b.out_wp[t] = w[t];
    }
}

}  // namespace pump
