// PlanSelection (Alg. 5): gather P_goal, reduce it to its Pareto front, sort
// by cp_hat, and certify with Monte Carlo (MC(p), Sec. IV).  The bodies live
// in select_ops.hpp.
#include "select_ops.hpp"
#include "smooth_ops.hpp"

namespace pump {

__global__ __launch_bounds__(1024) void k_goal_collect(SelectArgs a) { goal_collect_block(a); }

__global__ __launch_bounds__(256) void k_front(SelectArgs a) { front_block(a, kMaxFront); }

void launch_select_front(hipStream_t s, const SelectArgs& a) {
    k_goal_collect<<<1, 1024, 0, s>>>(a);
    k_front<<<1, 256, 0, s>>>(a);
}

__global__ void k_waypoints(SelectArgs a, int n_paths) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f < n_paths) waypoints_one(a, f);
}

void launch_waypoints(hipStream_t s, const SelectArgs& a, int32_t n_paths) {
    k_waypoints<<<(n_paths + 63) / 64, 64, 0, s>>>(a, n_paths);
}

__global__ __launch_bounds__(kMcThreads) void k_mc(SelectArgs a) {
    __shared__ float s_obs[kMaxObs * 6];
    __shared__ int s_hit[kMcParticles];
    for (int t = threadIdx.x; t < a.n_obs * 6; t += blockDim.x) s_obs[t] = a.obs[t];
    __syncthreads();
    const int f = blockIdx.y;
    mc_block_count(a, a.wp + (size_t)f * (a.S_max + 1) * 3, a.wp_len[f], blockIdx.x * kMcParticles,
                   s_obs, s_hit, &a.mc_counts[f]);
}

void launch_mc(hipStream_t s, const SelectArgs& a, int32_t n_paths) {
    if (n_paths <= 0) return;
    dim3 grid((a.M + kMcParticles - 1) / kMcParticles, n_paths);
    k_mc<<<grid, kMcThreads, 0, s>>>(a);
}

// ---- Smooth(p*, alpha) ----
__global__ __launch_bounds__(256) void k_smooth_prep(SelectArgs a, SmoothBuf b, int f_best,
                                                     const double* plan_cost) {
    smooth_prep_block(a, f_best, f_best >= 0 ? *plan_cost : 0.0, b);
}

__global__ __launch_bounds__(256) void k_smooth_wp(SelectArgs a, SmoothBuf b, int r) {
    smooth_wp_one(a, b, r, blockIdx.y, blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(kMcThreads) void k_smooth_mc(SelectArgs a, SmoothBuf b, int r) {
    __shared__ float s_obs[kMaxObs * 6];
    __shared__ int s_hit[kMcParticles];
    const int c = blockIdx.y;
    if (smooth_beta(*b.st, r, c) < 0.0 || b.st->K[c] < 0) return;   // uniform per block
    for (int t = threadIdx.x; t < a.n_obs * 6; t += blockDim.x) s_obs[t] = a.obs[t];
    __syncthreads();
    mc_block_count(a, b.wp + (size_t)c * (a.S_max + 1) * 3, b.st->K[c], blockIdx.x * kMcParticles,
                   s_obs, s_hit, &b.st->cnt[c]);
}

__global__ void k_smooth_resolve(SelectArgs a, SmoothBuf b, double alpha, int r) {
    if (threadIdx.x == 0) smooth_resolve_one(a, alpha, b, r);
}

__global__ __launch_bounds__(256) void k_smooth_final(SelectArgs a, SmoothBuf b, int plan_count,
                                                      int plan_steps) {
    smooth_final_block(a, b, a.r_steer, plan_count, plan_steps);
}

void launch_smooth(hipStream_t s, const SelectArgs& a, const SmoothBuf& b, int f_best,
                   const double* plan_cost, double alpha, int plan_count, int plan_steps) {
    k_smooth_prep<<<1, 256, 0, s>>>(a, b, f_best, plan_cost);
    for (int r = 0; r < kSmoothRounds; ++r) {
        k_smooth_wp<<<dim3((a.S_max + 1 + 255) / 256, kSmoothCands), 256, 0, s>>>(a, b, r);
        k_smooth_mc<<<dim3((a.M + kMcParticles - 1) / kMcParticles, kSmoothCands), kMcThreads, 0,
                      s>>>(a, b, r);
        k_smooth_resolve<<<1, 64, 0, s>>>(a, b, alpha, r);
    }
    k_smooth_final<<<1, 256, 0, s>>>(a, b, plan_count, plan_steps);
}

}  // namespace pump
