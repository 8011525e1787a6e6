// PlanSelection (Alg. 5): gather P_goal, reduce it to its Pareto front, sort
// by cp_hat, and certify with Monte Carlo (MC(p), Sec. IV).  The bodies live
// in select_ops.hpp.
#include "select_ops.hpp"
#include "smooth_ops.hpp"

namespace pump {

// P_goal and its sorted Pareto front in one workgroup (the front reads the
// goal count thread 0 stored, after the workgroup barrier).
__global__ __launch_bounds__(1024) void k_goal_front(SelectArgs a) {
    for (int f = threadIdx.x; f < kMaxFront; f += blockDim.x) a.mc_counts[f] = 0;
    goal_collect_block(a);
    __syncthreads();
    front_block(a, kMaxFront);
}

// The same with P_goal gathered by the whole device (plan stores of many
// plans): flags, an exclusive scan over them in plan order, a scatter; the
// goal list is the one goal_collect_block writes.
__device__ __forceinline__ bool is_goal_plan(const SelectArgs& a, int p) {
    return a.p_state[p] != kRemoved && a.goal[a.p_head[p]];
}

__global__ __launch_bounds__(256) void k_goal_flags(SelectArgs a, int32_t* flag) {
    const int n = a.ctl->n_plans;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x)
        flag[p] = is_goal_plan(a, p) ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_goal_scatter(SelectArgs a, const int32_t* pos) {
    const int n = a.ctl->n_plans;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x)
        if (is_goal_plan(a, p) && pos[p] < kMaxGoal) a.goal_ids[pos[p]] = p;
}

__global__ __launch_bounds__(1024) void k_front(SelectArgs a) {
    for (int f = threadIdx.x; f < kMaxFront; f += blockDim.x) a.mc_counts[f] = 0;
    front_block(a, kMaxFront);
}

// Below this many plans (or when the count is not known on the host) one
// workgroup gathers P_goal; from it on the device-wide gather is faster.
constexpr int32_t kGoalGatherWide = 1 << 14;

void launch_select_front(hipStream_t s, const SelectArgs& a, int32_t* scratch, int32_t* blk) {
    if (a.n_plans < kGoalGatherWide) {
        k_goal_front<<<1, 1024, 0, s>>>(a);
        return;
    }
    int b = (a.n_plans + 255) / 256;
    if (b > 4096) b = 4096;
    k_goal_flags<<<b, 256, 0, s>>>(a, scratch);
    scan_exclusive(s, scratch, scratch, &a.ctl->n_plans, a.n_plans, &a.ctl->n_goal, blk);
    k_goal_scatter<<<b, 256, 0, s>>>(a, scratch);
    k_front<<<1, 1024, 0, s>>>(a);
}

// One wave per path (waypoints_wave).
__global__ __launch_bounds__(64) void k_waypoints(SelectArgs a, int n_paths) {
    const int n = n_paths < 0 ? a.ctl->n_front : n_paths;
    const int f = blockIdx.x;
    if (f < n) waypoints_wave(a, f);
}

void launch_waypoints(hipStream_t s, const SelectArgs& a, int32_t n_paths) {
    const int n = n_paths < 0 ? kMaxFront : n_paths;
    if (n <= 0) return;
    k_waypoints<<<n, 64, 0, s>>>(a, n_paths);
}

// Rows of the MC grid when the front size is read on the device: each row
// of workgroups takes front plans blockIdx.y, + kMcRows, ...
constexpr int kMcRows = 16;

__global__ __launch_bounds__(kMcThreads) void k_mc(SelectArgs a, int n_paths) {
    __shared__ float s_obs[kMaxObs * 6];
    __shared__ int s_hit[kMcParticles];
    const int n = n_paths < 0 ? a.ctl->n_front : n_paths;
    if ((int)blockIdx.y >= n) return;   // uniform per workgroup
    for (int t = threadIdx.x; t < a.n_obs * 6; t += blockDim.x) s_obs[t] = a.obs[t];
    __syncthreads();
    for (int f = blockIdx.y; f < n; f += gridDim.y) {
        mc_block_count(a, a.wp + (size_t)f * (a.S_max + 1) * 3, a.wp_len[f],
                       blockIdx.x * kMcParticles, s_obs, s_hit, &a.mc_counts[f]);
        __syncthreads();   // s_hit is reused by the next plan
    }
}

void launch_mc(hipStream_t s, const SelectArgs& a, int32_t n_paths) {
    if (n_paths == 0) return;
    const int rows = n_paths < 0 ? kMcRows : n_paths;
    dim3 grid((a.M + kMcParticles - 1) / kMcParticles, rows);
    k_mc<<<grid, kMcThreads, 0, s>>>(a, n_paths);
}

// Alg. 5: with the front sorted by cp_hat, bisect (1-based m) on
// MC(P_m) > alpha for the last plan certified below alpha; every front plan
// must fit S_max steps.  One workgroup; thread 0 decides.
__global__ __launch_bounds__(256) void k_select_final(SelectArgs a, double alpha) {
    __shared__ int s_w[4];
    int nv = 0;
    for (int v = threadIdx.x; v < a.n_nodes; v += blockDim.x) nv += a.valid[v] ? 1 : 0;
    for (int o = 32; o > 0; o >>= 1) nv += __shfl_down(nv, o, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = nv;
    __syncthreads();
    if (threadIdx.x != 0) return;
    Ctl* c = a.ctl;
    c->n_valid = s_w[0] + s_w[1] + s_w[2] + s_w[3];
    c->sel_best = -1;
    c->sel_plan = -1;
    c->sel_bad_wp = 0;
    const int nf = c->n_front;
    if (c->n_goal == 0 || nf <= 0) {
        c->sel_status = PUMP_NO_GOAL_PLAN;
        return;
    }
    for (int f = 0; f < nf; ++f)
        if (a.wp_len[f] < 0) c->sel_bad_wp = 1;
    const int k = certified_pick(a.mc_counts, nf, a.M, alpha);
    if (k < 0) {
        c->sel_status = PUMP_INFEASIBLE;
        return;
    }
    const int id = a.front_ids[k];
    c->sel_status = PUMP_OK;
    c->sel_best = k;
    c->sel_plan = id;
    c->sel_mc = a.mc_counts[k];
    c->sel_len = a.path_len[k];
    c->sel_steps = a.wp_len[k];
    c->sel_pop = a.p_pop[id];
    c->sel_cost = a.p_cost[id];
}

void launch_select_final(hipStream_t s, const SelectArgs& a, double alpha) {
    k_select_final<<<1, 256, 0, s>>>(a, alpha);
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
