// Batched engine: many planning queries of uneven size in one sequence of
// launches with no host round trips (so it can be captured in one HIP graph).
// Setup and selection run as batched kernels (the query index is a grid
// dimension); Explore runs in one persistent kernel whose workgroups pull
// whole queries from a queue and run every round of a query with block-level
// synchronisation only.  Every per-element body is shared with the
// single-query path (explore_ops.hpp, setup_ops.hpp, select_ops.hpp) and runs
// in the same orders, so each query's results equal its single-query results.
#include "explore_team.hpp"
#include "select_ops.hpp"
#include "setup_ops.hpp"
#include "roadmap_ops.hpp"
#include "smooth_ops.hpp"

namespace pump {

// Pareto-front entries kept per query: as many as the single-query path
// keeps, so a batched query's result is the one pump_plan returns; the
// certification grid has kBatchMcRows rows of front plans and strides over
// larger fronts.
constexpr int kBatchFront = kMaxFront;
constexpr int kBatchMcRows = 32;

// ----------------------------- setup ---------------------------------------
__global__ void k_b_load(BatchQuery* qs) {
    const BatchQuery& Q = qs[blockIdx.y];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = Q.n_nodes - 1;
    if (t < 6) Q.X[t] = Q.x_init[t];
    if (t < n * 6) Q.X[6 + t] = Q.samples[t];
    if (t < Q.ra[0].n_obs * 6) Q.obs[t] = Q.obs_src[t];
}

__device__ __forceinline__ DevCoef dev_coef(const BatchQuery& Q) {
    return DevCoef{Q.Acl[0], Q.Acl[1], Q.Acl[2], Q.Acl[3], Q.L[0], Q.L[2], Q.L[3]};
}

// Deviation table per query (LQR or LQG tracking; the scratch holds the chunk
// responses, then the chunk start states: 2 or 4 doubles per column each).
__global__ void k_b_dev_local(BatchQuery* qs, int S) {
    const BatchQuery& Q = qs[blockIdx.y];
    if (Q.estimator)
        lqg_local_dev(Q.noise, Q.noise_meas, Q.dev_scratch, Q.N, S, Q.lqg);
    else
        dev_local_dev(Q.noise, Q.dev_scratch, Q.N, S, dev_coef(Q));
}

__global__ void k_b_dev_carry(BatchQuery* qs, int S) {
    const BatchQuery& Q = qs[blockIdx.y];
    const int K = (S + kDevChunk - 1) / kDevChunk;
    const int per = Q.estimator ? 4 : 2;
    double* X0 = Q.dev_scratch + (size_t)per * K * 3 * Q.N;
    if (Q.estimator)
        lqg_carry_dev(Q.dev_scratch, X0, Q.N, S, Q.lqg);
    else
        dev_carry_dev(Q.dev_scratch, X0, Q.N, S, dev_coef(Q));
}

__global__ void k_b_dev_final(BatchQuery* qs, int S) {
    const BatchQuery& Q = qs[blockIdx.y];
    const int K = (S + kDevChunk - 1) / kDevChunk;
    const int per = Q.estimator ? 4 : 2;
    const double* X0 = Q.dev_scratch + (size_t)per * K * 3 * Q.N;
    float* D = const_cast<float*>(Q.ra[0].D);
    if (Q.estimator)
        lqg_final_dev(Q.noise, Q.noise_meas, X0, D, Q.N, S, Q.lqg);
    else
        dev_final_dev(Q.noise, X0, D, Q.N, S, dev_coef(Q));
}

__global__ void k_b_cloud(BatchQuery* qs) {
    const BatchQuery& Q = qs[blockIdx.y];
    cloud_dev(Q.ra[0].D, const_cast<float*>(Q.ra[0].cloud), Q.N);
}

__global__ void k_b_gcloud(BatchQuery* qs, int S1) {
    const BatchQuery& Q = qs[blockIdx.y];
    gcloud_dev(Q.ra[0].cloud, const_cast<float*>(Q.ra[0].gcloud), S1);
}

__global__ void k_b_valid(BatchQuery* qs) {
    BatchQuery& Q = qs[blockIdx.y];
    const float* g = Q.goal_box;
    mark_valid_dev(Q.X, Q.n_nodes, Q.obs, Q.ra[0].n_obs, g[0], g[1], g[2], g[3], g[4], g[5], Q.valid,
                   Q.goal, &Q.bad);
}

// BuildGraph pass 1 stages per query (setup_ops.hpp); the work lists live in
// the query's Explore candidate arrays, the counters in its descriptor.
__device__ __forceinline__ GraphWork graph_work(BatchQuery& Q) {
    const RoundArgs& a = Q.ra[0];
    return GraphWork{Q.esrc, Q.col, Q.etau, a.c_pop, a.c_pos, Q.gcount, Q.cap_edges, Q.cap_pairs};
}

__global__ __launch_bounds__(256) void k_b_zero_ebits(BatchQuery* qs) {
    const BatchQuery& Q = qs[blockIdx.y];
    const size_t n = (size_t)Q.n_nodes * Q.words;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (size_t)gridDim.x * blockDim.x)
        Q.ebits[t] = 0u;
}

// With a cached roadmap only row 0 and column 0 (the pairs at x_init) are
// steered here; the cached connections go through k_b_gw_boxes_rm.
__global__ __launch_bounds__(256) void k_b_rm_check(BatchQuery* qs) {
    BatchQuery& Q = qs[blockIdx.y];
    if (Q.use_rm) rm_check_dev(Q.X, Q.rm.X, Q.n_nodes, &Q.bad, 1);
}

__global__ __launch_bounds__(256) void k_b_gw_near_col0(BatchQuery* qs) {
    BatchQuery& Q = qs[blockIdx.y];
    if (!Q.use_rm) return;
    gw_near_col0(Q.X, Q.valid, Q.n_nodes, blockIdx.x * blockDim.x + threadIdx.x, Q.r_steer, Q.r_conn,
                 graph_work(Q));
}

__global__ __launch_bounds__(kBoxThreads, 3) void k_b_gw_boxes_rm(BatchQuery* qs) {
    __shared__ float s_obs[kMaxObs * 6];
    __shared__ uint32_t s_q[kBoxThreads / 64 * kBoxQueue];
    __shared__ int s_src[kBoxThreads], s_dst[kBoxThreads], s_blk[kBoxThreads];
    __shared__ double s_tau[kBoxThreads];
    __shared__ BoxBins s_bins;
    BatchQuery& Q = qs[blockIdx.y];
    if (!Q.use_rm) return;
    const int n_obs = Q.ra[0].n_obs;
    for (int t = threadIdx.x; t < n_obs * 6; t += blockDim.x) s_obs[t] = Q.obs[t];
    __syncthreads();
    box_bins_build(s_obs, n_obs, &s_bins);
    gw_boxes(Q.X, Q.valid, Q.rm.esrc, Q.rm.col, Q.rm.tau, Q.rm.bbox, Q.rm.n_edges, false, true,
             s_obs, n_obs, &s_bins, graph_work(Q), Q.ebits, Q.words, blockIdx.x * blockDim.x + threadIdx.x,
             gridDim.x * blockDim.x, s_q, s_src, s_dst, s_tau, s_blk);
}

__global__ __launch_bounds__(kNearThreads) void k_b_gw_near_rows(BatchQuery* qs) {
    __shared__ int s_list[2 * kNearChunk];
    __shared__ int s_cnt[3 + 17];
    BatchQuery& Q = qs[blockIdx.y];
    if ((int)blockIdx.x >= Q.n_nodes || (Q.use_rm && blockIdx.x > 0)) return;
    gw_near_row(Q.X, Q.valid, Q.n_nodes, blockIdx.x, Q.r_steer, Q.r_conn, graph_work(Q), s_list,
                s_cnt);
}

__global__ __launch_bounds__(kBoxThreads, 3) void k_b_gw_boxes(BatchQuery* qs) {
    __shared__ float s_obs[kMaxObs * 6];
    __shared__ uint32_t s_q[kBoxThreads / 64 * kBoxQueue];
    __shared__ int s_src[kBoxThreads], s_dst[kBoxThreads], s_blk[kBoxThreads];
    __shared__ double s_tau[kBoxThreads];
    __shared__ BoxBins s_bins;
    BatchQuery& Q = qs[blockIdx.y];
    const int n_obs = Q.ra[0].n_obs;
    for (int t = threadIdx.x; t < n_obs * 6; t += blockDim.x) s_obs[t] = Q.obs[t];
    __syncthreads();
    box_bins_build(s_obs, n_obs, &s_bins);
    const GraphWork gw = graph_work(Q);
    gw_boxes(Q.X, Q.valid, gw.near_src, gw.near_dst, gw.near_tau, nullptr,
             min(gw.counts[0], gw.near_cap), true, false, s_obs, n_obs, &s_bins, gw, Q.ebits, Q.words,
             blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x, s_q, s_src, s_dst,
             s_tau, s_blk);
}

__global__ __launch_bounds__(256) void k_b_gw_exact(BatchQuery* qs) {
    BatchQuery& Q = qs[blockIdx.y];
    gw_exact(Q.X, Q.obs, graph_work(Q), Q.rm.esrc, Q.rm.col, Q.rm.tau, Q.ebits, Q.words,
             blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

__global__ __launch_bounds__(256) void k_b_row_deg(BatchQuery* qs) {
    const BatchQuery& Q = qs[blockIdx.y];
    row_deg_dev(Q.ebits, Q.n_nodes, Q.words, Q.deg,
                blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
}

// exclusive scan of arr_in[0..n) into arr_out (may alias), whole block;
// returns the total
__device__ int block_scan(const int32_t* in, int32_t* out, int n, int* s_w) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    int carry = 0;
    for (int b0 = 0; b0 < n; b0 += blockDim.x) {
        const int i = b0 + tid;
        const int v = i < n ? in[i] : 0;
        int x = v;
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) s_w[wave] = x;
        __syncthreads();
        int off = 0, tot = 0;
        for (int w = 0; w < nw; ++w) {
            if (w < wave) off += s_w[w];
            tot += s_w[w];
        }
        if (i < n) out[i] = carry + off + x - v;
        carry += tot;
        __syncthreads();
    }
    return carry;
}

__global__ __launch_bounds__(1024) void k_b_row_scan(BatchQuery* qs) {
    __shared__ int s_w[16];
    BatchQuery& Q = qs[blockIdx.x];
    const int total = block_scan(Q.deg, Q.row_ptr, Q.n_nodes, s_w);
    if (threadIdx.x == 0) {
        Q.row_ptr[Q.n_nodes] = total;
        if (total > Q.cap_edges) atomicOr(&Q.bad, 4);
        if (Q.gcount[0] > Q.cap_edges || Q.gcount[1] > Q.cap_pairs) atomicOr(&Q.bad, 4);
    }
}

// pass 2 without steering again (setup_ops.hpp): the near list's tau* go to
// their CSR slots before the fill overwrites the list; a cached roadmap's
// edges take theirs from the roadmap instead
__global__ __launch_bounds__(256) void k_b_word_start(BatchQuery* qs) {
    const BatchQuery& Q = qs[blockIdx.y];
    if (Q.bad || Q.use_rm) return;
    word_start_dev(Q.n_nodes, Q.ebits, Q.row_ptr, Q.wstart, Q.words);
}

__global__ __launch_bounds__(256) void k_b_near_to_slot(BatchQuery* qs) {
    BatchQuery& Q = qs[blockIdx.y];
    if (Q.bad || Q.use_rm) return;
    near_to_slot_dev(graph_work(Q), Q.ebits, Q.wstart, Q.words, Q.ecost);
}

__global__ __launch_bounds__(256) void k_b_graph_fill(BatchQuery* qs) {
    const BatchQuery& Q = qs[blockIdx.y];
    if (Q.bad) return;
    graph_fill_dev(Q.n_nodes, Q.ebits, Q.row_ptr, Q.col, Q.esrc, Q.words);
}

__global__ __launch_bounds__(256) void k_b_edge_cost(BatchQuery* qs) {
    const BatchQuery& Q = qs[blockIdx.y];
    if (Q.bad) return;
    if (Q.use_rm)
        rm_fill_dev(Q.X, Q.n_nodes, Q.r_steer, Q.row_ptr, Q.col, Q.esrc, Q.rm, Q.etau, Q.ecost);
    else
        edge_cost_dev(Q.X, Q.n_nodes, Q.r_steer, Q.row_ptr, Q.col, Q.esrc, Q.etau, Q.ecost);
}

// ----------------------------- explore --------------------------------------
// Persistent kernel: every workgroup pops a slot of the schedule; slot k
// belongs to entry e (off[e] <= k < off[e + 1]), whose query is planned by
// the team of workgroups holding its slots (explore_team.hpp).  Slots are
// popped in order, so a team whose first member waits for the others only
// waits for slots that running workgroups will pop after their current work;
// with every workgroup resident (the launch is sized by occupancy) the queue
// drains.  A query's team sync words and totals were zeroed by k_b_reset.
// One kernel per particle count N (a schedule holds only queries of that N),
// so each gets the registers its own N needs: two workgroups of 256 per CU
// fit for N <= 128, one for N = 256.
template <int N>
__global__ __launch_bounds__(256, 2) void k_b_explore(BatchQuery* qs, BatchSched sch,
                                                                    int* counter, BatchOut* outs) {
    __shared__ float s_raw[kMaxObs * 6];
    __shared__ float s_in[kMaxObs * 6];
    __shared__ float s_out[kMaxObs * 6];
    __shared__ int s_w[16];
    __shared__ unsigned long long s_m[16];
    __shared__ long long s_ll[16];
    __shared__ int s_fail;
    __shared__ int s_next;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_next = atomicAdd(counter, 1);
        __syncthreads();
        const int k = s_next;
        if (k >= sch.total) break;
        int lo = 0, hi = sch.n_entries;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (sch.off[mid] <= k) lo = mid; else hi = mid;
        }
        const int qi = sch.query[lo];
        const BatchQuery& Q = qs[qi];
        TeamCtx t;
        t.rank = k - sch.off[lo];
        t.size = sch.off[lo + 1] - sch.off[lo];
        if (Q.bad) {
            if (t.rank == 0 && threadIdx.x == 0) outs[qi].err = -1;
            continue;
        }
        t.release = Q.team_sync;
        t.fail = reinterpret_cast<int*>(Q.team_sync + 1);
        t.patience = kDefaultPatience;
        t.arrive = Q.team_sync + 64;
        t.xa = Q.team_tot;
        t.xb = Q.team_tot + kMaxTeam;
        t.b_deg = Q.b_deg;
        t.open_cur = Q.open_a;
        t.open_next = Q.open_b;
        t.cap_pairs = Q.cap_pairs;
        explore_team<N>(Q.ra, t, true, Q.n_nodes, s_raw, s_in, s_out, s_w, s_m, s_ll, &s_fail);
        if (t.rank == 0 && threadIdx.x == 0) {
            const Ctl* c = Q.ra[0].ctl;
            BatchOut& o = outs[qi];
            o.rounds = c->rounds;
            o.partial_plans = c->partial;
            o.final_i = c->i;
            o.err = c->err;
            o.n_plans = c->n_plans;
        }
    }
}

// ----------------------------- selection ------------------------------------
__device__ __forceinline__ SelectArgs select_of(const BatchQuery& Q) {
    SelectArgs s = Q.s;
    s.n_plans = Q.ra[0].ctl->n_plans;
    return s;
}

__global__ __launch_bounds__(1024) void k_b_goal_collect(BatchQuery* qs) {
    const BatchQuery& Q = qs[blockIdx.x];
    if (Q.bad || Q.ra[0].ctl->err) return;
    goal_collect_block(select_of(Q));
}

__global__ __launch_bounds__(256) void k_b_front(BatchQuery* qs) {
    const BatchQuery& Q = qs[blockIdx.x];
    if (Q.bad || Q.ra[0].ctl->err) return;
    front_block(select_of(Q), kBatchFront);
}

__global__ void k_b_waypoints(BatchQuery* qs) {
    const BatchQuery& Q = qs[blockIdx.x];
    for (int f = threadIdx.x; f < kBatchFront; f += blockDim.x) Q.s.mc_counts[f] = 0;
    if (Q.bad || Q.ra[0].ctl->err) return;
    const int nf = Q.ra[0].ctl->n_front;
    for (int f = threadIdx.x; f < nf; f += blockDim.x) waypoints_one(Q.s, f);
}

__global__ __launch_bounds__(kMcThreads) void k_b_mc(BatchQuery* qs) {
    __shared__ float s_obs[kMaxObs * 6];
    __shared__ int s_hit[kMcParticles];
    const BatchQuery& Q = qs[blockIdx.z];
    if (Q.bad || Q.ra[0].ctl->err || (int)blockIdx.y >= Q.ra[0].ctl->n_front) return;   // uniform per block
    const int nf = Q.ra[0].ctl->n_front;
    for (int t = threadIdx.x; t < Q.s.n_obs * 6; t += blockDim.x) s_obs[t] = Q.s.obs[t];
    __syncthreads();
    for (int f = blockIdx.y; f < nf; f += gridDim.y) {   // trip count uniform per block
        mc_block_count(Q.s, Q.s.wp + (size_t)f * (Q.s.S_max + 1) * 3, Q.s.wp_len[f],
                       blockIdx.x * kMcParticles, s_obs, s_hit, &Q.s.mc_counts[f]);
        __syncthreads();   // the next plan's clear of s_hit waits for this plan's ballot
    }
}

// Alg. 5 bisection on the certified counts, and the per-query outcome.
__global__ void k_b_finalize(BatchQuery* qs, int q, BatchOut* outs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= q) return;
    const BatchQuery& Q = qs[i];
    BatchOut& o = outs[i];
    const Ctl* c = Q.ra[0].ctl;
    o.bad = Q.bad;
    o.best = -1;
    o.best_plan = -1;
    o.n_edges = Q.row_ptr[Q.n_nodes];
    if (Q.bad) {
        o.status = (Q.bad & 4) ? PUMP_E_CAPACITY : PUMP_E_ARG;
        return;
    }
    if (c->err) {
        o.status = (c->err == 3 || c->err >= 5) ? PUMP_E_STATE : PUMP_E_CAPACITY;
        return;
    }
    o.n_goal = c->n_goal;
    o.n_front = c->n_front;
    if (c->n_goal > kMaxGoal) {
        o.status = PUMP_E_CAPACITY;
        return;
    }
    if (c->n_goal == 0) {
        o.status = PUMP_NO_GOAL_PLAN;
        return;
    }
    const int nf = c->n_front;
    for (int f = 0; f < nf; ++f)
        if (Q.s.wp_len[f] < 0) {   // a front plan longer than max_steps
            o.status = PUMP_E_STATE;
            return;
        }
    const int M = Q.s.M;
    const int k = certified_pick(Q.s.mc_counts, nf, M, Q.alpha);
    if (k < 0) {
        o.status = PUMP_INFEASIBLE;
        return;
    }
    const int p = Q.s.front_ids[k];
    o.status = PUMP_OK;
    o.best = k;
    o.best_plan = p;
    o.best_pop = Q.ra[0].p_pop[p];
    o.best_mc = Q.s.mc_counts[k];
    o.best_len = Q.s.path_len[k];
    o.best_cost = Q.ra[0].p_cost[p];
    o.best_cp_mc = (double)o.best_mc / (double)M;
    // the identity Smooth (replaced when smoothing runs)
    o.smooth_beta = 0.0;
    o.smooth_cost = o.best_cost;
    o.smooth_count = o.best_mc;
    o.smooth_steps = Q.s.wp_len[k];
}

// Smooth(p*, alpha) per query (smooth_ops.hpp), after the outcome records:
// queries without a certified plan keep beta = 0.
__global__ __launch_bounds__(256) void k_b_smooth_prep(BatchQuery* qs, const BatchOut* outs) {
    const BatchQuery& Q = qs[blockIdx.x];
    const BatchOut& o = outs[blockIdx.x];
    const int f = o.status == PUMP_OK ? o.best : -1;
    smooth_prep_block(Q.s, f, f >= 0 ? o.best_cost : 0.0, Q.sm);
}

__global__ __launch_bounds__(256) void k_b_smooth_wp(BatchQuery* qs, int r) {
    const BatchQuery& Q = qs[blockIdx.z];
    smooth_wp_one(Q.s, Q.sm, r, blockIdx.y, blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(kMcThreads) void k_b_smooth_mc(BatchQuery* qs, int r) {
    __shared__ float s_obs[kMaxObs * 6];
    __shared__ int s_hit[kMcParticles];
    const BatchQuery& Q = qs[blockIdx.z];
    const int c = blockIdx.y;
    if (smooth_beta(*Q.sm.st, r, c) < 0.0 || Q.sm.st->K[c] < 0) return;   // uniform per block
    for (int t = threadIdx.x; t < Q.s.n_obs * 6; t += blockDim.x) s_obs[t] = Q.s.obs[t];
    __syncthreads();
    mc_block_count(Q.s, Q.sm.wp + (size_t)c * (Q.s.S_max + 1) * 3, Q.sm.st->K[c],
                   blockIdx.x * kMcParticles, s_obs, s_hit, &Q.sm.st->cnt[c]);
}

__global__ void k_b_smooth_resolve(BatchQuery* qs, int q, int r) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < q) smooth_resolve_one(qs[i].s, qs[i].alpha, qs[i].sm, r);
}

__global__ __launch_bounds__(256) void k_b_smooth_final(BatchQuery* qs, BatchOut* outs) {
    const BatchQuery& Q = qs[blockIdx.x];
    BatchOut& o = outs[blockIdx.x];
    const bool ok = o.status == PUMP_OK;
    smooth_final_block(Q.s, Q.sm, Q.r_steer, ok ? o.best_mc : 0, ok ? Q.s.wp_len[o.best] : -1);
    __syncthreads();
    if (threadIdx.x == 0 && ok) {
        o.smooth_beta = Q.sm.st->beta;
        o.smooth_cost = Q.sm.st->cost;
        o.smooth_count = Q.sm.st->count;
        o.smooth_steps = Q.sm.st->steps;
    }
}

// Queue counters and every query's team barrier words and totals to zero.
__global__ void k_b_reset(BatchQuery* qs, int* counter) {
    const BatchQuery& Q = qs[blockIdx.x];
    if (threadIdx.x < kBatchGroups && blockIdx.x == 0) counter[threadIdx.x] = 0;
    for (int t = threadIdx.x; t < 64 + kMaxTeam; t += blockDim.x) Q.team_sync[t] = 0u;
    for (int t = threadIdx.x; t < 2 * kMaxTeam; t += blockDim.x) Q.team_tot[t] = 0ull;
}

void launch_batch(hipStream_t s, BatchQuery* qs, int q, int N_max, int max_nodes, int S_max, int M,
                  int words, int explore_threads, int* counter, BatchOut* out,
                  const BatchGroup* groups, int n_groups, bool smooth) {
    const int max_elems = std::max(max_nodes * 6, kMaxObs * 6);
    k_b_load<<<dim3((max_elems + 255) / 256, q), 256, 0, s>>>(qs);
    {
        const int K = (S_max + kDevChunk - 1) / kDevChunk;
        const int threads = K * 3 * N_max;
        k_b_dev_local<<<dim3((threads + 255) / 256, q), 256, 0, s>>>(qs, S_max);
        k_b_dev_carry<<<dim3((3 * N_max + 63) / 64, q), 64, 0, s>>>(qs, S_max);
        k_b_dev_final<<<dim3((threads + 255) / 256, q), 256, 0, s>>>(qs, S_max);
    }
    k_b_cloud<<<dim3(S_max + 1, q), 256, 0, s>>>(qs);
    k_b_gcloud<<<dim3(1, q), 256, 0, s>>>(qs, S_max + 1);
    const int vmax = std::max(max_nodes, kMaxObs);
    k_b_valid<<<dim3((vmax + 255) / 256, q), 256, 0, s>>>(qs);
    k_b_zero_ebits<<<dim3(256, q), 256, 0, s>>>(qs);
    k_b_rm_check<<<dim3((max_nodes * 6 + 255) / 256, q), 256, 0, s>>>(qs);
    k_b_gw_near_rows<<<dim3(max_nodes, q), kNearThreads, 0, s>>>(qs);
    k_b_gw_near_col0<<<dim3((max_nodes + 255) / 256, q), 256, 0, s>>>(qs);
    k_b_gw_boxes<<<dim3(256, q), kBoxThreads, 0, s>>>(qs);
    k_b_gw_boxes_rm<<<dim3(256, q), kBoxThreads, 0, s>>>(qs);
    k_b_gw_exact<<<dim3(64, q), 256, 0, s>>>(qs);
    k_b_row_deg<<<dim3((max_nodes + 3) / 4, q), 256, 0, s>>>(qs);
    k_b_row_scan<<<q, 1024, 0, s>>>(qs);
    k_b_word_start<<<dim3((max_nodes + 3) / 4, q), 256, 0, s>>>(qs);
    k_b_near_to_slot<<<dim3(256, q), 256, 0, s>>>(qs);
    k_b_graph_fill<<<dim3((max_nodes + 3) / 4, q), 256, 0, s>>>(qs);
    k_b_edge_cost<<<dim3(256, q), 256, 0, s>>>(qs);
    k_b_reset<<<q, 64, 0, s>>>(qs, counter);
    for (int g = 0; g < n_groups; ++g) {
        const BatchGroup& G = groups[g];
        int* ctr = counter + g;
        switch (G.N) {
            case 32: k_b_explore<32><<<G.blocks, explore_threads, 0, s>>>(qs, G.sch, ctr, out); break;
            case 64: k_b_explore<64><<<G.blocks, explore_threads, 0, s>>>(qs, G.sch, ctr, out); break;
            case 128: k_b_explore<128><<<G.blocks, explore_threads, 0, s>>>(qs, G.sch, ctr, out); break;
            default: k_b_explore<256><<<G.blocks, explore_threads, 0, s>>>(qs, G.sch, ctr, out); break;
        }
    }
    k_b_goal_collect<<<q, 1024, 0, s>>>(qs);
    k_b_front<<<q, 256, 0, s>>>(qs);
    k_b_waypoints<<<q, 64, 0, s>>>(qs);
    k_b_mc<<<dim3((M + kMcParticles - 1) / kMcParticles, kBatchMcRows, q), kMcThreads, 0, s>>>(qs);
    k_b_finalize<<<(q + 63) / 64, 64, 0, s>>>(qs, q, out);
    if (smooth) {
        k_b_smooth_prep<<<q, 256, 0, s>>>(qs, out);
        for (int r = 0; r < kSmoothRounds; ++r) {
            k_b_smooth_wp<<<dim3((S_max + 1 + 255) / 256, kSmoothCands, q), 256, 0, s>>>(qs, r);
            k_b_smooth_mc<<<dim3((M + kMcParticles - 1) / kMcParticles, kSmoothCands, q), kMcThreads,
                            0, s>>>(qs, r);
            k_b_smooth_resolve<<<(q + 63) / 64, 64, 0, s>>>(qs, q, r);
        }
        k_b_smooth_final<<<q, 256, 0, s>>>(qs, out);
    }
}

int batch_explore_per_cu(int N, int threads) {
    const void* fn;
    switch (N) {
        case 32: fn = (const void*)k_b_explore<32>; break;
        case 64: fn = (const void*)k_b_explore<64>; break;
        case 128: fn = (const void*)k_b_explore<128>; break;
        default: fn = (const void*)k_b_explore<256>; break;
    }
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, threads, 0) != hipSuccess) return 0;
    return n;
}

}  // namespace pump
