// Batched engine: many planning queries of uneven size in one sequence of
// launches with no host round trips (so it can be captured in one HIP graph).
// Setup and selection run as batched kernels (the query index is a grid
// dimension); Explore runs in one persistent kernel whose workgroups pull
// whole queries from a queue and run every round of a query with block-level
// synchronisation only.  Every per-element body is shared with the
// single-query path (explore_ops.hpp, setup_ops.hpp, select_ops.hpp) and runs
// in the same orders, so each query's results equal its single-query results.
#include "explore_ops.hpp"
#include "select_ops.hpp"
#include "setup_ops.hpp"

namespace pump {

constexpr int kBatchFront = 32;   // Pareto-front entries certified per query

// ----------------------------- setup ---------------------------------------
__global__ void k_b_load(BatchQuery* qs) {
    const BatchQuery& Q = qs[blockIdx.y];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = Q.n_nodes - 1;
    if (t < 6) Q.X[t] = Q.x_init[t];
    if (t < n * 6) Q.X[6 + t] = Q.samples[t];
    if (t < Q.a.n_obs * 6) Q.obs[t] = Q.obs_src[t];
}

__global__ void k_b_deviation(BatchQuery* qs, int S) {
    const BatchQuery& Q = qs[blockIdx.y];
    deviation_dev(Q.noise, const_cast<float*>(Q.a.D), Q.N, S, Q.Acl[0], Q.Acl[1], Q.Acl[2],
                  Q.Acl[3], Q.L[0], Q.L[2], Q.L[3]);
}

__global__ void k_b_cloud(BatchQuery* qs) {
    const BatchQuery& Q = qs[blockIdx.y];
    cloud_dev(Q.a.D, const_cast<float*>(Q.a.cloud), Q.N);
}

__global__ void k_b_gcloud(BatchQuery* qs, int S1) {
    const BatchQuery& Q = qs[blockIdx.y];
    gcloud_dev(Q.a.cloud, const_cast<float*>(Q.a.gcloud), S1);
}

__global__ void k_b_valid(BatchQuery* qs) {
    BatchQuery& Q = qs[blockIdx.y];
    const float* g = Q.goal_box;
    mark_valid_dev(Q.X, Q.n_nodes, Q.obs, Q.a.n_obs, g[0], g[1], g[2], g[3], g[4], g[5], Q.valid,
                   Q.goal, &Q.bad);
}

__global__ __launch_bounds__(256) void k_b_graph_mark(BatchQuery* qs) {
    const BatchQuery& Q = qs[blockIdx.y];
    if ((int)blockIdx.x >= Q.n_nodes) return;
    graph_mark_dev(Q.X, Q.valid, Q.n_nodes, Q.obs, Q.a.n_obs, Q.r_steer, Q.r_conn, Q.ebits, Q.deg,
                   Q.words);
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
    }
}

__global__ __launch_bounds__(256) void k_b_graph_fill(BatchQuery* qs) {
    const BatchQuery& Q = qs[blockIdx.y];
    if (Q.bad) return;
    graph_fill_dev(Q.n_nodes, Q.ebits, Q.row_ptr, Q.col, Q.esrc, Q.words);
}

__global__ __launch_bounds__(256) void k_b_edge_steer(BatchQuery* qs) {
    const BatchQuery& Q = qs[blockIdx.y];
    if (Q.bad) return;
    edge_steer_dev(Q.X, Q.n_nodes, Q.r_steer, Q.row_ptr, Q.col, Q.esrc, Q.etau, Q.ecost);
}

// ----------------------------- explore --------------------------------------
__device__ __forceinline__ long long block_sum_ll(long long v, long long* s) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    long long t = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += s[w];
    __syncthreads();
    return t;   // valid in thread 0
}

template <int N>
__device__ void explore_block(const BatchQuery& Q, BatchOut& out, float* s_raw, float* s_in,
                              float* s_out, int* s_w, long long* s_ll) {
    constexpr int W = N / 32;
    const int tid = threadIdx.x, T = blockDim.x, lane = tid & 63, wave = tid >> 6, nw = T >> 6;
    RoundArgs a = Q.a;
    Ctl* c = a.ctl;
    stage_obstacles_block(a.obs, a.n_obs, s_raw, s_in, s_out);
    a.open_out = Q.open_a;
    explore_init_fill(a, Q.n_nodes, tid, T);
    __syncthreads();
    if (tid == 0) explore_init_root(a, N);
    int32_t* cur = Q.open_a;
    int32_t* nxt = Q.open_b;
    float gl[3], gh[3];
    for (int k = 0; k < 3; ++k) { gl[k] = a.gcloud[k]; gh[k] = a.gcloud[3 + k]; }
    long long n_sim = 0, n_pre = 0, n_drop = 0, n_flag = 0, kept = 0, partial = 0;
    long long w_pre = 0, w_flag = 0;   // wave-uniform counters of the simulation
    int rounds = 0;
    for (;;) {
        __syncthreads();
        const int done = c->done, n_pairs = c->n_pairs, n_B = c->n_B, n_open = c->n_open;
        if (done) break;
        __syncthreads();
        if (n_pairs > Q.cap_pairs) {
            if (tid == 0) { c->err = 4; c->done = 1; }
            break;
        }
        a.open_in = cur;
        a.open_out = nxt;
        partial += n_pairs;
        ++rounds;
        // expansion: pairs, then queued simulations
        for (int tile = wave * 64; tile < n_pairs; tile += nw * 64) {
            const int q = tile + lane;
            const int st = q < n_pairs ? expand_pair<N>(a, q, n_B, s_out, gl, gh, n_sim, n_pre, n_drop) : 0;
            queue_pairs(a, q, st);
        }
        __syncthreads();
        const int n_tasks = c->n_tasks;
        for (int task = wave; task < n_tasks; task += nw)
            simulate_pair<N>(a, a.tasks[task], s_raw, s_in, s_out, w_pre, w_flag);
        __syncthreads();
        // RemoveDominated
        for (int q = tid; q < n_pairs; q += T) stair_update_pair(a, q);
        __syncthreads();
        for (int t = tid; t < n_pairs + n_open; t += T) {
            if (t < n_pairs) kept += mark_pair(a, t) ? 1 : 0;
            else mark_open(a, t - n_pairs);
        }
        __syncthreads();
        // compaction
        const int n_surv = block_scan(a.c_pos, a.c_pos, n_pairs, s_w);
        const int n_keep = block_scan(a.o_keep, a.o_keep, n_open, s_w);
        const int n_plans = c->n_plans;
        const int i_round = c->i;
        const bool fits = (long long)n_plans + n_surv <= a.cap_plans;
        for (int t = tid; t < n_pairs + n_open; t += T) {
            if (t < n_pairs) {
                if (fits) compact_pair<W>(a, t, n_plans, n_keep, i_round);
            } else {
                compact_open(a, t - n_pairs);
            }
        }
        __syncthreads();
        if (tid == 0) {
            c->scan_total[0] = n_surv;
            c->scan_total[1] = n_keep;
            compact_finalize(c, a.cap_plans);
        }
        __syncthreads();
        // next group and the loop test
        const int n_open2 = c->n_open;
        unsigned long long m = 0x7FF0000000000000ull;
        for (int i = tid; i < n_open2; i += T) {
            const unsigned long long b = (unsigned long long)__double_as_longlong(a.p_cost[a.open_out[i]]);
            m = b < m ? b : m;
        }
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long y = __shfl_down(m, o, 64);
            m = y < m ? y : m;
        }
        if (lane == 0) atomicMin(&c->min_cost_bits, m);
        __syncthreads();
        if (tid == 0) pick_next_i(c, a.h);
        __syncthreads();
        if (!c->done) {
            const double thr = (double)c->i * a.h;
            int stop = 0;
            for (int i = tid; i < n_open2; i += T) stop |= flag_group_one(a, i, thr) ? 1 : 0;
            if (__any(stop) && lane == 0) atomicOr(&c->goal_stop, 1);
            __syncthreads();
            const int nB = block_scan(a.o_keep, a.o_keep, n_open2, s_w);
            for (int i = tid; i < n_open2; i += T) scatter_group_one(a, i, Q.b_deg);
            __syncthreads();
            const int np = block_scan(Q.b_deg, a.b_off, nB, s_w);
            if (tid == 0) {
                c->scan_total[2] = nB;
                c->scan_total[3] = np;
                c->n_B = nB;
                c->n_pairs = np;
                c->n_tasks = 0;
                a.b_off[nB] = np;
                c->done = c->goal_stop ? 1 : 0;
            }
        } else if (tid == 0) {
            c->n_B = 0;
            c->n_pairs = 0;
        }
        int32_t* t = cur;
        cur = nxt;
        nxt = t;
    }
    __syncthreads();
    const long long s_sim = block_sum_ll(n_sim, s_ll);
    const long long s_pre = block_sum_ll(n_pre + (lane == 0 ? w_pre : 0), s_ll);
    const long long s_drop = block_sum_ll(n_drop, s_ll);
    const long long s_flag = block_sum_ll(lane == 0 ? w_flag : 0, s_ll);
    const long long s_kept = block_sum_ll(kept, s_ll);
    if (tid == 0) {
        c->simulated += s_sim;
        c->preprune += s_pre;
        c->dropped_steps += s_drop;
        c->flagged += s_flag;
        c->inserted += s_kept;
        out.rounds = rounds;
        out.partial_plans = partial;
        out.final_i = c->i;
        out.err = c->err;
        out.n_plans = c->n_plans;
    }
    __syncthreads();
}

__global__ __launch_bounds__(512) void k_b_explore(BatchQuery* qs, int q, const int* order,
                                                    int* counter, BatchOut* outs) {
    __shared__ float s_raw[kMaxObs * 6];
    __shared__ float s_in[kMaxObs * 6];
    __shared__ float s_out[kMaxObs * 6];
    __shared__ int s_w[16];
    __shared__ long long s_ll[16];
    __shared__ int s_next;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_next = atomicAdd(counter, 1);
        __syncthreads();
        const int k = s_next;
        if (k >= q) break;
        const int qi = order[k];
        const BatchQuery& Q = qs[qi];
        BatchOut& o = outs[qi];
        if (Q.bad) {
            if (threadIdx.x == 0) o.err = -1;
            continue;
        }
        switch (Q.N) {
            case 32: explore_block<32>(Q, o, s_raw, s_in, s_out, s_w, s_ll); break;
            case 64: explore_block<64>(Q, o, s_raw, s_in, s_out, s_w, s_ll); break;
            case 128: explore_block<128>(Q, o, s_raw, s_in, s_out, s_w, s_ll); break;
            default: explore_block<256>(Q, o, s_raw, s_in, s_out, s_w, s_ll); break;
        }
    }
}

// ----------------------------- selection ------------------------------------
__device__ __forceinline__ SelectArgs select_of(const BatchQuery& Q) {
    SelectArgs s = Q.s;
    s.n_plans = Q.a.ctl->n_plans;
    return s;
}

__global__ __launch_bounds__(1024) void k_b_goal_collect(BatchQuery* qs) {
    const BatchQuery& Q = qs[blockIdx.x];
    if (Q.bad || Q.a.ctl->err) return;
    goal_collect_block(select_of(Q));
}

__global__ __launch_bounds__(256) void k_b_front(BatchQuery* qs) {
    const BatchQuery& Q = qs[blockIdx.x];
    if (Q.bad || Q.a.ctl->err) return;
    front_block(select_of(Q), kBatchFront);
}

__global__ void k_b_waypoints(BatchQuery* qs) {
    const BatchQuery& Q = qs[blockIdx.x];
    const int f = threadIdx.x;
    if (f < kBatchFront) Q.s.mc_counts[f] = 0;
    if (Q.bad || Q.a.ctl->err) return;
    if (f < Q.a.ctl->n_front) waypoints_one(Q.s, f);
}

__global__ __launch_bounds__(256) void k_b_mc(BatchQuery* qs) {
    __shared__ float s_obs[kMaxObs * 6];
    const BatchQuery& Q = qs[blockIdx.z];
    const int f = blockIdx.y;
    if (Q.bad || Q.a.ctl->err || f >= Q.a.ctl->n_front) return;   // uniform per block
    for (int t = threadIdx.x; t < Q.s.n_obs * 6; t += blockDim.x) s_obs[t] = Q.s.obs[t];
    __syncthreads();
    const bool hit = mc_particle(Q.s, f, blockIdx.x * blockDim.x + threadIdx.x, s_obs);
    const unsigned long long b = __ballot(hit);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(&Q.s.mc_counts[f], (int)__popcll(b));
}

// Alg. 5 bisection on the certified counts, and the per-query outcome.
__global__ void k_b_finalize(BatchQuery* qs, int q, BatchOut* outs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= q) return;
    const BatchQuery& Q = qs[i];
    BatchOut& o = outs[i];
    const Ctl* c = Q.a.ctl;
    o.bad = Q.bad;
    o.best = -1;
    o.best_plan = -1;
    o.n_edges = Q.row_ptr[Q.n_nodes];
    if (Q.bad) {
        o.status = (Q.bad & 4) ? PUMP_E_CAPACITY : PUMP_E_ARG;
        return;
    }
    if (c->err) {
        o.status = (c->err == 3) ? PUMP_E_STATE : PUMP_E_CAPACITY;
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
    auto gt = [&](int m1) { return (double)Q.s.mc_counts[m1 - 1] / (double)M > Q.alpha; };
    int l = 1, u = nf, m = (l + u + 1) / 2;
    while (l != u) {
        if (gt(m)) u = m - 1; else l = m;
        m = (l + u + 1) / 2;
    }
    if (gt(m)) {
        o.status = PUMP_INFEASIBLE;
        return;
    }
    const int p = Q.s.front_ids[m - 1];
    o.status = PUMP_OK;
    o.best = m - 1;
    o.best_plan = p;
    o.best_pop = Q.a.p_pop[p];
    o.best_mc = Q.s.mc_counts[m - 1];
    o.best_len = Q.s.path_len[m - 1];
    o.best_cost = Q.a.p_cost[p];
    o.best_cp_mc = (double)o.best_mc / (double)M;
}

__global__ void k_b_reset(int* counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

void launch_batch(hipStream_t s, BatchQuery* qs, int q, int N_max, int max_nodes, int S_max, int M,
                  int words, int explore_blocks, int explore_threads, int* counter, BatchOut* out,
                  const int* order) {
    (void)N_max;
    const int max_elems = std::max(max_nodes * 6, kMaxObs * 6);
    k_b_load<<<dim3((max_elems + 255) / 256, q), 256, 0, s>>>(qs);
    k_b_deviation<<<dim3(3, q), 256, 0, s>>>(qs, S_max);
    k_b_cloud<<<dim3(S_max + 1, q), 256, 0, s>>>(qs);
    k_b_gcloud<<<dim3(1, q), 256, 0, s>>>(qs, S_max + 1);
    const int vmax = std::max(max_nodes, kMaxObs);
    k_b_valid<<<dim3((vmax + 255) / 256, q), 256, 0, s>>>(qs);
    k_b_graph_mark<<<dim3(max_nodes, q), 256, (size_t)words * sizeof(uint32_t), s>>>(qs);
    k_b_row_scan<<<q, 1024, 0, s>>>(qs);
    k_b_graph_fill<<<dim3((max_nodes + 3) / 4, q), 256, 0, s>>>(qs);
    k_b_edge_steer<<<dim3(256, q), 256, 0, s>>>(qs);
    k_b_reset<<<1, 64, 0, s>>>(counter);
    k_b_explore<<<explore_blocks, explore_threads, 0, s>>>(qs, q, order, counter, out);
    k_b_goal_collect<<<q, 1024, 0, s>>>(qs);
    k_b_front<<<q, 256, 0, s>>>(qs);
    k_b_waypoints<<<q, 64, 0, s>>>(qs);
    k_b_mc<<<dim3((M + 255) / 256, kBatchFront, q), 256, 0, s>>>(qs);
    k_b_finalize<<<(q + 63) / 64, 64, 0, s>>>(qs, q, out);
}

}  // namespace pump
