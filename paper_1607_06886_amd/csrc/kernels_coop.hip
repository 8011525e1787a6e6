// Explore (Alg. 4) of one query as a single cooperative launch: every round's
// phases run back to back inside one kernel, separated by grid-wide barriers,
// so the loop needs no host round trip and no per-phase launch.  The phases
// call the same per-element bodies as the per-phase kernels
// (explore_ops.hpp) and keep their orders (scans over the same index ranges),
// so the plan store is identical to the one the per-round path builds.
//
// Work split: expansion strides over pairs by wave, the particle queue by
// wave, the staircase update by thread.  Marking, compaction and the next
// group use contiguous chunks of the pair and open lists, one chunk per
// workgroup, so each scan needs one barrier: a workgroup publishes its chunk
// total, and after the barrier adds the totals of the workgroups before it.
#include "explore_ops.hpp"

namespace pump {

namespace {

constexpr int kCoopThreads = 256;
constexpr long long kSpinLimit = 1ll << 25;   // about 1-2 s of polling per wait

// Grid barrier without a contended counter: workgroup b announces arrival at
// barrier number `epoch` by storing it in its own word arrive[b]; the threads
// of workgroup 0 poll all arrival words, then store `epoch` in the release
// word that every other workgroup polls.  Agent-scope fences around the
// stores and after the polls order the workgroups' memory.  A wait that
// exceeds the spin limit records a failure, so the kernel always ends.
// Returns true (the same in every thread of the workgroup) when the grid has
// failed; the caller then leaves its loop.
__device__ __forceinline__ bool grid_barrier(const CoopSync& g, unsigned& epoch, int* s_flag) {
    __syncthreads();
    epoch += 1u;
    if (threadIdx.x == 0) {
        __threadfence();
        __hip_atomic_store(g.arrive + blockIdx.x, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (blockIdx.x == 0) {
        int ok = 1;
        for (unsigned k = threadIdx.x; k < g.n_blocks && ok; k += blockDim.x) {
            long long spins = 0;
            while (__hip_atomic_load(g.arrive + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > kSpinLimit) {
                    ok = 0;
                    break;
                }
            }
        }
        if (!ok) atomicOr(g.fail, 1);
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence();
            __hip_atomic_store(g.release, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    } else if (threadIdx.x == 0) {
        long long spins = 0;
        while (__hip_atomic_load(g.release, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > kSpinLimit) {
                atomicOr(g.fail, 1);
                break;
            }
        }
    }
    if (threadIdx.x == 0) {
        __threadfence();
        *s_flag = __hip_atomic_load(g.fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    return *s_flag != 0;
}

// Contiguous chunk [lo, hi) of n items owned by workgroup b of G.
__device__ __forceinline__ void chunk_of(int n, int b, int G, int& lo, int& hi) {
    const long long c = ((long long)n + G - 1) / G;
    const long long l = (long long)b * c;
    lo = (int)(l < n ? l : n);
    hi = (int)(l + c < n ? l + c : n);
}

// Block sum of an int (all threads get the result).
__device__ __forceinline__ int block_sum_int(int v, int* s_w) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = v;
    __syncthreads();
    int t = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += s_w[w];
    __syncthreads();
    return t;
}

// Sum of tot[0..b) and of tot[0..G) (all threads get both).
__device__ __forceinline__ void prefix_of(const int* tot, int b, int G, int* s_w, int& before,
                                          int& all) {
    int x = 0, y = 0;
    for (int k = threadIdx.x; k < G; k += blockDim.x) {
        const int v = __hip_atomic_load(tot + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        y += v;
        if (k < b) x += v;
    }
    before = block_sum_int(x, s_w);
    all = block_sum_int(y, s_w);
}

// Exclusive scan of v over the block's threads in thread order, for one
// tile of blockDim.x items; returns the tile total (all threads).
__device__ __forceinline__ int block_excl(int v, int& excl, int* s_w) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    __syncthreads();
    if (lane == 63) s_w[wave] = x;
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < nw; ++w) {
        if (w < wave) off += s_w[w];
        tot += s_w[w];
    }
    excl = off + x - v;
    return tot;
}

__device__ __forceinline__ unsigned long long block_min_u64(unsigned long long m,
                                                            unsigned long long* s) {
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_down(m, o, 64);
        m = y < m ? y : m;
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = m;
    __syncthreads();
    unsigned long long r = s[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = s[w] < r ? s[w] : r;
    __syncthreads();
    return r;
}

__device__ __forceinline__ long long block_sum_ll2(long long v, long long* s) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    long long t = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += s[w];
    __syncthreads();
    return t;
}

}  // namespace

template <int N>
__global__ __launch_bounds__(kCoopThreads) void k_explore_coop(RoundArgs a, CoopArgs ca) {
    constexpr int W = N / 32;
    __shared__ float s_raw[kMaxObs * 6];
    __shared__ float s_in[kMaxObs * 6];
    __shared__ float s_out[kMaxObs * 6];
    __shared__ int s_w[16];
    __shared__ unsigned long long s_m[16];
    __shared__ long long s_ll[16];
    __shared__ int s_fail;
    const CoopSync g = ca.sync;
    unsigned epoch = 0;
    const int G = gridDim.x, b = blockIdx.x, T = blockDim.x, tid = threadIdx.x;
    const int lane = tid & 63;
    const int gwave = b * (T >> 6) + (tid >> 6), n_gwaves = G * (T >> 6);
    Ctl* c = a.ctl;
    const bool leader = (b == 0 && tid == 0);
    stage_obstacles_block(a.obs, a.n_obs, s_raw, s_in, s_out);
    float gl[3], gh[3];
    for (int k = 0; k < 3; ++k) { gl[k] = a.gcloud[k]; gh[k] = a.gcloud[3 + k]; }
    // loop state, identical in every workgroup
    int n_pairs = c->n_pairs, n_B = c->n_B, n_open = c->n_open, n_plans = c->n_plans;
    int i_cur = c->i, done = c->done;
    int32_t* cur = ca.open_cur;
    int32_t* nxt = ca.open_next;
    long long n_sim = 0, n_pre = 0, n_drop = 0, kept = 0;
    long long w_pre = 0, w_flag = 0;     // wave-uniform
    long long partial = 0;
    int rounds = 0, err = 0;
    __syncthreads();
    while (!done) {
        if ((long long)n_pairs > ca.cap_pairs) {
            err = 4;
            break;
        }
        if (rounds >= (1 << 22)) {   // the loop must have ended long before
            err = 6;
            break;
        }
        a.open_in = cur;
        a.open_out = nxt;
        partial += n_pairs;
        ++rounds;
        // (1) expansion, one pair per lane; particle simulations queued
        for (int tile = gwave * 64; tile < n_pairs; tile += n_gwaves * 64) {
            const int q = tile + lane;
            const int st = q < n_pairs ? expand_pair<N>(a, q, n_B, s_out, gl, gh, n_sim, n_pre, n_drop) : 0;
            queue_pairs(a, q, st);
        }
        if (grid_barrier(g, epoch, &s_fail)) break;
        // (2) particle simulation, one queued pair per wave
        const int n_tasks = __hip_atomic_load(&c->n_tasks, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int task = gwave; task < n_tasks; task += n_gwaves)
            simulate_pair<N>(a, a.tasks[task], s_raw, s_in, s_out, w_pre, w_flag);
        if (grid_barrier(g, epoch, &s_fail)) break;
        // (3) staircase update; the leader resets the per-round accumulators
        //     (nothing reads them until after the next barrier)
        for (int q = b * T + tid; q < n_pairs; q += G * T) stair_update_pair(a, q);
        if (leader) {
            c->n_tasks = 0;
            c->min_cost_bits = 0x7FF0000000000000ull;
            c->goal_stop = 0;
        }
        if (grid_barrier(g, epoch, &s_fail)) break;
        // (4) marks over contiguous chunks; chunk totals of the survivor and
        //     kept-open flags
        int p_lo, p_hi, o_lo, o_hi;
        chunk_of(n_pairs, b, G, p_lo, p_hi);
        chunk_of(n_open, b, G, o_lo, o_hi);
        int my_s = 0, my_k = 0;
        for (int t = p_lo + tid; t < p_hi; t += T) {
            kept += mark_pair(a, t) ? 1 : 0;
            my_s += a.c_pos[t];
        }
        for (int t = o_lo + tid; t < o_hi; t += T) {
            mark_open(a, t);
            my_k += a.o_keep[t];
        }
        my_s = block_sum_int(my_s, s_w);
        my_k = block_sum_int(my_k, s_w);
        if (tid == 0) {
            ca.tot_a[b] = my_s;
            ca.tot_b[b] = my_k;
        }
        if (grid_barrier(g, epoch, &s_fail)) break;
        // (5) scans of both flag arrays, compaction, cheapest new open plan
        int s_before, n_surv, k_before, n_keep;
        prefix_of(ca.tot_a, b, G, s_w, s_before, n_surv);
        prefix_of(ca.tot_b, b, G, s_w, k_before, n_keep);
        const bool fits = (long long)n_plans + n_surv <= a.cap_plans;
        unsigned long long m = 0x7FF0000000000000ull;
        {
            int carry = s_before;
            for (int t0 = p_lo; t0 < p_hi; t0 += T) {
                const int t = t0 + tid;
                const int v = t < p_hi ? a.c_pos[t] : 0;
                int ex;
                const int tot = block_excl(v, ex, s_w);
                if (t < p_hi) a.c_pos[t] = carry + ex;
                carry += tot;
            }
            carry = k_before;
            for (int t0 = o_lo; t0 < o_hi; t0 += T) {
                const int t = t0 + tid;
                const int v = t < o_hi ? a.o_keep[t] : 0;
                int ex;
                const int tot = block_excl(v, ex, s_w);
                if (t < o_hi) a.o_keep[t] = carry + ex;
                carry += tot;
            }
        }
        __syncthreads();
        for (int t = p_lo + tid; t < p_hi; t += T) {
            if (fits) {
                compact_pair<W>(a, t, n_plans, n_keep, i_cur);
                if (a.c_flag[t] == 1) {
                    const unsigned long long bits =
                        (unsigned long long)__double_as_longlong(a.c_cost[t]);
                    m = bits < m ? bits : m;
                }
            }
        }
        for (int t = o_lo + tid; t < o_hi; t += T) {
            compact_open(a, t);
            const int p = a.open_in[t];
            if (a.p_state[p] == kOpen) {
                const unsigned long long bits = (unsigned long long)__double_as_longlong(a.p_cost[p]);
                m = bits < m ? bits : m;
            }
        }
        m = block_min_u64(m, s_m);
        if (tid == 0 && m != 0x7FF0000000000000ull) atomicMin(&c->min_cost_bits, m);
        if (!fits) {
            err = 1;
            break;
        }
        n_plans += n_surv;
        n_open = n_keep + n_surv;
        {
            // the list just written is current from here on (the phases
            // below still address it as a.open_out)
            int32_t* tmp = cur;
            cur = nxt;
            nxt = tmp;
        }
        if (grid_barrier(g, epoch, &s_fail)) break;
        // (6) next group index; flag the group and count it per chunk
        if (n_open == 0) {
            done = 1;
            i_cur += 1;
        } else {
            const double mc = __longlong_as_double((long long)__hip_atomic_load(
                &c->min_cost_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            if (!(mc >= 0.0 && mc < 1e300) || !(mc / a.h < 2.0e9)) {
                err = 3;
                break;
            }
            long long k = (long long)ceil(mc / a.h);
            if (k < 0) k = 0;
            while (k > 0 && mc <= (double)(k - 1) * a.h) --k;
            while (!(mc <= (double)k * a.h)) ++k;
            const long long inext = (long long)i_cur + 1;
            i_cur = (int)(k > inext ? k : inext);
        }
        if (done) break;
        const double thr = (double)i_cur * a.h;
        int n_lo, n_hi;
        chunk_of(n_open, b, G, n_lo, n_hi);
        int stop = 0, my_b = 0;
        for (int t = n_lo + tid; t < n_hi; t += T) {
            stop |= flag_group_one(a, t, thr) ? 1 : 0;
            my_b += a.o_keep[t];
        }
        if (__any(stop) && lane == 0) atomicOr(&c->goal_stop, 1);
        my_b = block_sum_int(my_b, s_w);
        if (tid == 0) ca.tot_a[b] = my_b;
        if (grid_barrier(g, epoch, &s_fail)) break;
        // (7) scan of the group flags, scatter of the group and its degrees;
        //     chunk totals of the degrees
        int b_before, nB;
        prefix_of(ca.tot_a, b, G, s_w, b_before, nB);
        int my_d = 0;
        {
            int carry = b_before;
            for (int t0 = n_lo; t0 < n_hi; t0 += T) {
                const int t = t0 + tid;
                const int v = t < n_hi ? a.o_keep[t] : 0;
                int ex;
                const int tot = block_excl(v, ex, s_w);
                if (t < n_hi) a.o_keep[t] = carry + ex;
                carry += tot;
            }
        }
        __syncthreads();
        for (int t = n_lo + tid; t < n_hi; t += T) {
            scatter_group_one(a, t, ca.b_deg);
            if (a.o_inB[t]) {
                const int h = a.p_head[a.open_out[t]];
                my_d += a.row_ptr[h + 1] - a.row_ptr[h];
            }
        }
        my_d = block_sum_int(my_d, s_w);
        if (tid == 0) ca.tot_b[b] = my_d;
        if (grid_barrier(g, epoch, &s_fail)) break;
        // (8) pair offsets of the group: exclusive scan of the degrees in
        //     group order (= open-list order), per chunk
        int d_before, n_pairs_next;
        prefix_of(ca.tot_b, b, G, s_w, d_before, n_pairs_next);
        {
            int carry = d_before;
            for (int t0 = n_lo; t0 < n_hi; t0 += T) {
                const int t = t0 + tid;
                int v = 0;
                if (t < n_hi && a.o_inB[t]) {
                    const int h = a.p_head[a.open_out[t]];
                    v = a.row_ptr[h + 1] - a.row_ptr[h];
                }
                int ex;
                const int tot = block_excl(v, ex, s_w);
                if (t < n_hi && a.o_inB[t]) a.b_off[a.o_keep[t]] = carry + ex;
                carry += tot;
            }
        }
        const int goal_stop = __hip_atomic_load(&c->goal_stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (leader) a.b_off[nB] = n_pairs_next;
        n_B = nB;
        n_pairs = n_pairs_next;
        done = goal_stop ? 1 : 0;
        if (grid_barrier(g, epoch, &s_fail)) break;
    }
    // counters and the final loop state
    const long long s_sim = block_sum_ll2(n_sim, s_ll);
    const long long s_pre = block_sum_ll2(n_pre + (lane == 0 ? w_pre : 0), s_ll);
    const long long s_drop = block_sum_ll2(n_drop, s_ll);
    const long long s_flag = block_sum_ll2(lane == 0 ? w_flag : 0, s_ll);
    const long long s_kept = block_sum_ll2(kept, s_ll);
    if (tid == 0) {
        if (s_sim) atomicAdd((unsigned long long*)&c->simulated, (unsigned long long)s_sim);
        if (s_pre) atomicAdd((unsigned long long*)&c->preprune, (unsigned long long)s_pre);
        if (s_drop) atomicAdd((unsigned long long*)&c->dropped_steps, (unsigned long long)s_drop);
        if (s_flag) atomicAdd((unsigned long long*)&c->flagged, (unsigned long long)s_flag);
        if (s_kept) atomicAdd((unsigned long long*)&c->inserted, (unsigned long long)s_kept);
    }
    if (leader) {
        const bool failed =
            __hip_atomic_load(g.fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        c->n_plans = n_plans;
        c->n_open = n_open;
        c->n_B = done ? 0 : n_B;
        c->n_pairs = done ? 0 : n_pairs;
        c->i = i_cur;
        c->err = failed ? 5 : err;
        c->done = 1;
        c->rounds = rounds;
        c->partial = partial;
        c->open_final = (cur == ca.open_cur) ? 0 : 1;
    }
}

hipError_t launch_explore_coop(hipStream_t s, const RoundArgs& a, const CoopArgs& ca, int N,
                               int blocks) {
    void* args[2] = {(void*)&a, (void*)&ca};
    const void* fn;
    switch (N) {
        case 32: fn = (const void*)k_explore_coop<32>; break;
        case 64: fn = (const void*)k_explore_coop<64>; break;
        case 128: fn = (const void*)k_explore_coop<128>; break;
        default: fn = (const void*)k_explore_coop<256>; break;
    }
    return hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(kCoopThreads), args, 0, s);
}

int coop_max_blocks(int N) {
    int per_cu = 0, dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return 0;
    const void* fn;
    switch (N) {
        case 32: fn = (const void*)k_explore_coop<32>; break;
        case 64: fn = (const void*)k_explore_coop<64>; break;
        case 128: fn = (const void*)k_explore_coop<128>; break;
        default: fn = (const void*)k_explore_coop<256>; break;
    }
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kCoopThreads, 0) != hipSuccess)
        return 0;
    return per_cu * prop.multiProcessorCount;
}

}  // namespace pump
