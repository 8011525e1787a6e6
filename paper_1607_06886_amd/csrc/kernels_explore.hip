// Explore (Alg. 4): one round = expand the group B to every neighbour,
// RemoveDominated, retire B, select the next group.
#include "explore_ops.hpp"

namespace pump {

// ---------------------------------------------------------------------------
// Device-wide exclusive scan of int32 (length read from device memory).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int block_exclusive_sum(int v, int* s_tmp, int& total) {
    // 256 threads = 4 waves
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_tmp[wave] = x;
    __syncthreads();
    int off = 0;
    for (int w = 0; w < wave; ++w) off += s_tmp[w];
    total = s_tmp[0] + s_tmp[1] + s_tmp[2] + s_tmp[3];
    __syncthreads();
    return off + x - v;
}

__global__ __launch_bounds__(256) void k_scan_reduce(const int32_t* __restrict__ in,
                                                     const int32_t* __restrict__ n_dev,
                                                     int32_t* __restrict__ blk) {
    __shared__ int s_tmp[4];
    const int n = *n_dev;
    const int base = blockIdx.x * kScanBlock;
    if (base >= n) {
        if (threadIdx.x == 0) blk[blockIdx.x] = 0;
        return;
    }
    int sum = 0;
    for (int k = 0; k < 4; ++k) {
        int idx = base + threadIdx.x * 4 + k;
        if (idx < n) sum += in[idx];
    }
    int total;
    block_exclusive_sum(sum, s_tmp, total);
    if (threadIdx.x == 0) blk[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void k_scan_blocks(int32_t* __restrict__ blk, int nblk,
                                                     int32_t* __restrict__ total_dev,
                                                     int32_t* __restrict__ total2_dev) {
    __shared__ int s_tmp[4];
    int carry = 0;
    for (int b0 = 0; b0 < nblk; b0 += 256) {
        int idx = b0 + threadIdx.x;
        int v = idx < nblk ? blk[idx] : 0;
        int total;
        int ex = block_exclusive_sum(v, s_tmp, total);
        if (idx < nblk) blk[idx] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) {
        *total_dev = carry;
        if (total2_dev) *total2_dev = carry;
    }
}

__global__ __launch_bounds__(256) void k_scan_down(const int32_t* __restrict__ in,
                                                   int32_t* __restrict__ out,
                                                   const int32_t* __restrict__ n_dev,
                                                   const int32_t* __restrict__ blk) {
    __shared__ int s_tmp[4];
    const int n = *n_dev;
    const int base = blockIdx.x * kScanBlock;
    if (base >= n) return;
    int v[4];
    int sum = 0;
    for (int k = 0; k < 4; ++k) {
        int idx = base + threadIdx.x * 4 + k;
        v[k] = idx < n ? in[idx] : 0;
        sum += v[k];
    }
    int total;
    int ex = block_exclusive_sum(sum, s_tmp, total) + blk[blockIdx.x];
    for (int k = 0; k < 4; ++k) {
        int idx = base + threadIdx.x * 4 + k;
        if (idx < n) out[idx] = ex;
        ex += v[k];
    }
}

void scan_exclusive(hipStream_t s, const int32_t* in, int32_t* out, const int32_t* n_dev,
                    int32_t n_upper, int32_t* total_dev, int32_t* blk, int32_t* total2_dev) {
    int nblk = (n_upper + kScanBlock - 1) / kScanBlock;
    if (nblk < 1) nblk = 1;
    k_scan_reduce<<<nblk, 256, 0, s>>>(in, n_dev, blk);
    k_scan_blocks<<<1, 256, 0, s>>>(blk, nblk, total_dev, total2_dev);
    k_scan_down<<<nblk, 256, 0, s>>>(in, out, n_dev, blk);
}

// ---------------------------------------------------------------------------
// Initialisation (Alg. 4 first lines): P_open = P(x_init) = B = {root},
// root = (x_init, [], 0, 0), i = 0.  The dominance staircase of every node
// starts empty (+inf); the root puts cost 0 at every pop level of node 0.
// ---------------------------------------------------------------------------
__global__ void k_init_fill(RoundArgs a, int n_nodes, unsigned* zero, int n_zero) {
    const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    explore_init_fill(a, n_nodes, t0, stride);
    for (size_t t = t0; t < (size_t)n_zero; t += stride) zero[t] = 0u;
}

// The whole control block is cleared before the root's fields are set.
__global__ void k_root(RoundArgs a, int N) {
    unsigned* w = reinterpret_cast<unsigned*>(a.ctl);
    for (int t = threadIdx.x; t < (int)(sizeof(Ctl) / sizeof(unsigned)); t += blockDim.x) w[t] = 0u;
    __syncthreads();
    if (threadIdx.x == 0 && blockIdx.x == 0) explore_init_root(a, N);
}

void launch_explore_init(hipStream_t s, const RoundArgs& a, int n_nodes, int N, unsigned* zero,
                         int n_zero) {
    size_t n = (size_t)n_nodes * a.stair_w;
    if ((size_t)n_zero > n) n = (size_t)n_zero;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    k_init_fill<<<(unsigned)blocks, 256, 0, s>>>(a, n_nodes, zero, n_zero);
    k_root<<<1, 64, 0, s>>>(a, N);
}

// ---------------------------------------------------------------------------
// Counter partials: each workgroup adds its sums to its own slots of a.part
// (no atomics on the control block, whose one line every workgroup would
// otherwise queue on); k_counters_reduce folds them in once a round.
// ---------------------------------------------------------------------------
// Sum over the workgroup, valid in thread 0 (all threads call it; s holds
// blockDim.x / 64 entries).
__device__ __forceinline__ long long block_sum(long long v, long long* s) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    long long t = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += s[w];
    __syncthreads();
    return t;
}

__device__ __forceinline__ void part_add(const RoundArgs& a, int k, long long v) {
    if (v) a.part[(size_t)blockIdx.x * kPartK + k] += v;   // this workgroup's slot
}

// kReduceBlocks workgroups, each over its share of the slots; each adds its
// sums into the control block (a handful of atomics in all).
constexpr int kReduceBlocks = 16;

__global__ __launch_bounds__(256) void k_counters_reduce(RoundArgs a, int add) {
    __shared__ long long s[4];
    long long v[kPartK];
    for (int k = 0; k < kPartK; ++k) v[k] = 0;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < kPartSlots; t += gridDim.x * blockDim.x) {
        for (int k = 0; k < kPartK; ++k) {
            v[k] += a.part[(size_t)t * kPartK + k];
            a.part[(size_t)t * kPartK + k] = 0;
        }
    }
    long long tot[kPartK];
    for (int k = 0; k < kPartK; ++k) tot[k] = block_sum(v[k], s);
    if (threadIdx.x == 0 && add) {
        Ctl* c = a.ctl;
        auto add_ll = [](long long* dst, long long x) {
            if (x) atomicAdd((unsigned long long*)dst, (unsigned long long)x);
        };
        add_ll(&c->simulated, tot[kPartSimulated]);
        add_ll(&c->preprune, tot[kPartPreprune]);
        add_ll(&c->dropped_steps, tot[kPartDropped]);
        add_ll(&c->flagged, tot[kPartFlagged]);
        add_ll(&c->sim_waypoints, tot[kPartWaypoints]);
        add_ll(&c->sim_box_tests, tot[kPartBoxTests]);
        add_ll(&c->inserted, tot[kPartInserted]);
    }
}

void launch_counters_reduce(hipStream_t s, const RoundArgs& a) {
    k_counters_reduce<<<kReduceBlocks, 256, 0, s>>>(a, 1);
}

void launch_counters_clear(hipStream_t s, const RoundArgs& a) {
    k_counters_reduce<<<kReduceBlocks, 256, 0, s>>>(a, 0);
}

static int part_grid(long long n, int per_block) {
    long long b = (n + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > kPartSlots) b = kPartSlots;
    return (int)b;
}

// ---------------------------------------------------------------------------
// Expansion (Alg. 4: every pair (p in B, x in N(p.head)) forms q with
// Cost and CP_hat, then the CP cutoff): k_expand_pairs runs the first part
// with one pair per lane and queues the pairs whose particles must be
// simulated; k_expand_sim simulates them with one pair per wave.
//
// The queue records of a workgroup gather in LDS (one LDS atomic per wave)
// and go out in one coalesced copy, behind one global atomic, after each
// 256-pair pass that queued any.  The box-model pair stage runs six waves
// per SIMD (80 VGPRs, a few values spilled; 20 KB of LDS per workgroup): on
// the 20,000-sample indoor query it took 1.48 ms per query against 1.59 ms
// at four waves (105 VGPRs, a 768-record stage) and 1.61 ms at eight.  The
// half-space model's, with more live values, stays at four.
// ---------------------------------------------------------------------------
constexpr int kTaskStage = 256;   // records staged per workgroup (8 KB): one pass

__device__ __forceinline__ void flush_tasks(const RoundArgs& a, SimTask* s_tq, int* s_tn, int* s_tb) {
    const int n = *s_tn;   // (read after a barrier: the same in every thread)
    if (n == 0) return;
    if (threadIdx.x == 0) *s_tb = atomicAdd(&a.ctl->n_tasks, n);
    __syncthreads();
    const int b = *s_tb;
    for (int i = threadIdx.x; i < n; i += blockDim.x) a.tasks[b + i] = s_tq[i];
    __syncthreads();
    if (threadIdx.x == 0) *s_tn = 0;
    __syncthreads();
}

template <int N, int CP>
__global__ __launch_bounds__(256, CP == 0 ? 6 : 4) void k_expand_pairs(RoundArgs a) {
    __shared__ float s_raw[kMaxObs * 6];
    __shared__ float s_out[kMaxObs * 6];
    __shared__ SimTask s_tq[kTaskStage];
    __shared__ int s_tn, s_tb;
    __shared__ long long s_ll[4];
    stage_obstacles_block(a.obs, a.n_obs, s_raw, nullptr, s_out);
    if (threadIdx.x == 0) s_tn = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    // pairs [a.q0, q_end) of the round: all of them, or one chunk
    const int q_end = a.chunked ? a.q0 + a.ctl->chunk_n : a.ctl->n_pairs;
    const int n_B = a.ctl->n_B;
    float gl[3], gh[3];
    for (int k = 0; k < 3; ++k) { gl[k] = a.gcloud[k]; gh[k] = a.gcloud[3 + k]; }
    long long n_sim = 0, n_pre = 0, n_drop = 0;
    // workgroup passes of 256 pairs (the same count in every thread)
    for (int base = a.q0 + blockIdx.x * 256; base < q_end; base += gridDim.x * 256) {
        const int tile = base + (threadIdx.x & ~63);
        const int q = base + threadIdx.x;
        SimTask tk;
        int st = 0;
        if (tile < q_end) {   // the wave's pairs
            const int grp = wave_group_of(a.b_off, n_B, tile, q);
            st = q < q_end ? expand_pair<N, CP>(a, q, grp, s_raw, s_out, gl, gh, n_sim, n_pre, n_drop,
                                                tk) : 0;
        }
        const unsigned long long need = __ballot(st == 2);
        int wb = 0;
        if (lane == 0 && need) wb = atomicAdd(&s_tn, (int)__popcll(need));
        wb = __shfl(wb, 0, 64);
        if (st == 2) s_tq[wb + (int)__popcll(need & lanemask_lt(lane))] = tk;
        __syncthreads();
        if (s_tn > kTaskStage - 256) flush_tasks(a, s_tq, &s_tn, &s_tb);
    }
    flush_tasks(a, s_tq, &s_tn, &s_tb);
    const long long t_sim = block_sum(n_sim, s_ll);
    const long long t_pre = block_sum(n_pre, s_ll);
    const long long t_drop = block_sum(n_drop, s_ll);
    if (threadIdx.x == 0 && !a.quiet) {
        part_add(a, kPartSimulated, t_sim);
        part_add(a, kPartPreprune, t_pre);
        part_add(a, kPartDropped, t_drop);
    }
}

// CP = 0: the box predicate, 1: the half-space model (one instantiation each,
// so the box kernel keeps only its own registers: 4 waves per SIMD).
template <int N, int CP>
__global__ __launch_bounds__(256) void k_expand_sim(RoundArgs a) {
    __shared__ float s_raw[kMaxObs * 6];
    __shared__ float s_in[kMaxObs * 6];
    __shared__ float s_out[kMaxObs * 6];
    __shared__ long long s_ll[4];
    stage_obstacles_block(a.obs, a.n_obs, s_raw, s_in, s_out);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int n_tasks = a.ctl->n_tasks;
    long long n_pre = 0, n_flag = 0, n_wp = 0, n_bt = 0;
    for (int task = blockIdx.x * 4 + (threadIdx.x >> 6); task < n_tasks; task += gridDim.x * 4) {
        if (CP == 1)
            simulate_pair_hsmc<N>(a, task, s_raw, n_pre, n_flag, n_wp, n_bt);
        else
            simulate_pair_box<N>(a, task, s_raw, s_in, s_out, n_pre, n_flag, n_wp, n_bt);
    }
    // the counts are wave-uniform: lane 0 brings them
    const long long t_pre = block_sum(lane == 0 ? n_pre : 0, s_ll);
    const long long t_flag = block_sum(lane == 0 ? n_flag : 0, s_ll);
    const long long t_wp = block_sum(lane == 0 ? n_wp : 0, s_ll);
    const long long t_bt = block_sum(lane == 0 ? n_bt : 0, s_ll);
    if (threadIdx.x == 0 && !a.quiet) {
        part_add(a, kPartPreprune, t_pre);
        part_add(a, kPartFlagged, t_flag);
        part_add(a, kPartWaypoints, t_wp);
        part_add(a, kPartBoxTests, t_bt);
    }
}

template <int N>
static void launch_expand_n(hipStream_t s, const RoundArgs& a, unsigned blocks, unsigned sim_blocks,
                            int part) {
    if (part & 1) {
        if (a.cp_model == 1)
            k_expand_pairs<N, 1><<<blocks, 256, 0, s>>>(a);
        else
            k_expand_pairs<N, 0><<<blocks, 256, 0, s>>>(a);
    }
    if (part & 2) {
        if (a.cp_model == 1)
            k_expand_sim<N, 1><<<sim_blocks, 256, 0, s>>>(a);
        else
            k_expand_sim<N, 0><<<sim_blocks, 256, 0, s>>>(a);
    }
}

void launch_expand(hipStream_t s, const RoundArgs& a, int N, int32_t n_pairs, int part) {
    if (n_pairs <= 0) return;
    // pair stage: a workgroup per 256 pairs, at most kPartSlots of them (each
    // owns a counter slot); one pass per workgroup measured faster than four
    // (indoor query: 1.92 -> 1.59 ms), more workgroups hiding the loads'
    // latency better than fewer that flush their queue records less often
    const int blocks = part_grid(n_pairs, 256);
    // the particle kernel's grid covers the worst case (every pair queued),
    // capped; its waves stride over the queue length read on the device
    const int sim_blocks = part_grid(n_pairs, 4);
    switch (N) {
        case 32: launch_expand_n<32>(s, a, (unsigned)blocks, (unsigned)sim_blocks, part); break;
        case 64: launch_expand_n<64>(s, a, (unsigned)blocks, (unsigned)sim_blocks, part); break;
        case 128: launch_expand_n<128>(s, a, (unsigned)blocks, (unsigned)sim_blocks, part); break;
        default: launch_expand_n<256>(s, a, (unsigned)blocks, (unsigned)sim_blocks, part); break;
    }
}

// RemoveDominated (staircase update, then marks; see explore_ops.hpp).
__global__ __launch_bounds__(256) void k_stair_update(RoundArgs a) {
    const int n_pairs = a.chunked ? a.ctl->chunk_n : a.ctl->n_pairs;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n_pairs; q += gridDim.x * blockDim.x)
        stair_update_pair(a, q);
}

__global__ __launch_bounds__(256) void k_mark(RoundArgs a) {
    __shared__ long long s_ll[4];
    const int n_pairs = a.ctl->n_pairs;
    const int n_open = a.ctl->n_open;
    const int total = n_pairs + n_open;
    long long kept = 0;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
        if (t < n_pairs) kept += mark_pair(a, t) ? 1 : 0;
        else mark_open(a, t - n_pairs);
    }
    const long long t_kept = block_sum(kept, s_ll);
    if (threadIdx.x == 0) part_add(a, kPartInserted, t_kept);
}

static int grid_of(long long n) {
    long long b = (n + 255) / 256;
    if (b < 1) b = 1;
    if (b > 16384) b = 16384;
    return (int)b;
}

void launch_prune(hipStream_t s, const RoundArgs& a, int N, int32_t n_pairs, int32_t n_open) {
    (void)N;
    int b1 = (n_pairs + 255) / 256;
    if (b1 < 1) b1 = 1;
    if (b1 > 16384) b1 = 16384;
    k_stair_update<<<b1, 256, 0, s>>>(a);
    k_mark<<<part_grid((long long)n_pairs + n_open, 256), 256, 0, s>>>(a);
}

// Compaction: P_open <- (P_open \ B \ removed) U survivors.
// scan_total[0] = survivors, scan_total[1] = open plans kept.
template <int W>
__global__ __launch_bounds__(256) void k_compact(RoundArgs a) {
    const int n_pairs = a.ctl->n_pairs;
    const int n_open = a.ctl->n_open;
    const int n_plans = a.ctl->n_plans;
    const int n_surv = a.ctl->scan_total[0];
    const int n_keep = a.ctl->scan_total[1];
    const bool fits = (long long)n_plans + n_surv <= a.cap_plans;
    const int i_round = a.ctl->i;
    const int total = n_pairs + n_open;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
        if (t < n_pairs) {
            if (fits) compact_pair<W>(a, t, n_plans, n_keep, i_round);
        } else {
            compact_open(a, t - n_pairs);
        }
    }
}

__global__ void k_compact_finalize(Ctl* c, int64_t cap) { compact_finalize(c, cap); }

void launch_compact(hipStream_t s, const RoundArgs& a, int N, int32_t n_pairs, int32_t n_open,
                    int32_t* blk) {
    scan_exclusive(s, a.c_pos, a.c_pos, &a.ctl->n_pairs, n_pairs, &a.ctl->scan_total[0], blk);
    scan_exclusive(s, a.o_keep, a.o_keep, &a.ctl->n_open, n_open,
                   &a.ctl->scan_total[1], blk + 65536);
    int b = (n_pairs + n_open + 255) / 256;
    if (b < 1) b = 1;
    if (b > 16384) b = 16384;
    switch (N / 32) {
        case 1: k_compact<1><<<b, 256, 0, s>>>(a); break;
        case 2: k_compact<2><<<b, 256, 0, s>>>(a); break;
        case 4: k_compact<4><<<b, 256, 0, s>>>(a); break;
        default: k_compact<8><<<b, 256, 0, s>>>(a); break;
    }
    k_compact_finalize<<<1, 1, 0, s>>>(a.ctl, a.cap_plans);
}

// ---------------------------------------------------------------------------
// A round with more pairs than candidate slots runs in chunks of the pair
// list, in two passes.  RemoveDominated's outcome depends only on the final
// staircase of each node (the minimum over every kept candidate of the round
// and the plans before it), so
//   pass 1: per chunk, expansion and the staircase update (the candidates
//           are then dropped);
//   then:   the open list is marked against the final staircase and
//           compacted (P_open \ B \ removed);
//   pass 2: per chunk, the expansion again (the same candidates), marks
//           against the final staircase and compaction of the survivors
//           after those of the chunks before it.
// Survivors get the plan ids and open-list places the round would give them
// in one piece (pair order).  A pass-1 expansion already sees the entries of
// earlier chunks, so it may resolve a pair without simulating it that the
// round in one piece would simulate and then remove: that pair is dominated
// either way, and the staircase it would have updated already holds a lower
// cost at every level it reaches.  The counters count pass 1 (and the
// candidates kept before the test in pass 2).
// ---------------------------------------------------------------------------
__global__ void k_chunk_begin(Ctl* c, int32_t n) {
    c->chunk_n = n;
    c->n_tasks = 0;
}

__global__ __launch_bounds__(256) void k_mark_open_only(RoundArgs a) {
    const int n_open = a.ctl->n_open;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_open; i += gridDim.x * blockDim.x)
        mark_open(a, i);
}

__global__ __launch_bounds__(256) void k_compact_open_only(RoundArgs a) {
    const int n_open = a.ctl->n_open;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_open; i += gridDim.x * blockDim.x)
        compact_open(a, i);
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl->chunk_base = 0;
}

__global__ __launch_bounds__(256) void k_mark_chunk(RoundArgs a) {
    __shared__ long long s_ll[4];
    const int n = a.ctl->chunk_n;
    long long kept = 0;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
        kept += mark_pair(a, t) ? 1 : 0;
    const long long t_kept = block_sum(kept, s_ll);
    if (threadIdx.x == 0) part_add(a, kPartInserted, t_kept);
}

// survivors of this chunk after those of the chunks before it; nothing is
// written once the plan store would overflow (the final check reports it)
template <int W>
__global__ __launch_bounds__(256) void k_compact_chunk(RoundArgs a) {
    const int n = a.ctl->chunk_n;
    const int base = a.ctl->chunk_base;
    const int n_plans = a.ctl->n_plans;
    const int n_keep = a.ctl->scan_total[1];
    const bool fits = (long long)n_plans + base + a.ctl->scan_total[0] <= a.cap_plans;
    if (!fits) return;
    const int i_round = a.ctl->i;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
        compact_pair<W>(a, t, n_plans + base, n_keep + base, i_round);
}

__global__ void k_chunk_end(Ctl* c) { c->chunk_base += c->scan_total[0]; }

__global__ void k_chunks_finalize(Ctl* c, int64_t cap) {
    c->scan_total[0] = c->chunk_base;
    compact_finalize(c, cap);
}

void launch_chunk_begin(hipStream_t s, const RoundArgs& a, int32_t n) {
    k_chunk_begin<<<1, 1, 0, s>>>(a.ctl, n);
}

void launch_stair_update(hipStream_t s, const RoundArgs& a, int32_t n) {
    k_stair_update<<<grid_of(n), 256, 0, s>>>(a);
}

void launch_open_compact(hipStream_t s, const RoundArgs& a, int32_t n_open, int32_t* blk) {
    k_mark_open_only<<<grid_of(n_open), 256, 0, s>>>(a);
    scan_exclusive(s, a.o_keep, a.o_keep, &a.ctl->n_open, n_open, &a.ctl->scan_total[1],
                   blk + 65536);
    k_compact_open_only<<<grid_of(n_open), 256, 0, s>>>(a);
}

void launch_chunk_compact(hipStream_t s, const RoundArgs& a, int N, int32_t n, int32_t* blk) {
    k_mark_chunk<<<part_grid(n, 256), 256, 0, s>>>(a);
    scan_exclusive(s, a.c_pos, a.c_pos, &a.ctl->chunk_n, n, &a.ctl->scan_total[0], blk);
    switch (N / 32) {
        case 1: k_compact_chunk<1><<<grid_of(n), 256, 0, s>>>(a); break;
        case 2: k_compact_chunk<2><<<grid_of(n), 256, 0, s>>>(a); break;
        case 4: k_compact_chunk<4><<<grid_of(n), 256, 0, s>>>(a); break;
        default: k_compact_chunk<8><<<grid_of(n), 256, 0, s>>>(a); break;
    }
    k_chunk_end<<<1, 1, 0, s>>>(a.ctl);
}

void launch_chunks_finalize(hipStream_t s, const RoundArgs& a) {
    k_chunks_finalize<<<1, 1, 0, s>>>(a.ctl, a.cap_plans);
}

// Next group (Alg. 4: i <- i + 1, B <- cheap open plans) and the loop test.
__global__ __launch_bounds__(256) void k_open_min(RoundArgs a) {
    // after a failed compaction (plan store full: err set, done set) the
    // open list holds only the kept plans while n_open still counts the
    // previous round's, so there is nothing to read
    if (a.ctl->err || a.ctl->done) return;
    __shared__ unsigned long long s_m[4];
    const int n_open = a.ctl->n_open;
    unsigned long long m = 0x7FF0000000000000ull;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_open; i += gridDim.x * blockDim.x) {
        unsigned long long b = (unsigned long long)__double_as_longlong(a.p_cost[a.open_out[i]]);
        m = b < m ? b : m;
    }
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long y = __shfl_down(m, o, 64);
        m = y < m ? y : m;
    }
    // one atomic per workgroup (one per wave on a single word was the
    // kernel's cost: 0.23 ms a round on the indoor query)
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = s_m[w] < m ? s_m[w] : m;
        if (m != 0x7FF0000000000000ull) atomicMin(&a.ctl->min_cost_bits, m);
    }
}

__global__ void k_pick_i(RoundArgs a) { pick_next_i(a.ctl, a.h); }

__global__ __launch_bounds__(256) void k_flag_group(RoundArgs a) {
    const int n_open = a.ctl->n_open;
    if (a.ctl->done) return;
    const double thr = (double)a.ctl->i * a.h;
    int stop = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_open; i += gridDim.x * blockDim.x)
        stop |= flag_group_one(a, i, thr) ? 1 : 0;
    if (__any(stop) && (threadIdx.x & 63) == 0) atomicOr(&a.ctl->goal_stop, 1);
}

__global__ __launch_bounds__(256) void k_scatter_group(RoundArgs a, int32_t* deg) {
    const int n_open = a.ctl->n_open;
    if (a.ctl->done) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_open; i += gridDim.x * blockDim.x)
        scatter_group_one(a, i, deg);
}

__global__ void k_group_finalize(RoundArgs a) {
    Ctl* c = a.ctl;
    if (c->done) {
        c->n_B = 0;
        c->n_pairs = 0;
        return;
    }
    c->n_B = c->scan_total[2];
    c->n_pairs = c->scan_total[3];
    c->n_tasks = 0;
    a.b_off[c->n_B] = c->n_pairs;
    c->done = c->goal_stop ? 1 : 0;
}

__global__ void k_copy_ngroup(Ctl* c) {
    // the degree scan runs over n_B entries; publish it before the scan
    if (!c->done) c->n_B = c->scan_total[2];
    else c->n_B = 0;
}

void launch_next_group(hipStream_t s, const RoundArgs& a, int32_t n_open_upper, int32_t* deg,
                       int32_t* blk) {
    int b = (n_open_upper + 255) / 256;
    if (b < 1) b = 1;
    if (b > 16384) b = 16384;
    // (the bound counts this round's pairs too; the open list is much
    // shorter, so the minimum strides over it with at most 512 workgroups)
    k_open_min<<<b < 512 ? b : 512, 256, 0, s>>>(a);
    k_pick_i<<<1, 1, 0, s>>>(a);
    k_flag_group<<<b, 256, 0, s>>>(a);
    scan_exclusive(s, a.o_keep, a.o_keep, &a.ctl->n_open, n_open_upper, &a.ctl->scan_total[2],
                   blk);
    k_scatter_group<<<b, 256, 0, s>>>(a, deg);
    k_copy_ngroup<<<1, 1, 0, s>>>(a.ctl);
    scan_exclusive(s, deg, a.b_off, &a.ctl->n_B, n_open_upper, &a.ctl->scan_total[3],
                   blk + 65536);
    k_group_finalize<<<1, 1, 0, s>>>(a);
}

}  // namespace pump
