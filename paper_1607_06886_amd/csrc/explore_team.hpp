// Explore (Alg. 4) of one query by a team of workgroups that meet at
// barriers: all rounds run back to back without host round trips or
// per-phase launches.  A team is the whole grid of the single launch (one
// query on the whole device) or a few workgroups of the batched engine's
// persistent kernel.  The phases call the same per-element bodies as the
// per-phase kernels (explore_ops.hpp) and keep their orders (scans over the
// same index ranges), so the plan store is identical to the one the
// per-round path builds, whatever the team size.
//
// Work split: expansion strides over pairs by wave, the particle queue by
// wave, the staircase update by thread.  Marking, compaction and the next
// group use contiguous chunks of the pair and open lists, one chunk per
// member, so each scan needs one exchange of chunk totals: a member publishes
// its totals and then adds those of the members before it.
#pragma once

#include "explore_ops.hpp"

namespace pump {


__device__ __forceinline__ unsigned long long rt_ticks() { return __builtin_amdgcn_s_memrealtime(); }

// Deadline of one wait: the counter is read once every 64 polls.
struct WaitClock {
    unsigned long long t0, limit;
    unsigned polls;
    __device__ __forceinline__ explicit WaitClock(unsigned long long patience)
        : t0(rt_ticks()), limit(patience), polls(0) {}
    __device__ __forceinline__ bool expired() {
        return (++polls & 63u) == 0u && rt_ticks() - t0 > limit;
    }
};

// Team of workgroups working on one query: its rank/size, barrier words,
// per-workgroup scan totals and buffers.
struct TeamCtx {
    unsigned* arrive;          // [size] last barrier each member reached
    unsigned* release;         // last barrier member 0 released
    int* fail;                 // set when a wait ran out of patience
    unsigned long long patience;   // longest wait, in 100 MHz ticks
    int rank, size;
    unsigned long long* xa;    // [size] exchanged chunk totals, tagged (team_exchange)
    unsigned long long* xb;    // [size]
    int32_t* b_deg;            // group degrees (scatter output)
    int32_t* open_cur;         // open list read by the first round
    int32_t* open_next;
    int64_t cap_pairs;
};

// Team barrier without a contended counter: member r announces arrival at
// barrier number `epoch` by storing it in its own word arrive[r]; the threads
// of member 0 poll all arrival words, then store `epoch` in the release word
// that every other member polls.  Each member releases its writes
// (agent-scope release fence) before it arrives and acquires the others'
// (agent-scope acquire fence) once released: one cache write-back and one
// invalidation per member and barrier.  A team of one workgroup needs only
// the workgroup barrier.  A wait that exceeds the spin limit records a
// failure, so the kernel always ends.  Returns true (the same in every thread
// of the workgroup) when the team has failed; the caller then leaves its loop.
// With kFenced false the barrier only synchronises (no cache maintenance);
// team_exchange uses that form.
template <bool kFenced = true>
__device__ __forceinline__ bool team_barrier(const TeamCtx& g, unsigned& epoch, int* s_flag) {
    __syncthreads();
    if (g.size == 1) return false;
    epoch += 1u;
    if (threadIdx.x == 0) {
        if (kFenced) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(g.arrive + g.rank, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (g.rank == 0) {
        int ok = 1;
        for (int k = threadIdx.x; k < g.size && ok; k += blockDim.x) {
            WaitClock wc(g.patience);
            while (__hip_atomic_load(g.arrive + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
                __builtin_amdgcn_s_sleep(1);
                if (wc.expired()) {
                    ok = 0;
                    break;
                }
            }
        }
        if (!ok) atomicOr(g.fail, 1);
        __syncthreads();
        if (threadIdx.x == 0) {
            if (kFenced) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __hip_atomic_store(g.release, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    } else if (threadIdx.x == 0) {
        WaitClock wc(g.patience);
        while (__hip_atomic_load(g.release, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
            __builtin_amdgcn_s_sleep(1);
            if (wc.expired()) {
                atomicOr(g.fail, 1);
                break;
            }
        }
    }
    if (threadIdx.x == 0) {
        if (kFenced && g.rank != 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_flag = __hip_atomic_load(g.fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    return *s_flag != 0;
}

// A value that is the same in every lane, declared so to the compiler.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

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

// Totals gathered by team_exchange: sums of the members before this one and
// of all members, for both values, and the OR of the flags.
struct XSum {
    int a_before, a_all, b_before, b_all, flag;
};

// Exchange of two chunk totals per member (va, vb >= 0, below 2^31) and a
// flag between two phases, without cache maintenance.  Each member stores its
// values in its own 64-bit words (value in the low half, the exchange's
// number in the high half; the flag in bit 31 of the second word) with
// relaxed agent-scope atomic stores, passes an unfenced barrier, and reads
// every member's words with agent-scope atomic loads, waiting for any word
// that does not yet carry the current number.  An atomic word is coherent
// across the L2 caches of the XCDs by itself, so no write-back or
// invalidation is needed as long as the totals are all that crosses
// workgroups at this point: the phase before the exchange writes only the
// member's own chunk (and the words), and the phase after it reads that chunk
// back in the same workgroup.  The words are zero before the team's first
// exchange.  Returns true when the team has failed, like team_barrier.
__device__ __forceinline__ bool team_exchange(const TeamCtx& g, unsigned& epoch, int* s_flag,
                                              int va, int vb, int flag, int* s_w, XSum& r) {
    if (g.size == 1) {
        __syncthreads();
        r = XSum{0, va, 0, vb, flag};
        return false;
    }
    const unsigned long long tag = (unsigned long long)(epoch + 1u) << 32;
    if (threadIdx.x == 0) {
        __hip_atomic_store(g.xa + g.rank, tag | (unsigned)va, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(g.xb + g.rank, tag | (unsigned)vb | (flag ? 0x80000000ull : 0ull),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (team_barrier<false>(g, epoch, s_flag)) return true;
    int ab = 0, aa = 0, bb = 0, ba = 0, f = 0, ok = 1;
    for (int k = threadIdx.x; k < g.size && ok; k += blockDim.x) {
        unsigned long long w[2];
        for (int h = 0; h < 2 && ok; ++h) {
            unsigned long long* p = h ? g.xb + k : g.xa + k;
            WaitClock wc(g.patience);
            while (((w[h] = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) &
                    ~0xFFFFFFFFull) != tag) {
                __builtin_amdgcn_s_sleep(1);
                if (wc.expired()) {
                    ok = 0;
                    break;
                }
            }
        }
        if (!ok) break;
        const int a = (int)(unsigned)w[0];
        const int bv = (int)((unsigned)w[1] & 0x7FFFFFFFu);
        aa += a;
        ba += bv;
        f |= (int)((unsigned)w[1] >> 31);
        if (k < g.rank) {
            ab += a;
            bb += bv;
        }
    }
    if (!ok) atomicOr(g.fail, 1);
    r.a_before = uni(block_sum_int(ab, s_w));
    r.a_all = uni(block_sum_int(aa, s_w));
    r.b_before = uni(block_sum_int(bb, s_w));
    r.b_all = uni(block_sum_int(ba, s_w));
    r.flag = uni(block_sum_int(f, s_w));
    if (threadIdx.x == 0)
        *s_flag = __hip_atomic_load(g.fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    return *s_flag != 0;
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

// All rounds of Alg. 4 for one query by one team (see the file comment).
// With `init`, the team first empties the staircases and creates the root
// (otherwise the loop state is read from the control block as left by the
// caller).  ra[0] and ra[1] are the round arguments with the open lists
// (open_cur -> open_next) and (open_next -> open_cur); they are read through
// the pointer, so they stay in memory rather than in registers.  The LDS
// arrays are the caller's: obstacles raw/in/out
// [kMaxObs * 6] each, and small reduction scratch.
template <int N>
__device__ void explore_team(const RoundArgs* __restrict__ ra, const TeamCtx& g, bool init,
                             int n_nodes, float* s_raw,
                             float* s_in, float* s_out, int* s_w, unsigned long long* s_m,
                             long long* s_ll, int* s_fail_p) {
    constexpr int W = N / 32;
    unsigned epoch = 0;
    const int G = g.size, b = g.rank, T = blockDim.x, tid = threadIdx.x;
    const int lane = tid & 63;
    const int gwave = b * (T >> 6) + (tid >> 6), n_gwaves = G * (T >> 6);
    Ctl* c = ra[0].ctl;
    const bool leader = (b == 0 && tid == 0);
    stage_obstacles_block(ra[0].obs, ra[0].n_obs, s_raw, s_in, s_out);
    if (init) {
        // the root goes to the list the first round reads (ra[1].open_out)
        explore_init_fill(ra[1], n_nodes, (size_t)b * T + tid, (size_t)G * T);
        if (team_barrier(g, epoch, s_fail_p)) return;
        if (leader) explore_init_root(ra[1], N);
        if (team_barrier(g, epoch, s_fail_p)) return;
    }
    float gl[3], gh[3];
    for (int k = 0; k < 3; ++k) { gl[k] = ra[0].gcloud[k]; gh[k] = ra[0].gcloud[3 + k]; }
    // loop state, identical in every workgroup
    // (readfirstlane: the values are the same in every lane, so the loop
    // state and the round arguments can live in scalar registers)
    int n_pairs = uni(c->n_pairs), n_B = uni(c->n_B), n_open = uni(c->n_open);
    int n_plans = uni(c->n_plans), i_cur = uni(c->i), done = uni(c->done);
    int32_t* cur = g.open_cur;
    int32_t* nxt = g.open_next;
    int par = 0;
    long long n_sim = 0, n_pre = 0, n_drop = 0, kept = 0;
    long long w_pre = 0, w_flag = 0, w_wp = 0, w_bt = 0;     // wave-uniform
    long long partial = 0;
    int rounds = 0, err = 0;
    int fail_surv = 0;            // survivors of the round that overflowed the plan store
    // phase wall times seen by the leader (constant-rate real-time counter)
    unsigned long long t_prev = 0, ticks[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    auto tick = [&](int k) {
        const unsigned long long now = __builtin_amdgcn_s_memrealtime();
        ticks[k] += now - t_prev;
        t_prev = now;
    };
    __syncthreads();
    while (!done) {
        if ((long long)n_pairs > g.cap_pairs) {
            err = 4;
            break;
        }
        if (rounds >= (1 << 22)) {   // the loop must have ended long before
            err = 6;
            break;
        }
        // the round's arguments: ra[par] reads cur and writes nxt
        const RoundArgs& a = ra[par];
        partial += n_pairs;
        ++rounds;
        if (leader) t_prev = __builtin_amdgcn_s_memrealtime();
        // (1) expansion, one pair per lane (a wave per 64 pairs, the
        //     workgroup's waves side by side); particle simulations queued
        //     with one atomic per workgroup and pass
        for (int base = b * T; base < n_pairs; base += G * T) {
            const int tile = base + (tid & ~63);
            const int q = base + tid;
            SimTask tk;
            int st = 0;
            if (tile < n_pairs) {   // the wave's pairs
                const int grp = wave_group_of(a.b_off, n_B, tile, q);
                st = q < n_pairs ? expand_pair<N>(a, q, grp, s_raw, s_out, gl, gh, n_sim, n_pre, n_drop,
                                                  tk) : 0;
            }
            queue_pairs_block(a, st, tk, s_w);
        }
        if (team_barrier(g, epoch, s_fail_p)) break;
        if (leader) tick(0);
        // (2) particle simulation, one queued pair per wave; the leader
        //     resets the cheapest-open-cost accumulator of phase 5 (its store
        //     is written back at the next barrier)
        const int n_tasks = uni(__hip_atomic_load(&c->n_tasks, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (leader) c->min_cost_bits = 0x7FF0000000000000ull;
        for (int task = gwave; task < n_tasks; task += n_gwaves)
            simulate_pair<N>(a, task, s_raw, s_in, s_out, w_pre, w_flag, w_wp, w_bt);
        if (team_barrier(g, epoch, s_fail_p)) break;
        if (leader) tick(1);
        // (3) staircase update (atomic minima only).  The barrier after it
        //     needs no cache maintenance: phase 4 reads the staircase with
        //     atomic loads, and every other array it reads is unchanged since
        //     the barrier before this phase.
        for (int q = b * T + tid; q < n_pairs; q += G * T) stair_update_pair(a, q);
        if (team_barrier<false>(g, epoch, s_fail_p)) break;
        if (leader) tick(2);
        // (4) marks over contiguous chunks; chunk totals of the survivor and
        //     kept-open flags
        int p_lo, p_hi, o_lo, o_hi;
        chunk_of(n_pairs, b, G, p_lo, p_hi);
        chunk_of(n_open, b, G, o_lo, o_hi);
        int my_s = 0, my_k = 0;
        for (int t = p_lo + tid; t < p_hi; t += T) {
            kept += mark_pair<true>(a, t) ? 1 : 0;
            my_s += a.c_pos[t];
        }
        for (int t = o_lo + tid; t < o_hi; t += T) {
            mark_open<true>(a, t);
            my_k += a.o_keep[t];
        }
        my_s = block_sum_int(my_s, s_w);
        my_k = block_sum_int(my_k, s_w);
        // (only the totals cross workgroups here: marks and scans stay in
        //  the member's own chunks)
        XSum xs;
        if (team_exchange(g, epoch, s_fail_p, my_s, my_k, 0, s_w, xs)) break;
        if (leader) tick(3);
        // (5) scans of both flag arrays, compaction, cheapest new open plan
        const int s_before = xs.a_before, n_surv = xs.a_all;
        const int k_before = xs.b_before, n_keep = xs.b_all;
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
            fail_surv = n_surv;
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
            par ^= 1;
        }
        if (team_barrier(g, epoch, s_fail_p)) break;
        if (leader) tick(4);
        // (6) next group index; flag the group and count it per chunk.  The
        //     leader empties the simulation queue for the next round (written
        //     back at the barrier after phase 7).
        if (leader) c->n_tasks = 0;
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
        int stop = 0, my_b = 0, my_d = 0;
        for (int t = n_lo + tid; t < n_hi; t += T) {
            stop |= flag_group_one(a, t, thr) ? 1 : 0;
            if (a.o_inB[t]) {
                const int h = a.p_head[a.open_out[t]];
                ++my_b;
                my_d += a.row_ptr[h + 1] - a.row_ptr[h];
            }
        }
        my_b = block_sum_int(my_b, s_w);
        my_d = block_sum_int(my_d, s_w);
        stop = block_sum_int(stop, s_w);
        // (the flags and scans stay in the member's own chunk of the new
        //  open list; the stop flag travels with the totals)
        XSum xg;
        if (team_exchange(g, epoch, s_fail_p, my_b, my_d, stop, s_w, xg)) break;
        if (leader) tick(5);
        // (7) scans of the group flags and of the group's degrees in group
        //     order (= open-list order), per chunk: scatter of the group and
        //     its pair offsets
        const int b_before = xg.a_before, nB = xg.a_all;
        const int d_before = xg.b_before, n_pairs_next = xg.b_all;
        {
            int carry = b_before, dcarry = d_before;
            for (int t0 = n_lo; t0 < n_hi; t0 += T) {
                const int t = t0 + tid;
                const int v = t < n_hi ? a.o_keep[t] : 0;
                int dv = 0;
                if (v) {
                    const int h = a.p_head[a.open_out[t]];
                    dv = a.row_ptr[h + 1] - a.row_ptr[h];
                }
                int ex, dex;
                const int tot = block_excl(v, ex, s_w);
                const int dtot = block_excl(dv, dex, s_w);
                if (t < n_hi) a.o_keep[t] = carry + ex;
                if (v) a.b_off[carry + ex] = dcarry + dex;
                carry += tot;
                dcarry += dtot;
            }
        }
        __syncthreads();
        for (int t = n_lo + tid; t < n_hi; t += T) scatter_group_one(a, t, g.b_deg);
        if (leader) a.b_off[nB] = n_pairs_next;
        n_B = nB;
        n_pairs = n_pairs_next;
        done = xg.flag ? 1 : 0;
        if (team_barrier(g, epoch, s_fail_p)) break;
        if (leader) tick(6);
    }
    // counters and the final loop state
    const long long s_sim = block_sum_ll2(n_sim, s_ll);
    const long long s_pre = block_sum_ll2(n_pre + (lane == 0 ? w_pre : 0), s_ll);
    const long long s_drop = block_sum_ll2(n_drop, s_ll);
    const long long s_flag = block_sum_ll2(lane == 0 ? w_flag : 0, s_ll);
    const long long s_wp = block_sum_ll2(lane == 0 ? w_wp : 0, s_ll);
    const long long s_bt = block_sum_ll2(lane == 0 ? w_bt : 0, s_ll);
    const long long s_kept = block_sum_ll2(kept, s_ll);
    if (tid == 0) {
        if (s_sim) atomicAdd((unsigned long long*)&c->simulated, (unsigned long long)s_sim);
        if (s_pre) atomicAdd((unsigned long long*)&c->preprune, (unsigned long long)s_pre);
        if (s_drop) atomicAdd((unsigned long long*)&c->dropped_steps, (unsigned long long)s_drop);
        if (s_flag) atomicAdd((unsigned long long*)&c->flagged, (unsigned long long)s_flag);
        if (s_wp) atomicAdd((unsigned long long*)&c->sim_waypoints, (unsigned long long)s_wp);
        if (s_bt) atomicAdd((unsigned long long*)&c->sim_box_tests, (unsigned long long)s_bt);
        if (s_kept) atomicAdd((unsigned long long*)&c->inserted, (unsigned long long)s_kept);
    }
    if (leader) {
        const bool failed =
            __hip_atomic_load(g.fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        c->n_plans = n_plans;
        c->n_surv = fail_surv;
        c->n_open = n_open;
        c->n_B = done ? 0 : n_B;
        c->n_pairs = done ? 0 : n_pairs;
        c->i = i_cur;
        c->err = failed ? 5 : err;
        c->done = 1;
        c->rounds = rounds;
        c->partial = partial;
        c->open_final = (cur == g.open_cur) ? 0 : 1;
        for (int k = 0; k < 8; ++k) c->phase_ticks[k] += (long long)ticks[k];
    }
}

}  // namespace pump
