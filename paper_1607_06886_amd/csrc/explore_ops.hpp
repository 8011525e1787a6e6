// Per-element operations of one Explore round (Alg. 4), shared by the
// single-query kernels (one launch per phase, whole device) and the batched
// engine (one workgroup per query).  Both drivers run these same bodies, in
// the same orders, so they produce identical plan stores.
#pragma once

#include "device_math.hpp"
#include "pump_internal.hpp"

namespace pump {

__device__ __forceinline__ double stair_get(const unsigned long long* st, int w, int x, int c) {
    return __longlong_as_double((long long)st[(size_t)x * w + c]);
}

// The same entry read with an agent-scope atomic load: current even where
// this XCD's L2 still holds the line from before other workgroups' atomic
// minima (no cache invalidation in between).
__device__ __forceinline__ double stair_get_coherent(const unsigned long long* st, int w, int x,
                                                     int c) {
    unsigned long long* p = const_cast<unsigned long long*>(st) + (size_t)x * w + c;
    return __longlong_as_double(
        (long long)__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

__device__ __forceinline__ unsigned long long lanemask_lt(int lane) {
    return lane ? ((1ull << lane) - 1ull) : 0ull;
}

__device__ __forceinline__ bool boxes_overlap(const float* lo3, const float* hi3, const float* b) {
    return (lo3[0] <= b[3]) & (hi3[0] >= b[0]) & (lo3[1] <= b[4]) & (hi3[1] >= b[1]) &
           (lo3[2] <= b[5]) & (hi3[2] >= b[2]);
}

// Obstacles as stored (raw), grown by the guard band (out), and as centre and
// half extent shrunk by the band (in: c xyz, h - kGuard xyz), the form the
// particle test takes.  FP32; the rounding of c and h is far below kGuard.
__device__ __forceinline__ void stage_obstacles_block(const float* obs, int n_obs, float* s_raw,
                                                      float* s_in, float* s_out) {
    for (int t = threadIdx.x; t < n_obs * 6; t += blockDim.x) {
        const float v = obs[t];
        const int a = t % 6;
        const bool is_lo = a < 3;
        if (s_raw) s_raw[t] = v;
        if (s_in) {
            const float lo = is_lo ? v : obs[t - 3], hi = is_lo ? obs[t + 3] : v;
            s_in[t] = is_lo ? 0.5f * (lo + hi) : 0.5f * (hi - lo) - kGuard;
        }
        s_out[t] = is_lo ? v - kGuard : v + kGuard;
    }
}

// Root plan and empty staircases (Alg. 4 first lines).  `t0`/`stride`
// distribute the staircase fill; the root itself is written by thread t0 == 0.
__device__ __forceinline__ void explore_init_fill(const RoundArgs& a, int n_nodes, size_t t0,
                                                  size_t stride) {
    const size_t n = (size_t)n_nodes * a.stair_w;
    for (size_t t = t0; t < n; t += stride) a.stair[t] = 0x7FF0000000000000ull;
}

__device__ __forceinline__ void explore_init_root(const RoundArgs& a, int N) {
    const int W = N / 32;
    a.p_head[0] = 0;
    a.p_parent[0] = -1;
    a.p_edge[0] = -1;
    a.p_step[0] = 0;
    a.p_pop[0] = 0;
    a.p_round[0] = 0;
    a.p_cost[0] = 0.0;
    a.p_state[0] = kOpen;
    for (int w = 0; w < W; ++w) a.p_mask[w] = 0u;
    for (int c = 0; c < a.c_cut && c < a.stair_w; ++c) a.stair[c] = 0ull;  // 0.0 bits
    a.open_out[0] = 0;  // the initial open list is written to open_out
    a.o_inB[0] = 1;
    a.b_ids[0] = 0;
    const int deg = a.row_ptr[1] - a.row_ptr[0];
    a.b_off[0] = 0;
    a.b_off[1] = deg;
    Ctl* c = a.ctl;
    c->n_plans = 1;
    c->n_open = 1;
    c->n_B = 1;
    c->n_pairs = deg;
    c->i = 0;
    c->goal_stop = (a.goal[0] && 0 < a.c_min) ? 1 : 0;
    c->done = c->goal_stop;
    c->err = 0;
    c->n_tasks = 0;
    c->simulated = c->preprune = c->inserted = c->dropped_steps = c->flagged = 0;
    c->sim_waypoints = c->sim_box_tests = 0;
}

// Group of pair q = tile + lane of the wave: the largest g < n_B with
// b_off[g] <= q (b_off nondecreasing, b_off[0] = 0 <= tile < n_pairs =
// b_off[n_B]).  The wave searches together: 64-way steps (one load per lane
// and a ballot each) narrow the groups down to a window of 64 that holds the
// tile's first pair, one more load brings the window's offsets into the
// lanes, and each lane counts the offsets <= q with a binary search over the
// lanes.  Only a lane whose pair lies past the window (a tile spanning more
// than 64 groups, i.e. groups of degree 0 or 1) searches on in memory.  All
// lanes must call this together.
__device__ __forceinline__ int wave_group_of(const int32_t* __restrict__ b_off, int n_B, int tile,
                                             int q) {
    const int lane = threadIdx.x & 63;
    int lo = 0, hi = n_B;                  // b_off[lo] <= tile, and tile < b_off[hi] or hi = n_B
    while (hi - lo > 64) {
        const int step = (hi - lo + 63) >> 6;
        const int idx = lo + lane * step;
        const unsigned long long le = __ballot(idx < hi && b_off[idx] <= tile);
        const int j = 63 - __clzll((long long)le);   // lane 0 always qualifies
        lo += j * step;
        hi = min(hi, lo + step);
    }
    const int idx = lo + 1 + lane;
    const int v = idx < n_B ? b_off[idx] : INT_MAX;
    int cnt = 0;                           // lanes j with v_j <= q (a prefix of the lanes)
    for (int s = 32; s >= 1; s >>= 1) {
        const int vv = __shfl(v, cnt + s - 1, 64);
        if (vv <= q) cnt += s;
    }
    if (cnt == 63 && __shfl(v, 63, 64) <= q) {
        int l2 = lo + 64, h2 = n_B;        // b_off[l2] <= q < b_off[h2]
        while (h2 - l2 > 1) {
            const int mid = (l2 + h2) >> 1;
            if (b_off[mid] <= q) l2 = mid; else h2 = mid;
        }
        return l2;
    }
    return lo + cnt;
}

// ---------------------------------------------------------------------------
// Expansion, first part (one pair per lane): pair q (q < n_pairs) of group
// lo (wave_group_of), written to candidate slot q - a.q0, its edge and parent plan; cost, step count and K_e waypoints; drop it past
// S_max; resolve it if the parent's own cp_hat already makes it dominated;
// otherwise evaluate the nominal trajectory and mark the waypoints where the
// particle cloud's bounding box, shifted onto the nominal point and widened by
// the guard band, touches an obstacle.  Returns 1 if q keeps the parent's
// bits (written here), 2 if its particles must be simulated (its queue record
// in tk), 0 if resolved.
// ---------------------------------------------------------------------------
// CP: 0 the box model, 1 the half-space model, 2 whichever a.cp_model names
// (a kernel instantiated for one model keeps only that model's registers).
template <int N, int CP = 2>
__device__ __forceinline__ int expand_pair(const RoundArgs& a, int q, int lo, const float* s_raw,
                                           const float* s_out, const float* gl, const float* gh,
                                           long long& n_sim, long long& n_pre, long long& n_drop,
                                           SimTask& tk) {
    constexpr int W = N / 32;
    const int n_obs = a.n_obs;
    const int p = a.b_ids[lo];
    const int head = a.p_head[p];
    const int e = a.row_ptr[head] + (q - a.b_off[lo]);
    const int x = a.col[e];
    const int sl = q - a.q0;   // candidate slot
    a.c_parent[sl] = p;   // every formed pair records its identity
    a.c_head[sl] = x;
    const double tau = a.etau[e];
    const double cost = a.p_cost[p] + a.ecost[e];
    const int K = max(1, (int)ceil(tau / a.dt));
    const int s_p = a.p_step[p];
    const int pop_p = a.p_pop[p];
    if (s_p + K > a.S_max) {
        a.c_flag[sl] = 0;
        a.c_pop[sl] = -2;
        ++n_drop;
        return 0;
    }
    if (a.preprune && stair_get(a.stair, a.stair_w, x, pop_p) < cost) {
        a.c_flag[sl] = 0;
        a.c_pop[sl] = -1;
        ++n_pre;
        return 0;
    }
    ++n_sim;
    Cubic cs[3];
    hermite(a.X + (size_t)head * 6, a.X + (size_t)x * 6, tau, cs);
    if (CP == 1 || (CP == 2 && a.cp_model == 1)) {
        // HSMC: mark the waypoints where some particle of the cloud box can
        // reach a plane of the local region, or come within the flag distance
        unsigned near = 0u;
        for (int k = 1; k <= K; ++k) {
            const double t = ((double)k * tau) / (double)K;
            double y[3], v[3];
            for (int ax = 0; ax < 3; ++ax) {
                y[ax] = cs[ax].at(t);
                v[ax] = cs[ax].c1 + t * (2.0 * cs[ax].c2 + t * 3.0 * cs[ax].c3);
            }
            const float* cl = a.cloud + (size_t)(s_p + k) * 6;
            unsigned long long rem[kMaxObsWords];
            all_boxes(n_obs, rem);
            double dd[3];
            while (hs_next(y, s_raw, n_obs, rem, dd)) {
                double av[3], b;
                hs_project(dd, v, av, b);
                double reach = 0.0;
                for (int ax = 0; ax < 3; ++ax)
                    reach += fmax(av[ax] * (double)cl[ax], av[ax] * (double)cl[3 + ax]);
                if (reach > b - kFlagEps * sqrt(b) - 1e-12 * (b + 1.0)) {
                    near |= 1u << (k - 1);
                    break;
                }
            }
        }
        a.c_edge[sl] = e;
        a.c_cost[sl] = cost;
        a.c_step[sl] = s_p + K;
        if (near == 0u) {
            a.c_flag[sl] = 1;
            a.c_pop[sl] = pop_p;
            for (int w = 0; w < W; ++w) a.c_mask[(size_t)sl * W + w] = a.p_mask[(size_t)p * W + w];
            return 1;
        }
        tk = SimTask{sl, p, K, near, (uint32_t)head | ((uint32_t)x << 16), s_p, tau};
        return 2;
    }
    // obstacles the cloud can reach anywhere along the edge
    float elo[3], ehi[3];
    for (int k = 0; k < 3; ++k) {
        double mn, mx;
        cubic_range(cs[k], tau, mn, mx);
        elo[k] = (float)mn + gl[k] - 1e-6f;
        ehi[k] = (float)mx + gh[k] + 1e-6f;
    }
    unsigned long long cand[kMaxObs / 64];
    bool any = false;
    for (int c = 0; c < kMaxObs / 64; ++c) cand[c] = 0ull;
    for (int o = 0; o < n_obs; ++o) {
        if (boxes_overlap(elo, ehi, s_out + o * 6)) {
            cand[o >> 6] |= 1ull << (o & 63);
            any = true;
        }
    }
    unsigned near = 0u;
    if (any) {
        const double dtk = tau / (double)K;   // waypoint spacing
        for (int k = 1; k <= K; ++k) {
            const double t = (double)k * dtk;
            const float* cl = a.cloud + (size_t)(s_p + k) * 6;
            float lo3[3], hi3[3];
            for (int ax = 0; ax < 3; ++ax) {
                const float nom = (float)cs[ax].at(t);
                lo3[ax] = nom + cl[ax] - 1e-6f;
                hi3[ax] = nom + cl[3 + ax] + 1e-6f;
            }
            bool hitk = false;
            for (int c = 0; c < (n_obs + 63) / 64 && !hitk; ++c) {
                unsigned long long m = cand[c];
                while (m && !hitk) {
                    const int o = c * 64 + __ffsll((long long)m) - 1;
                    m &= m - 1ull;
                    hitk = boxes_overlap(lo3, hi3, s_out + o * 6);
                }
            }
            if (hitk) near |= 1u << (k - 1);
        }
    }
    a.c_edge[sl] = e;
    a.c_cost[sl] = cost;
    a.c_step[sl] = s_p + K;
    if (near == 0u) {
        // no particle can touch an obstacle on this edge: q keeps p's bits
        a.c_flag[sl] = 1;
        a.c_pop[sl] = pop_p;
        for (int w = 0; w < W; ++w) a.c_mask[(size_t)sl * W + w] = a.p_mask[(size_t)p * W + w];
        return 1;
    }
    tk = SimTask{sl, p, K, near, (uint32_t)head | ((uint32_t)x << 16), s_p, tau};
    return 2;
}

// Append the workgroup's pairs with st == 2 (records tk) to the simulation
// queue (all threads call it): one global atomic per workgroup.
// s_w: [blockDim.x / 64].
__device__ __forceinline__ void queue_pairs_block(const RoundArgs& a, int st, const SimTask& tk,
                                                  int* s_w) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const unsigned long long need = __ballot(st == 2);
    if (lane == 0) s_w[w] = (int)__popcll(need);
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int k = 0; k < nw; ++k) {
            const int c = s_w[k];
            s_w[k] = tot;
            tot += c;
        }
        const int base = tot ? atomicAdd(&a.ctl->n_tasks, tot) : 0;
        for (int k = 0; k < nw; ++k) s_w[k] += base;
    }
    __syncthreads();
    if (st == 2) a.tasks[s_w[w] + (int)__popcll(need & lanemask_lt(lane))] = tk;
    __syncthreads();   // s_w is reused
}

// ---------------------------------------------------------------------------
// Expansion, second part (one queued pair per wave, particles across lanes):
// at each marked waypoint, lanes test their particles against the obstacles
// the cloud touches (FP32 with an FP64 re-test inside the guard band); hits
// are gathered into the N-bit mask, ORed with the parent's bits and counted;
// the pair is cut if pop >= c_cut.  Counters are wave-uniform (n_wp:
// waypoints tested, n_bt: waypoint-box tests, each over all particles).
//
// Lane l holds particles l, l + 64, ..., l + 64 (PPL-1), so the hit bits of
// particle row r are one wave ballot (mask words 2r and 2r+1 as they stand)
// and a waypoint's deviations are PPL coalesced loads per axis.  The loads of
// the next marked waypoint are issued before the current one is tested, and
// the parent's bits, the pair's cost and the head's staircase entries are
// loaded before the waypoint loop, so a pair costs about one memory latency
// per waypoint instead of two, plus one at its start.
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void load_deviations(const float* __restrict__ D, int s, int lane,
                                                float (&d)[(N >= 64 ? N / 64 : 1)][3]) {
    constexpr int PPL = N >= 64 ? N / 64 : 1;
    const int j = N >= 64 ? lane : (lane & (N - 1));   // N = 32: lanes 32..63 repeat (ignored)
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const float* row = D + ((size_t)s * 3 + ax) * N + j;
#pragma unroll
        for (int r = 0; r < PPL; ++r) d[r][ax] = row[r * 64];
    }
}

// Broadcast of lane k's double to the whole wave (wave-uniform result).
__device__ __forceinline__ double readlane_f64(double v, int k) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(unsigned)(bits & 0xFFFFFFFFll), k);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), k);
    return __longlong_as_double(((long long)(unsigned)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ float readlane_f32(float v, int k) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}

template <int N>
__device__ __forceinline__ void simulate_pair_box(const RoundArgs& a, int task, const float* s_raw,
                                                  const float* s_in, const float* s_out,
                                                  long long& n_pre, long long& n_flag,
                                                  long long& n_wp, long long& n_bt) {
    constexpr int W = N / 32;                      // u32 mask words
    constexpr int PPL = N >= 64 ? N / 64 : 1;      // particles per lane
    const int n_obs = a.n_obs;
    const int lane = threadIdx.x & 63;
    const bool valid_lane = (N >= 64) || (lane < N);
    const SimTask tk = a.tasks[task];
    const int qj = tk.q, pj = tk.p;
    const int hj = (int)(tk.nodes & 0xFFFFu), xj = (int)(tk.nodes >> 16);
    const double tj = tk.tau;
    const int Kj = tk.K;
    const int spj = tk.s_p;
    unsigned wm = tk.near;                         // non-zero for a queued pair
    // loads that do not depend on the waypoint loop, issued first
    int k = __ffs((int)wm);
    float dc[PPL][3], dn[PPL][3];
    load_deviations<N>(a.D, spj + k, lane, dc);
    uint32_t pm[W];
#pragma unroll
    for (int w = 0; w < W; ++w) pm[w] = a.p_mask[(size_t)pj * W + w];
    const double cj = a.c_cost[qj];
    const bool pre = a.preprune != 0;
    const int c_cut = a.c_cut;
    // staircase entries M_x(c) of the pair's head for c = lane (c < c_cut)
    double st_lane = 0.0;
    if (pre && lane < c_cut) st_lane = stair_get(a.stair, a.stair_w, xj, lane);
    // lane k-1 holds waypoint k (k = 1..K_e <= 32): its nominal position
    // (FP64 and FP32) and the particle cloud's box around it
    double my_nom[3] = {0.0, 0.0, 0.0};
    float my_n32[3] = {0.f, 0.f, 0.f}, my_lo[3] = {0.f, 0.f, 0.f}, my_hi[3] = {0.f, 0.f, 0.f};
    {
        // (reciprocals from the hardware estimate: the nominal points need
        // no exactly rounded quotient, only FP64 accuracy)
        Cubic cs[3];
        hermite_r(a.X + (size_t)hj * 6, a.X + (size_t)xj * 6, tj, recip_fast(tj), cs);
        if (lane < Kj) {
            const double t = (double)(lane + 1) * (tj * recip_fast((double)Kj));
            const float* cl = a.cloud + (size_t)(spj + lane + 1) * 6;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                my_nom[ax] = cs[ax].at(t);
                my_n32[ax] = (float)my_nom[ax];
                my_lo[ax] = my_n32[ax] + cl[ax] - 1e-6f;
                my_hi[ax] = my_n32[ax] + cl[3 + ax] + 1e-6f;
            }
        }
    }
    uint32_t hm = 0u, dm = 0u, nm = 0u;           // per particle r: hit, deep, near a face
    // one marked waypoint k with its deviations d (the next one's are in flight)
    auto test_waypoint = [&](const float (&d)[PPL][3], int kk) {
        ++n_wp;
        float nom32[3], lo3[3], hi3[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            nom32[ax] = readlane_f32(my_n32[ax], kk - 1);
            lo3[ax] = readlane_f32(my_lo[ax], kk - 1);
            hi3[ax] = readlane_f32(my_hi[ax], kk - 1);
        }
        float y[PPL][3];
#pragma unroll
        for (int r = 0; r < PPL; ++r)
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) y[r][ax] = nom32[ax] + d[r][ax];
        for (int c0 = 0; c0 < n_obs; c0 += 64) {
            const int o = c0 + lane;
            const bool ov = o < n_obs && boxes_overlap(lo3, hi3, s_out + o * 6);
            unsigned long long om = __ballot(ov);
            n_bt += __popcll(om);   // boxes tested against every particle
            while (om) {
                const int ob = c0 + __ffsll((long long)om) - 1;
                om &= om - 1ull;
                // u = max over axes of |y - c| - (h - g): u <= 0, inside by
                // more than the guard band (a hit, deep); 0 < u <= 2g,
                // within the band, decided below in FP64 (rare, so the wave
                // branches once per box rather than once per particle).  The
                // FP32 error of u is far below the band.
                const float* bc = s_in + ob * 6;
                const float cx = bc[0], cy = bc[1], cz = bc[2];
                const float hx = bc[3], hy = bc[4], hz = bc[5];
                uint32_t inb = 0u, bnd = 0u;
#pragma unroll
                for (int r = 0; r < PPL; ++r) {
                    const float u = fmaxf(fmaxf(fabsf(y[r][0] - cx) - hx, fabsf(y[r][1] - cy) - hy),
                                          fabsf(y[r][2] - cz) - hz);
                    inb |= (u <= 0.0f ? 1u : 0u) << r;
                    bnd |= (u > 0.0f && u <= 2.0f * kGuard ? 1u : 0u) << r;
                }
                hm |= inb;
                dm |= inb;
                if (!valid_lane) bnd = 0u;
                if (__ballot(bnd != 0u)) {
                    // the FP64 nominal point only where some particle needs it
                    double nom64[3];
#pragma unroll
                    for (int ax = 0; ax < 3; ++ax) nom64[ax] = readlane_f64(my_nom[ax], kk - 1);
                    const float* br = s_raw + ob * 6;
#pragma unroll
                    for (int r = 0; r < PPL; ++r) {
                        if (!(bnd & (1u << r))) continue;
                        double dmin = INFINITY;
#pragma unroll
                        for (int ax = 0; ax < 3; ++ax) {
                            // (kept inside the branch: without the empty
                            // asm the compiler hoists these FP64 sums out of
                            // the box loop for every waypoint)
                            float dv = d[r][ax];
                            asm volatile("" : "+v"(dv));
                            const double yy = nom64[ax] + (double)dv;
                            dmin = fmin(dmin, fmin(yy - (double)br[ax], (double)br[3 + ax] - yy));
                        }
                        if (dmin >= 0.0) hm |= 1u << r;
                        if (dmin >= kFlagEps) dm |= 1u << r;
                        if (fabs(dmin) < kFlagEps) nm |= 1u << r;
                    }
                }
            }
        }
    };
    // the waypoint loop unrolled by two so the in-flight buffer alternates
    // between dc and dn without copies
    // (the next load is issued unconditionally -- the last waypoint reloads
    // its own row -- so no branch has to wait for it before merging)
    //
    // Once the pair's count (the parent's bits and the hits so far) reaches
    // c_cut the pair is cut whatever the remaining waypoints add, so the loop
    // stops there: a cut pair's count is then some value >= c_cut rather than
    // its full count.
    uint32_t pml = 0u;   // the parent's bits of this lane's particles
#pragma unroll
    for (int r = 0; r < PPL; ++r) {
        // particle r * 64 + lane: bit lane of words 2r, 2r+1 taken as one 64-bit word
        const unsigned long long wv =
            N >= 64 ? ((unsigned long long)pm[(2 * r + 1) % W] << 32) | pm[(2 * r) % W] : pm[0];
        pml |= (uint32_t)((wv >> lane) & 1ull) << r;
    }
    if (!valid_lane) pml = 0u;
    auto reached_cut = [&]() {
        const uint32_t b = valid_lane ? (hm | pml) : 0u;
        int cnt = 0;
#pragma unroll
        for (int r = 0; r < PPL; ++r) cnt += (int)__popcll(__ballot((b >> r) & 1u));
        return cnt >= c_cut;
    };
    for (;;) {
        unsigned rest = wm & (wm - 1u);
        int kn = rest ? __ffs((int)rest) : 0;
        load_deviations<N>(a.D, spj + (kn ? kn : k), lane, dn);
        test_waypoint(dc, k);
        if (!kn || reached_cut()) break;
        k = kn;
        wm = rest;
        rest = wm & (wm - 1u);
        kn = rest ? __ffs((int)rest) : 0;
        load_deviations<N>(a.D, spj + (kn ? kn : k), lane, dc);
        test_waypoint(dn, k);
        if (!kn || reached_cut()) break;
        k = kn;
        wm = rest;
    }
    // particle row r's bits are ballot r: words 2r and 2r+1 (N = 32: word 0)
    uint32_t words[W];
    int popc = 0;
    long long flg = 0;
    const uint32_t fm = nm & ~dm;                  // near a face and never deep
#pragma unroll
    for (int r = 0; r < PPL; ++r) {
        const unsigned long long hb = __ballot(valid_lane && ((hm >> r) & 1u));
        const unsigned long long fb = __ballot(valid_lane && ((fm >> r) & 1u));
        if constexpr (N >= 64) {
            words[2 * r] = pm[2 * r] | (uint32_t)hb;
            words[2 * r + 1] = pm[2 * r + 1] | (uint32_t)(hb >> 32);
            flg += __popc((uint32_t)fb & ~pm[2 * r]) + __popc((uint32_t)(fb >> 32) & ~pm[2 * r + 1]);
        } else {
            words[0] = pm[0] | (uint32_t)hb;
            flg += __popc((uint32_t)fb & ~pm[0]);
        }
    }
#pragma unroll
    for (int w = 0; w < W; ++w) popc += __popc(words[w]);
    bool keep = popc < c_cut;
    if (keep && pre) {
        const double m = popc < 64 ? readlane_f64(st_lane, popc)
                                   : stair_get(a.stair, a.stair_w, xj, popc);
        if (m < cj) {
            keep = false;
            ++n_pre;
        }
    }
    if (lane == 0) {
        a.c_flag[qj] = keep ? 1 : 0;
        a.c_pop[qj] = popc;
    }
    if (keep && lane < W) {
        uint32_t v = 0;
#pragma unroll
        for (int w = 0; w < W; ++w)
            if (w == lane) v = words[w];
        a.c_mask[(size_t)qj * W + lane] = v;
    }
    if (popc < c_cut) n_flag += flg;   // flagged decisions of pairs below the cut
}

// Half-space model (Sec. III-B, eq. (7)) of the same step: per marked waypoint
// the planes of the local convex region against every particle, in FP64.
template <int N>
__device__ __forceinline__ void simulate_pair_hsmc(const RoundArgs& a, int task, const float* s_raw,
                                              long long& n_pre, long long& n_flag, long long& n_wp,
                                              long long& n_bt) {
    constexpr int W = N / 32;                      // u32 mask words
    constexpr int PPL = N >= 64 ? N / 64 : 1;      // particles per lane
    const int n_obs = a.n_obs;
    const int lane = threadIdx.x & 63;
    const bool valid_lane = (N >= 64) || (lane < N);
    const SimTask tk = a.tasks[task];
    const int qj = tk.q, pj = tk.p;
    const int hj = (int)(tk.nodes & 0xFFFFu), xj = (int)(tk.nodes >> 16);
    const double tj = tk.tau, cj = a.c_cost[qj];
    const int Kj = tk.K;
    const int spj = tk.s_p;
    const unsigned nj = tk.near;
    Cubic cs[3];
    hermite(a.X + (size_t)hj * 6, a.X + (size_t)xj * 6, tj, cs);
    bool hit[PPL], deep[PPL], nearp[PPL];
    for (int r = 0; r < PPL; ++r) { hit[r] = false; deep[r] = false; nearp[r] = false; }
    // the parent's bit of each of this lane's particles (particle r * 64 + lane)
    bool par[PPL];
    for (int r = 0; r < PPL; ++r) {
        const int j = valid_lane ? r * 64 + lane : 0;
        par[r] = valid_lane && ((a.p_mask[(size_t)pj * W + (j >> 5)] >> (j & 31)) & 1u);
    }
    unsigned wm = nj;
    {
        // at each marked waypoint, every plane of the local region against
        // every particle's deviation, in FP64; as with the box model, the
        // pair stops at the waypoint where its count reaches c_cut
        while (wm) {
            ++n_wp;   // waypoints whose cloud box meets an obstacle (or a plane)
            const int k = __ffs((int)wm);
            wm &= wm - 1u;
            const int s = spj + k;
            const double t = ((double)k * tj) / (double)Kj;
            double y[3], v[3];
            for (int ax = 0; ax < 3; ++ax) {
                y[ax] = cs[ax].at(t);
                v[ax] = cs[ax].c1 + t * (2.0 * cs[ax].c2 + t * 3.0 * cs[ax].c3);
            }
            double dy[PPL][3];
            for (int r = 0; r < PPL; ++r) {
                const int jj = valid_lane ? r * 64 + lane : 0;
                for (int ax = 0; ax < 3; ++ax) dy[r][ax] = (double)a.D[((size_t)s * 3 + ax) * N + jj];
            }
            unsigned long long rem[kMaxObsWords];
            all_boxes(n_obs, rem);
            double dd[3];
            while (hs_next_wave(y, s_raw, n_obs, rem, dd)) {
                double av[3], b;
                hs_project(dd, v, av, b);
                ++n_bt;
                const double na = sqrt(b);
                if (!(na > 0.0)) continue;
                for (int r = 0; r < PPL; ++r) {
                    const double g = (av[0] * dy[r][0] + av[1] * dy[r][1]) + av[2] * dy[r][2];
                    const double mg = (g - b) / na;
                    if (g > b) hit[r] = true;
                    if (mg >= kFlagEps) deep[r] = true;
                    if (fabs(mg) < kFlagEps) nearp[r] = true;
                }
            }
            int cnt = 0;
            for (int r = 0; r < PPL; ++r) cnt += (int)__popcll(__ballot(valid_lane && (hit[r] || par[r])));
            if (cnt >= a.c_cut) break;
        }
    }
    // gather hits into the N-bit mask and OR with the parent's bits
    uint32_t words[W];
    int popc = 0;
    long long flg = 0;
    for (int r = 0; r < PPL; ++r) {
        const unsigned long long hb = __ballot(hit[r] && valid_lane);
        const unsigned long long fb = __ballot(nearp[r] && !deep[r] && valid_lane);
        if (N >= 64) {
            const uint32_t pm0 = a.p_mask[(size_t)pj * W + 2 * r];
            const uint32_t pm1 = a.p_mask[(size_t)pj * W + 2 * r + 1];
            words[2 * r] = pm0 | (uint32_t)hb;
            words[2 * r + 1] = pm1 | (uint32_t)(hb >> 32);
            flg += __popc((uint32_t)fb & ~pm0) + __popc((uint32_t)(fb >> 32) & ~pm1);
        } else {
            const uint32_t pm0 = a.p_mask[(size_t)pj * W];
            words[0] = pm0 | (uint32_t)hb;
            flg += __popc((uint32_t)fb & ~pm0);
        }
    }
    for (int w = 0; w < W; ++w) popc += __popc(words[w]);
    bool keep = popc < a.c_cut;
    if (keep && a.preprune && stair_get(a.stair, a.stair_w, xj, popc) < cj) {
        keep = false;
        ++n_pre;
    }
    if (lane == 0) {
        a.c_flag[qj] = keep ? 1 : 0;
        a.c_pop[qj] = popc;
    }
    if (keep && lane < W) {
        uint32_t v = 0;
        for (int w = 0; w < W; ++w)
            if (w == lane) v = words[w];
        a.c_mask[(size_t)qj * W + lane] = v;
    }
    if (popc < a.c_cut) n_flag += flg;   // flagged decisions of pairs below the cut
}


// One queued pair: the box predicate (default) or the half-space model.
template <int N>
__device__ __forceinline__ void simulate_pair(const RoundArgs& a, int task, const float* s_raw,
                                              const float* s_in, const float* s_out,
                                              long long& n_pre, long long& n_flag, long long& n_wp,
                                              long long& n_bt) {
    if (a.cp_model == 1)
        simulate_pair_hsmc<N>(a, task, s_raw, n_pre, n_flag, n_wp, n_bt);
    else
        simulate_pair_box<N>(a, task, s_raw, s_in, s_out, n_pre, n_flag, n_wp, n_bt);
}

// ---------------------------------------------------------------------------
// RemoveDominated (Sec. IV): remove every open plan p for which some plan d
// with the same head has d.cost < p.cost and d.cp_hat <= p.cp_hat.  Per node
// the library keeps the staircase M_x(c) = min{cost of plans in P(x) with
// pop <= c}; p is dominated iff M_{p.head}(p.pop) < p.cost.  Plans removed as
// dominated never change M (their dominator is counted with a lower cost), so
// M needs only insertions: one atomic minimum per kept candidate and level.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void stair_update_pair(const RoundArgs& a, int q) {
    if (a.c_flag[q] != 1) return;
    const int x = a.c_head[q];
    const unsigned long long bits = (unsigned long long)__double_as_longlong(a.c_cost[q]);
    for (int c = a.c_pop[q]; c < a.c_cut; ++c) atomicMin(&a.stair[(size_t)x * a.stair_w + c], bits);
}

// Candidate q: dominated -> flag 2; scan input = survivor.  Returns whether q
// was kept before the test (counts toward `inserted`).  kCoherent: read the
// staircase with atomic loads (the team loop, whose barrier after the
// staircase update does not invalidate the caches).
template <bool kCoherent = false>
__device__ __forceinline__ bool mark_pair(const RoundArgs& a, int t) {
    uint8_t f = a.c_flag[t];
    bool kept = false;
    if (f == 1) {
        kept = true;
        const int x = a.c_head[t], c = a.c_pop[t];
        const double m = kCoherent ? stair_get_coherent(a.stair, a.stair_w, x, c)
                                   : stair_get(a.stair, a.stair_w, x, c);
        if (m < a.c_cost[t]) {
            f = 2;
            a.c_flag[t] = 2;
        }
    }
    a.c_pos[t] = (f == 1) ? 1 : 0;
    return kept;
}

// Open entry i: removed if dominated, closed if in B (P_open \ B), else kept.
template <bool kCoherent = false>
__device__ __forceinline__ void mark_open(const RoundArgs& a, int i) {
    const int p = a.open_in[i];
    const int x = a.p_head[p], c = a.p_pop[p];
    const double m = kCoherent ? stair_get_coherent(a.stair, a.stair_w, x, c)
                               : stair_get(a.stair, a.stair_w, x, c);
    const bool dom = m < a.p_cost[p];
    const bool inB = a.o_inB[i] != 0;
    const uint8_t stt = dom ? kRemoved : (inB ? kClosed : kOpen);
    a.p_state[p] = stt;
    a.o_keep[i] = (stt == kOpen) ? 1 : 0;
}

// Compaction: survivors are appended to the plan store in pair order after
// the kept open plans (c_pos / o_keep hold exclusive scans).
template <int W>
__device__ __forceinline__ void compact_pair(const RoundArgs& a, int t, int n_plans, int n_keep,
                                             int i_round) {
    if (a.c_flag[t] != 1) return;
    const int r = a.c_pos[t];
    const int id = n_plans + r;
    a.p_head[id] = a.c_head[t];
    a.p_parent[id] = a.c_parent[t];
    a.p_edge[id] = a.c_edge[t];
    a.p_step[id] = a.c_step[t];
    a.p_pop[id] = a.c_pop[t];
    a.p_round[id] = i_round;
    a.p_cost[id] = a.c_cost[t];
    a.p_state[id] = kOpen;
    for (int w = 0; w < W; ++w) a.p_mask[(size_t)id * W + w] = a.c_mask[(size_t)t * W + w];
    a.open_out[n_keep + r] = id;
}

__device__ __forceinline__ void compact_open(const RoundArgs& a, int i) {
    const int p = a.open_in[i];
    if (a.p_state[p] == kOpen) a.open_out[a.o_keep[i]] = p;
}

// After compaction (one thread): publish the new counts; err on overflow.
__device__ __forceinline__ void compact_finalize(Ctl* c, int64_t cap) {
    const int n_surv = c->scan_total[0];
    const int n_keep = c->scan_total[1];
    if ((long long)c->n_plans + n_surv > cap) {
        c->err = 1;
        c->done = 1;
        c->n_surv = n_surv;   // the plan store needs n_plans + n_surv entries
        return;
    }
    c->n_plans += n_surv;
    c->n_open = n_keep + n_surv;
    c->min_cost_bits = 0x7FF0000000000000ull;
    c->goal_stop = 0;
}

// Next group (one thread): i <- i + 1; when that group would be empty the
// loop only advances i, so i jumps to the first value admitting the cheapest
// open plan (cost <= i lambda r_n).
__device__ __forceinline__ void pick_next_i(Ctl* c, double h) {
    if (c->err) return;
    if (c->n_open == 0) {
        c->done = 1;
        c->i = c->i + 1;
        return;
    }
    const double mc = __longlong_as_double((long long)c->min_cost_bits);
    if (!(mc >= 0.0 && mc < 1e300) || !(mc / h < 2.0e9)) {  // no finite cheapest open plan
        c->err = 3;
        c->done = 1;
        return;
    }
    long long k = (long long)ceil(mc / h);
    if (k < 0) k = 0;
    while (k > 0 && mc <= (double)(k - 1) * h) --k;
    while (!(mc <= (double)k * h)) ++k;
    const long long inext = c->i + 1;
    c->i = (int)(k > inext ? k : inext);
}

// Open entry i of the new list: in B?  (scan input in o_keep).  Returns
// whether it stops the loop (a goal plan of B with cp_hat < alpha_min).
__device__ __forceinline__ bool flag_group_one(const RoundArgs& a, int i, double thr) {
    const int p = a.open_out[i];
    const bool inB = a.p_cost[p] <= thr;
    a.o_inB[i] = inB ? 1 : 0;
    a.o_keep[i] = inB ? 1 : 0;
    return inB && a.goal[a.p_head[p]] && a.p_pop[p] < a.c_min;
}

__device__ __forceinline__ void scatter_group_one(const RoundArgs& a, int i, int32_t* deg) {
    if (!a.o_inB[i]) return;
    const int p = a.open_out[i];
    const int pos = a.o_keep[i];
    const int h = a.p_head[p];
    a.b_ids[pos] = p;
    deg[pos] = a.row_ptr[h + 1] - a.row_ptr[h];
}

}  // namespace pump
