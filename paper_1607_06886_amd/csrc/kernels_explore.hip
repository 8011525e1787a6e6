// Explore (Alg. 4): one round = expand the group B to every neighbour,
// RemoveDominated, retire B, select the next group.
#include "device_math.hpp"
#include "pump_internal.hpp"

namespace pump {

__device__ __forceinline__ double stair_get(const unsigned long long* st, int w, int x, int c) {
    return __longlong_as_double((long long)st[(size_t)x * w + c]);
}

__device__ __forceinline__ int readlane_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ double readlane_d(double v, int l) {
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ unsigned long long lanemask_lt(int lane) {
    return lane ? ((1ull << lane) - 1ull) : 0ull;
}

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
                                                     int32_t* __restrict__ total_dev) {
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
    if (threadIdx.x == 0) *total_dev = carry;
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
                    int32_t n_upper, int32_t* total_dev, int32_t* blk) {
    int nblk = (n_upper + kScanBlock - 1) / kScanBlock;
    if (nblk < 1) nblk = 1;
    k_scan_reduce<<<nblk, 256, 0, s>>>(in, n_dev, blk);
    k_scan_blocks<<<1, 256, 0, s>>>(blk, nblk, total_dev);
    k_scan_down<<<nblk, 256, 0, s>>>(in, out, n_dev, blk);
}

// ---------------------------------------------------------------------------
// Initialisation (Alg. 4 first lines): P_open = P(x_init) = B = {root},
// root = (x_init, [], 0, 0), i = 0.  The dominance staircase of every node
// starts empty (+inf); the root puts cost 0 at every pop level of node 0.
// ---------------------------------------------------------------------------
__global__ void k_fill_u64(unsigned long long* p, size_t n, unsigned long long v) {
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

__global__ void k_root(RoundArgs a, int N) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
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
    int deg = a.row_ptr[1] - a.row_ptr[0];
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
    c->simulated = c->preprune = c->inserted = c->dropped_steps = c->flagged = 0;
}

void launch_explore_init(hipStream_t s, const RoundArgs& a, int n_nodes, int N) {
    size_t n = (size_t)n_nodes * a.stair_w;
    k_fill_u64<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(a.stair, n, 0x7FF0000000000000ull);
    k_root<<<1, 64, 0, s>>>(a, N);
}

// ---------------------------------------------------------------------------
// Expansion: every pair (p in B, x in N(p.head)) forms q = (x, p.path + head,
// p.cost + Cost(p.head, x), CP_hat(x, p)) (Alg. 4), then the CP cutoff.
//
// A wave owns 64 consecutive pairs.  Phase 1 (one pair per lane): locate the
// pair, its edge and the parent plan; cost, step count and K_e waypoints;
// drop pairs past S_max; optionally resolve pairs that the parent's own
// cp_hat already makes dominated; evaluate the nominal trajectory and mark the
// waypoints where the particle cloud's bounding box (shifted onto the nominal
// point, widened by the guard band) touches an obstacle.  Pairs with no such
// waypoint keep the parent's particle bits and are written out directly.
// Phase 2 (one pair per wave, particles across lanes): at each marked
// waypoint, lanes test their particles against the obstacles the cloud
// touches; hits are gathered with ballots into the N-bit mask, ORed with the
// parent's bits, counted, and the pair is cut if pop >= c_cut.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(256) void k_expand(RoundArgs a) {
    constexpr int W = N / 32;                      // u32 mask words
    constexpr int PPL = N >= 64 ? N / 64 : 1;      // particles per lane
    __shared__ float s_raw[kMaxObs * 6];
    __shared__ float s_in[kMaxObs * 6];            // box shrunk by the guard
    __shared__ float s_out[kMaxObs * 6];           // box grown by the guard
    const int n_obs = a.n_obs;
    for (int t = threadIdx.x; t < n_obs * 6; t += blockDim.x) {
        float v = a.obs[t];
        bool is_lo = (t % 6) < 3;
        s_raw[t] = v;
        s_in[t] = is_lo ? v + kGuard : v - kGuard;
        s_out[t] = is_lo ? v - kGuard : v + kGuard;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int n_pairs = a.ctl->n_pairs;
    const int n_B = a.ctl->n_B;
    const double dt = a.dt;
    const int c_cut = a.c_cut;
    float gl[3], gh[3];
    for (int k = 0; k < 3; ++k) { gl[k] = a.gcloud[k]; gh[k] = a.gcloud[3 + k]; }

    long long n_sim = 0, n_pre = 0, n_drop = 0, n_flag = 0;
    const int wave_global = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int wave_stride = gridDim.x * 4;
    for (int tile = wave_global * 64; tile < n_pairs; tile += wave_stride * 64) {
        const int q = tile + lane;
        // ---------------- phase 1: lane = pair ----------------
        int st = 0;                 // 0 resolved, 1 write parent bits, 2 simulate
        int p = 0, x = 0, e = 0, K = 1, s_p = 0, pop_p = 0, head = 0;
        double cost = 0.0, tau = 0.0;
        unsigned near = 0u;
        if (q < n_pairs) {
            int lo = 0, hi = n_B;  // b_off[lo] <= q < b_off[hi]
            while (hi - lo > 1) {
                int mid = (lo + hi) >> 1;
                if (a.b_off[mid] <= q) lo = mid; else hi = mid;
            }
            p = a.b_ids[lo];
            head = a.p_head[p];
            e = a.row_ptr[head] + (q - a.b_off[lo]);
            x = a.col[e];
            a.c_parent[q] = p;   // every formed pair records its identity
            a.c_head[q] = x;
            tau = a.etau[e];
            cost = a.p_cost[p] + a.ecost[e];
            K = max(1, (int)ceil(tau / dt));
            s_p = a.p_step[p];
            pop_p = a.p_pop[p];
            if (s_p + K > a.S_max) {
                st = 0;
                a.c_flag[q] = 0;
                a.c_pop[q] = -2;
                ++n_drop;
            } else if (a.preprune && stair_get(a.stair, a.stair_w, x, pop_p) < cost) {
                st = 0;
                a.c_flag[q] = 0;
                a.c_pop[q] = -1;
                ++n_pre;
            } else {
                ++n_sim;
                Cubic cs[3];
                hermite(a.X + (size_t)head * 6, a.X + (size_t)x * 6, tau, cs);
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
                    const float* b = s_out + o * 6;
                    bool ov = (elo[0] <= b[3]) & (ehi[0] >= b[0]) & (elo[1] <= b[4]) &
                              (ehi[1] >= b[1]) & (elo[2] <= b[5]) & (ehi[2] >= b[2]);
                    if (ov) { cand[o >> 6] |= 1ull << (o & 63); any = true; }
                }
                if (any) {
                    for (int k = 1; k <= K; ++k) {
                        double t = ((double)k * tau) / (double)K;
                        const float* cl = a.cloud + (size_t)(s_p + k) * 6;
                        float lo3[3], hi3[3];
                        for (int ax = 0; ax < 3; ++ax) {
                            float nom = (float)cs[ax].at(t);
                            lo3[ax] = nom + cl[ax] - 1e-6f;
                            hi3[ax] = nom + cl[3 + ax] + 1e-6f;
                        }
                        bool hitk = false;
                        for (int c = 0; c < (n_obs + 63) / 64 && !hitk; ++c) {
                            unsigned long long m = cand[c];
                            while (m && !hitk) {
                                int o = c * 64 + __ffsll((long long)m) - 1;
                                m &= m - 1ull;
                                const float* b = s_out + o * 6;
                                hitk = (lo3[0] <= b[3]) & (hi3[0] >= b[0]) & (lo3[1] <= b[4]) &
                                       (hi3[1] >= b[1]) & (lo3[2] <= b[5]) & (hi3[2] >= b[2]);
                            }
                        }
                        if (hitk) near |= 1u << (k - 1);
                    }
                }
                st = near ? 2 : 1;
            }
        }
        if (st == 1) {
            // no particle can touch an obstacle on this edge: q keeps p's bits
            a.c_flag[q] = 1;
            a.c_edge[q] = e;
            a.c_cost[q] = cost;
            a.c_step[q] = s_p + K;
            a.c_pop[q] = pop_p;
            for (int w = 0; w < W; ++w) a.c_mask[(size_t)q * W + w] = a.p_mask[(size_t)p * W + w];
        }
        // ---------------- phase 2: wave = pair, lanes = particles ----------------
        unsigned long long need = __ballot(st == 2);
        while (need) {
            const int j = __ffsll((long long)need) - 1;
            need &= need - 1ull;
            const int pj = readlane_i(p, j), xj = readlane_i(x, j), ej = readlane_i(e, j);
            const int Kj = readlane_i(K, j), spj = readlane_i(s_p, j);
            const int hj = readlane_i(head, j);
            const unsigned nj = (unsigned)readlane_i((int)near, j);
            const double tj = readlane_d(tau, j), cj = readlane_d(cost, j);
            Cubic cs[3];
            hermite(a.X + (size_t)hj * 6, a.X + (size_t)xj * 6, tj, cs);
            bool hit[PPL], deep[PPL], nearp[PPL];
            for (int r = 0; r < PPL; ++r) { hit[r] = false; deep[r] = false; nearp[r] = false; }
            unsigned wm = nj;
            while (wm) {
                const int k = __ffs((int)wm);
                wm &= wm - 1u;
                const int s = spj + k;
                const double t = ((double)k * tj) / (double)Kj;
                double nom64[3];
                float nom32[3];
                for (int ax = 0; ax < 3; ++ax) { nom64[ax] = cs[ax].at(t); nom32[ax] = (float)nom64[ax]; }
                const float* cl = a.cloud + (size_t)s * 6;
                float lo3[3], hi3[3];
                for (int ax = 0; ax < 3; ++ax) {
                    lo3[ax] = nom32[ax] + cl[ax] - 1e-6f;
                    hi3[ax] = nom32[ax] + cl[3 + ax] + 1e-6f;
                }
                float y[PPL][3];
                bool loaded = false;
                for (int c0 = 0; c0 < n_obs; c0 += 64) {
                    const int o = c0 + lane;
                    bool ov = false;
                    if (o < n_obs) {
                        const float* b = s_out + o * 6;
                        ov = (lo3[0] <= b[3]) & (hi3[0] >= b[0]) & (lo3[1] <= b[4]) &
                             (hi3[1] >= b[1]) & (lo3[2] <= b[5]) & (hi3[2] >= b[2]);
                    }
                    unsigned long long om = __ballot(ov);
                    if (om && !loaded) {
                        for (int r = 0; r < PPL; ++r) {
                            const int pj_ = r * 64 + lane;
                            for (int ax = 0; ax < 3; ++ax)
                                y[r][ax] = (N >= 64 || lane < N)
                                    ? nom32[ax] + a.D[((size_t)s * 3 + ax) * N + (pj_ % N)]
                                    : 0.0f;
                        }
                        loaded = true;
                    }
                    while (om) {
                        const int ob = c0 + __ffsll((long long)om) - 1;
                        om &= om - 1ull;
                        const float* bi = s_in + ob * 6;
                        const float* bo = s_out + ob * 6;
                        for (int r = 0; r < PPL; ++r) {
                            const float y0 = y[r][0], y1 = y[r][1], y2 = y[r][2];
                            const bool inner = (y0 >= bi[0]) & (y0 <= bi[3]) & (y1 >= bi[1]) &
                                               (y1 <= bi[4]) & (y2 >= bi[2]) & (y2 <= bi[5]);
                            const bool outer = (y0 >= bo[0]) & (y0 <= bo[3]) & (y1 >= bo[1]) &
                                               (y1 <= bo[4]) & (y2 >= bo[2]) & (y2 <= bo[5]);
                            if (inner) {
                                hit[r] = true;
                                deep[r] = true;
                            } else if (outer) {
                                // within the guard band of a face: decide in FP64
                                const int jj = r * 64 + lane;
                                if (N >= 64 || lane < N) {
                                    const float* br = s_raw + ob * 6;
                                    double dmin = INFINITY;
                                    for (int ax = 0; ax < 3; ++ax) {
                                        double yy = nom64[ax] +
                                            (double)a.D[((size_t)s * 3 + ax) * N + (jj % N)];
                                        dmin = fmin(dmin, fmin(yy - (double)br[ax],
                                                               (double)br[3 + ax] - yy));
                                    }
                                    if (dmin >= 0.0) hit[r] = true;
                                    if (dmin >= kFlagEps) deep[r] = true;
                                    if (fabs(dmin) < kFlagEps) nearp[r] = true;
                                }
                            }
                        }
                    }
                }
            }
            // gather hits into the N-bit mask and OR with the parent's bits
            uint32_t words[W];
            int popc = 0;
            long long flg = 0;
            for (int r = 0; r < PPL; ++r) {
                const bool valid_lane = (N >= 64) || (lane < N);
                unsigned long long hb = __ballot(hit[r] && valid_lane);
                unsigned long long fb = __ballot(nearp[r] && !deep[r] && valid_lane);
                if (N >= 64) {
                    uint32_t h0 = (uint32_t)hb, h1 = (uint32_t)(hb >> 32);
                    uint32_t pm0 = a.p_mask[(size_t)pj * W + 2 * r];
                    uint32_t pm1 = a.p_mask[(size_t)pj * W + 2 * r + 1];
                    words[2 * r] = pm0 | h0;
                    words[2 * r + 1] = pm1 | h1;
                    flg += __popc((uint32_t)fb & ~pm0) + __popc((uint32_t)(fb >> 32) & ~pm1);
                } else {
                    uint32_t pm0 = a.p_mask[(size_t)pj * W];
                    words[0] = pm0 | (uint32_t)hb;
                    flg += __popc((uint32_t)fb & ~pm0);
                }
            }
            for (int w = 0; w < W; ++w) popc += __popc(words[w]);
            n_flag += (lane == 0) ? flg : 0;
            const int qj = tile + j;
            bool keep = popc < c_cut;
            if (keep && a.preprune && stair_get(a.stair, a.stair_w, xj, popc) < cj) {
                keep = false;
                if (lane == 0) ++n_pre;
            }
            if (lane == 0) {
                a.c_flag[qj] = keep ? 1 : 0;
                a.c_pop[qj] = popc;
                if (keep) {
                    a.c_edge[qj] = ej;
                    a.c_cost[qj] = cj;
                    a.c_step[qj] = spj + Kj;
                }
            }
            if (keep && lane < W) {
                uint32_t v = 0;
                for (int w = 0; w < W; ++w) if (w == lane) v = words[w];
                a.c_mask[(size_t)qj * W + lane] = v;
            }
        }
    }
    // per-wave statistics
    for (int o = 32; o > 0; o >>= 1) {
        n_sim += __shfl_down(n_sim, o, 64);
        n_drop += __shfl_down(n_drop, o, 64);
        n_flag += __shfl_down(n_flag, o, 64);
    }
    // n_pre counts phase-1 lanes plus phase-2 resolutions (lane 0)
    for (int o = 32; o > 0; o >>= 1) n_pre += __shfl_down(n_pre, o, 64);
    if (lane == 0) {
        if (n_sim) atomicAdd((unsigned long long*)&a.ctl->simulated, (unsigned long long)n_sim);
        if (n_pre) atomicAdd((unsigned long long*)&a.ctl->preprune, (unsigned long long)n_pre);
        if (n_drop) atomicAdd((unsigned long long*)&a.ctl->dropped_steps, (unsigned long long)n_drop);
        if (n_flag) atomicAdd((unsigned long long*)&a.ctl->flagged, (unsigned long long)n_flag);
    }
}

void launch_expand(hipStream_t s, const RoundArgs& a, int N, int32_t n_pairs) {
    if (n_pairs <= 0) return;
    long long waves = (n_pairs + 63) / 64;
    long long blocks = (waves + 3) / 4;
    if (blocks > 65536) blocks = 65536;
    switch (N) {
        case 32: k_expand<32><<<(unsigned)blocks, 256, 0, s>>>(a); break;
        case 64: k_expand<64><<<(unsigned)blocks, 256, 0, s>>>(a); break;
        case 128: k_expand<128><<<(unsigned)blocks, 256, 0, s>>>(a); break;
        default: k_expand<256><<<(unsigned)blocks, 256, 0, s>>>(a); break;
    }
}

// ---------------------------------------------------------------------------
// RemoveDominated (Sec. IV): remove every open plan p for which some plan d
// with the same head has d.cost < p.cost and d.cp_hat <= p.cp_hat.
// Per node the library keeps the staircase M_x(c) = min{cost of plans in
// P(x) with pop <= c}; p is dominated iff M_{p.head}(p.pop) < p.cost.  Plans
// removed as dominated never change M (their dominator is counted with a
// lower cost), so M needs only insertions: one atomic minimum per kept
// candidate and level, order-independent.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_stair_update(RoundArgs a) {
    const int n_pairs = a.ctl->n_pairs;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n_pairs; q += gridDim.x * blockDim.x) {
        if (a.c_flag[q] != 1) continue;
        const int x = a.c_head[q];
        const unsigned long long bits = (unsigned long long)__double_as_longlong(a.c_cost[q]);
        for (int c = a.c_pop[q]; c < a.c_cut; ++c)
            atomicMin(&a.stair[(size_t)x * a.stair_w + c], bits);
    }
}

__global__ __launch_bounds__(256) void k_mark(RoundArgs a) {
    const int n_pairs = a.ctl->n_pairs;
    const int n_open = a.ctl->n_open;
    const int total = n_pairs + n_open;
    long long kept = 0;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
        if (t < n_pairs) {
            uint8_t f = a.c_flag[t];
            if (f == 1) {
                ++kept;
                if (stair_get(a.stair, a.stair_w, a.c_head[t], a.c_pop[t]) < a.c_cost[t]) {
                    f = 2;
                    a.c_flag[t] = 2;
                }
            }
            a.c_pos[t] = (f == 1) ? 1 : 0;
        } else {
            const int i = t - n_pairs;
            const int p = a.open_in[i];
            const bool dom = stair_get(a.stair, a.stair_w, a.p_head[p], a.p_pop[p]) < a.p_cost[p];
            const bool inB = a.o_inB[i] != 0;
            uint8_t stt = dom ? kRemoved : (inB ? kClosed : kOpen);
            a.p_state[p] = stt;
            a.o_keep[i] = (stt == kOpen) ? 1 : 0;
        }
    }
    for (int o = 32; o > 0; o >>= 1) kept += __shfl_down(kept, o, 64);
    if ((threadIdx.x & 63) == 0 && kept)
        atomicAdd((unsigned long long*)&a.ctl->inserted, (unsigned long long)kept);
}

void launch_prune(hipStream_t s, const RoundArgs& a, int N, int32_t n_pairs, int32_t n_open) {
    (void)N;
    int b1 = (n_pairs + 255) / 256;
    if (b1 < 1) b1 = 1;
    if (b1 > 16384) b1 = 16384;
    k_stair_update<<<b1, 256, 0, s>>>(a);
    int b2 = (n_pairs + n_open + 255) / 256;
    if (b2 < 1) b2 = 1;
    if (b2 > 16384) b2 = 16384;
    k_mark<<<b2, 256, 0, s>>>(a);
}

// ---------------------------------------------------------------------------
// Compaction: P_open <- (P_open \ B \ removed) U survivors; survivors are
// appended to the plan store in pair order.
// scan_total[0] = survivors, scan_total[1] = open plans kept.
// ---------------------------------------------------------------------------
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
            if (a.c_flag[t] != 1 || !fits) continue;
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
        } else {
            const int i = t - n_pairs;
            const int p = a.open_in[i];
            if (a.p_state[p] == kOpen) a.open_out[a.o_keep[i]] = p;
        }
    }
}

__global__ void k_compact_finalize(Ctl* c, int64_t cap) {
    const int n_surv = c->scan_total[0];
    const int n_keep = c->scan_total[1];
    if ((long long)c->n_plans + n_surv > cap) {
        c->err = 1;
        c->done = 1;
        return;
    }
    c->n_plans += n_surv;
    c->n_open = n_keep + n_surv;
    c->min_cost_bits = 0x7FF0000000000000ull;
    c->goal_stop = 0;
}

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
// Next group: i <- i + 1; B <- {p in P_open : p.cost <= i lambda r_n}.  When
// that B would be empty the loop only advances i, so i jumps straight to the
// smallest value that admits the cheapest open plan.  The loop test (Alg. 4
// while line) is evaluated on the new B.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_open_min(RoundArgs a) {
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
    if ((threadIdx.x & 63) == 0) atomicMin(&a.ctl->min_cost_bits, m);
}

__global__ void k_pick_i(RoundArgs a) {
    Ctl* c = a.ctl;
    if (c->err) return;
    if (c->n_open == 0) {
        c->done = 1;
        c->i = c->i + 1;
        return;
    }
    const double mc = __longlong_as_double((long long)c->min_cost_bits);
    const double h = a.h;
    if (!(mc >= 0.0 && mc < 1e300) || !(mc / h < 2.0e9)) {  // no finite cheapest open plan
        c->err = 3;
        c->done = 1;
        return;
    }
    long long k = (long long)ceil(mc / h);
    if (k < 0) k = 0;
    while (k > 0 && mc <= (double)(k - 1) * h) --k;
    while (!(mc <= (double)k * h)) ++k;
    long long inext = c->i + 1;
    c->i = (int)(k > inext ? k : inext);
}

__global__ __launch_bounds__(256) void k_flag_group(RoundArgs a) {
    const int n_open = a.ctl->n_open;
    if (a.ctl->done) return;
    const double thr = (double)a.ctl->i * a.h;
    int stop = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_open; i += gridDim.x * blockDim.x) {
        const int p = a.open_out[i];
        const bool inB = a.p_cost[p] <= thr;
        a.o_inB[i] = inB ? 1 : 0;
        a.o_keep[i] = inB ? 1 : 0;
        if (inB && a.goal[a.p_head[p]] && a.p_pop[p] < a.c_min) stop = 1;
    }
    if (__any(stop) && (threadIdx.x & 63) == 0) atomicOr(&a.ctl->goal_stop, 1);
}

__global__ __launch_bounds__(256) void k_scatter_group(RoundArgs a, int32_t* deg) {
    const int n_open = a.ctl->n_open;
    if (a.ctl->done) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_open; i += gridDim.x * blockDim.x) {
        if (!a.o_inB[i]) continue;
        const int p = a.open_out[i];
        const int pos = a.o_keep[i];
        const int h = a.p_head[p];
        a.b_ids[pos] = p;
        deg[pos] = a.row_ptr[h + 1] - a.row_ptr[h];
    }
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
    k_open_min<<<b, 256, 0, s>>>(a);
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
