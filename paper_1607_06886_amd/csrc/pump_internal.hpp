// Internal declarations shared by the libpump translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "pump.h"

namespace pump {

constexpr int kMaxObs = 256;          // obstacle boxes per query
constexpr int kMaxWaypoints = 32;     // ceil(r_n / dt) bound (u32 waypoint masks)
constexpr int kScanBlock = 1024;      // items per block in the device-wide scans
constexpr int kMaxFront = 256;        // Pareto front entries handled by selection
// Patience of a team-barrier wait, in ticks of the 100 MHz real-time counter:
// 4 s unless the host sets another bound.
constexpr unsigned long long kDefaultPatience = 400000000ull;
constexpr int kMaxGoal = 1 << 16;     // goal plans gathered for selection
// FP32 guard band of the particle test: a particle whose FP32 position is
// within kGuard of a face is re-tested in FP64 (2^-14, far above the FP32
// error of a position of magnitude <= 16).
constexpr float kGuard = 6.103515625e-05f;
constexpr double kFlagEps = 1e-5;     // face distance counted as a flagged decision
constexpr double kTauMin = 1e-6;      // connections shorter than this are skipped

enum PlanState : uint8_t { kOpen = 0, kClosed = 1, kRemoved = 2 };

// LQG tracking of one axis (eq. (2) with a Kalman estimate): the state
// z = (dp, dv, p_hat, v_hat) follows z' = m z + e (xi_p0, xi_p1, xi_m),
// m row-major 4x4 and e row-major 4x3.
struct LqgCoef {
    double m[16];
    double e[12];
};

// One step of that recurrence in FP64.
__device__ __forceinline__ void lqg_step(const LqgCoef& q, double z[4], double w0, double w1,
                                         double w2) {
    double zn[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        zn[i] = q.m[4 * i] * z[0] + q.m[4 * i + 1] * z[1] + q.m[4 * i + 2] * z[2] +
                q.m[4 * i + 3] * z[3] + (q.e[3 * i] * w0 + q.e[3 * i + 1] * w1 + q.e[3 * i + 2] * w2);
#pragma unroll
    for (int i = 0; i < 4; ++i) z[i] = zn[i];
}

// Device-resident control block of the Explore loop.
struct Ctl {
    int32_t n_plans;
    int32_t n_open;
    int32_t n_B;
    int32_t n_pairs;
    int32_t i;
    int32_t done;
    int32_t goal_stop;
    int32_t err;
    int32_t n_keep_open;
    int32_t n_surv;
    int32_t n_goal;
    int32_t n_front;
    int32_t n_tasks;           // pairs queued for particle simulation this round
    int32_t pad_;
    unsigned long long min_cost_bits;
    long long simulated;
    long long preprune;
    long long inserted;
    long long dropped_steps;
    long long flagged;
    int32_t scan_total[8];
    long long partial;         // pairs formed by the single-launch Explore
    int32_t rounds;            // rounds run by the single-launch Explore
    int32_t open_final;        // which open-list buffer it left current (0/1)
    long long phase_ticks[8];  // its phase wall times (real-time counter ticks)
    long long sim_waypoints;   // simulated (pair, waypoint) tests, each over N particles
    long long sim_box_tests;   // simulated (pair, waypoint, box) tests, each over N particles
    // PlanSelection outcome (k_select_final)
    int32_t sel_status;        // PUMP_OK, PUMP_NO_GOAL_PLAN or PUMP_INFEASIBLE
    int32_t sel_best;          // front index of p* (-1: none)
    int32_t sel_plan;          // plan id of p*
    int32_t sel_mc;            // its Monte Carlo count
    int32_t sel_len;           // its node count
    int32_t sel_steps;         // its waypoint steps
    int32_t sel_pop;           // its cp_hat count
    int32_t sel_bad_wp;        // some front plan has more than S_max steps
    int32_t n_valid;           // valid nodes
    int32_t pad2_;
    double sel_cost;           // cost of p*
    // a round run in chunks: the current chunk's pair count and the
    // survivors of the chunks before it
    int32_t chunk_n;
    int32_t chunk_base;
};

// A pair queued for particle simulation, with what the simulation needs of
// it (written by the expansion, so the simulation reads one record instead of
// chasing the pair's parent and edge through the plan store and the graph).
struct SimTask {
    int32_t q;                 // pair index
    int32_t p;                 // parent plan
    int32_t K;                 // waypoints on the edge, ceil(tau / dt) (at most 32)
    uint32_t near;             // waypoints whose cloud box meets an obstacle (bit k-1)
    uint32_t nodes;            // edge endpoints: head | x << 16 (node ids < 65536)
    int32_t s_p;               // parent's step count
    double tau;                // edge duration
};
static_assert(sizeof(SimTask) == 32, "SimTask is two 16-byte loads");

// Counter partials of the per-phase Explore kernels: workgroup b of a kernel
// adds its sums to part[b * kPartK + k] (its own slot, no atomics), and one
// small kernel per round adds the slots into the control block and clears
// them.  Grids of those kernels stay within kPartSlots workgroups.
constexpr int kPartSlots = 4096;
constexpr int kPartK = 8;
enum PartCounter : int {
    kPartSimulated = 0, kPartPreprune = 1, kPartDropped = 2, kPartFlagged = 3,
    kPartWaypoints = 4, kPartBoxTests = 5, kPartInserted = 6
};

// Kernel arguments of one Explore round.
struct RoundArgs {
    // problem
    const float* X;            // [n_nodes][6]
    const uint8_t* goal;       // [n_nodes]
    const float* obs;          // [n_obs][6]
    int32_t n_obs;
    const float* D;            // [S_max+1][3][N]
    const float* cloud;        // [S_max+1][6] (lo xyz, hi xyz) of D over particles
    const float* gcloud;       // [6] union of cloud over all steps
    int32_t S_max;
    double dt;
    int32_t c_cut, c_min;
    double h;                  // lambda * r_n
    int32_t preprune;
    int32_t cp_model;          // exploration collision model: 0 box, 1 half-space (HSMC)
    // graph
    const int32_t* row_ptr;
    const int32_t* col;
    const double* etau;
    const double* ecost;
    // plans
    int32_t* p_head;
    int32_t* p_parent;
    int32_t* p_edge;
    int32_t* p_step;
    int32_t* p_pop;
    int32_t* p_round;
    double* p_cost;
    uint32_t* p_mask;
    uint8_t* p_state;
    int64_t cap_plans;
    unsigned long long* stair; // [n_nodes][N+1] min cost with pop <= c (FP64 bits)
    int32_t stair_w;
    // open list and group
    const int32_t* open_in;
    int32_t* open_out;
    uint8_t* o_inB;
    int32_t* o_keep;           // scan input/output over the open list
    int32_t* b_ids;
    int32_t* b_off;            // [n_B + 1]
    // candidates (slot = pair index)
    int32_t* c_head;
    int32_t* c_parent;
    int32_t* c_edge;
    int32_t* c_step;
    int32_t* c_pop;
    double* c_cost;
    uint32_t* c_mask;
    uint8_t* c_flag;
    int32_t* c_pos;            // scan input/output over the pairs
    SimTask* tasks;            // pairs queued for particle simulation
    Ctl* ctl;
    // a round run in chunks (more pairs than candidate slots): pair q of the
    // round is slot q - q0 (q0 = 0 otherwise); quiet = 1 in the second pass
    // over the chunks, whose expansion adds nothing to the counters
    // per-workgroup counter partials of the per-phase kernels
    // ([kPartSlots][kPartK], summed into the control block once a round)
    long long* part;
    int32_t chunked;           // 1: the launch covers pairs q0 .. q0 + ctl->chunk_n - 1
    int32_t q0;
    int32_t quiet;
};

// Work lists of BuildGraph's pass 1 (setup_ops.hpp): the near list lives in
// the final edge arrays (free until pass 2), the exact queue in two Explore
// candidate arrays (free until Explore).
struct GraphWork {
    int32_t* near_src;         // near connections [near_cap]
    int32_t* near_dst;
    double* near_tau;
    int32_t* xq_edge;          // (connection, box) pairs for the exact test [xq_cap]
    int32_t* xq_box;
    int32_t* counts;           // [0] near, [1] exact queue (device)
    int32_t near_cap, xq_cap;
};

// ---- launchers (kernels_*.hip) ----
// scratch: kDevScratchPer * ceil(S_max / 16) * 3 * N doubles
constexpr int kDevScratchPer = 8;
void launch_deviation_table(hipStream_t s, const float* noise, float* D, float* cloud,
                            float* gcloud, int N, int S_max, const double* Acl,
                            const double* L, double* scratch);
// The same table under LQG tracking: noise_meas [S_max][3][N].
void launch_deviation_table_lqg(hipStream_t s, const float* noise, const float* noise_meas,
                                float* D, float* cloud, float* gcloud, int N, int S_max,
                                const LqgCoef& q, double* scratch);
// The obstacle-independent part of BuildGraph over a fixed sample set
// (roadmap_ops.hpp): every Near connection between samples with its tau*,
// c* and nominal position range.  Node numbering as in a query (samples are
// nodes 1..n; row 0 is empty).
struct RoadmapDev {
    const float* X;            // [n + 1][6] (row 0 unused)
    const int32_t* row_ptr;    // [n + 2]
    const int32_t* col;        // [E], ascending within a row
    const int32_t* esrc;       // [E]
    const double* tau;         // [E]
    const double* cost;        // [E]
    const double* bbox;        // [E][6] nominal position range (lo xyz, hi xyz)
    int32_t n_nodes;           // n + 1
    int32_t n_edges;
};
void launch_rm_bbox(hipStream_t s, const float* X, const int32_t* esrc, const int32_t* col,
                    const double* tau, double* bbox, int E);
// Pass 1 from a roadmap (ebits cleared here), then the row degrees; bit 4 of
// *bad when the query's samples differ from it.  gw.counts must be zero.
void launch_rm_query(hipStream_t s, const float* X, const uint8_t* valid, int n_nodes,
                     const float* obs, int n_obs, double r_steer, double r_conn,
                     const RoadmapDev& rm, uint32_t* ebits, int words, int32_t* deg, int32_t* bad,
                     const GraphWork& gw);
// Pass 1 over cached connections (src, dst, tau, nominal range) plus the
// pairs at node 0 (kernels_setup.hip).
void launch_graph_pass1_roadmap(hipStream_t s, const float* X, const uint8_t* valid, int n_nodes,
                                const float* obs, int n_obs, double r_steer, double r_conn,
                                const int32_t* rm_src, const int32_t* rm_dst,
                                const double* rm_tau, const double* rm_bbox, int rm_edges,
                                uint32_t* ebits, int32_t* deg, int words, const GraphWork& gw);
void launch_rm_fill(hipStream_t s, const float* X, int n_nodes, double r_steer,
                    const int32_t* row_ptr, const int32_t* col, const int32_t* esrc,
                    const RoadmapDev& rm, double* etau, double* ecost, int n_edges);
// Pass 2 of BuildGraph without the edge controls (col and esrc only).
void launch_graph_cols(hipStream_t s, int n_nodes, const uint32_t* ebits, const int32_t* row_ptr,
                       int32_t* col, int32_t* esrc, int words);

// Halton points start .. start + n - 1 over the box [lo, hi] (6 floats each)
// into out [n][6] (kernels_sample.hip).
hipError_t launch_halton(hipStream_t s, int64_t start, int32_t n, const float* lo, const float* hi,
                         float* out);
void launch_mark_valid(hipStream_t s, const float* X, int n_nodes, const float* obs,
                       int n_obs, const float* goal_box, uint8_t* valid, uint8_t* goal,
                       int32_t* bad);
// BuildGraph pass 1 from scratch: the edge bit matrix (cleared here) and the
// row degrees.  gw.counts must be zero.
void launch_graph_mark(hipStream_t s, const float* X, const uint8_t* valid, int n_nodes,
                       const float* obs, int n_obs, double r_steer, double r_conn,
                       uint32_t* ebits, int32_t* deg, int words, const GraphWork& gw);
void launch_graph_fill(hipStream_t s, const float* X, int n_nodes, double r_steer,
                       const uint32_t* ebits, const int32_t* row_ptr, int32_t* col,
                       int32_t* esrc, double* etau, double* ecost, int words, int n_edges);
// The same from the pass-1 near list (gw, which aliases esrc / col / etau),
// without steering the edges again; wstart: n_nodes * words ints of scratch.
void launch_graph_fill_near(hipStream_t s, const float* X, int n_nodes, double r_steer,
                            const uint32_t* ebits, const int32_t* row_ptr, int32_t* col,
                            int32_t* esrc, double* etau, double* ecost, int32_t* wstart, int words,
                            int n_edges, const GraphWork& gw);

// The total goes to *total_dev and, if given, also to *total2_dev.
void scan_exclusive(hipStream_t s, const int32_t* in, int32_t* out, const int32_t* n_dev,
                    int32_t n_upper, int32_t* total_dev, int32_t* blk_scratch,
                    int32_t* total2_dev = nullptr);

// Also clears the control block and n_zero words at `zero` (the single
// launch's barrier words).
void launch_explore_init(hipStream_t s, const RoundArgs& a, int n_nodes, int N, unsigned* zero,
                         int n_zero);
// part: 1 the pair stage, 2 the particle stage, 3 both
void launch_expand(hipStream_t s, const RoundArgs& a, int N, int32_t n_pairs, int part = 3);
void launch_prune(hipStream_t s, const RoundArgs& a, int N, int32_t n_pairs, int32_t n_open);
void launch_compact(hipStream_t s, const RoundArgs& a, int N, int32_t n_pairs,
                    int32_t n_open, int32_t* blk_scratch);
void launch_next_group(hipStream_t s, const RoundArgs& a, int32_t n_open_upper,
                       int32_t* deg_scratch, int32_t* blk_scratch);
// A round in chunks (a.chunked = 1): chunk_begin sets the chunk's pair count
// (and empties the simulation queue) before its expansion; stair_update after
// each pass-1 expansion; open_compact once between the passes; chunk_compact
// after each pass-2 expansion; chunks_finalize at the end.
void launch_chunk_begin(hipStream_t s, const RoundArgs& a, int32_t n);
void launch_stair_update(hipStream_t s, const RoundArgs& a, int32_t n);
void launch_open_compact(hipStream_t s, const RoundArgs& a, int32_t n_open, int32_t* blk_scratch);
void launch_chunk_compact(hipStream_t s, const RoundArgs& a, int N, int32_t n, int32_t* blk_scratch);
void launch_chunks_finalize(hipStream_t s, const RoundArgs& a);
// Adds the counter partials into the control block and clears them; clear
// only drops them (start of Explore).
void launch_counters_reduce(hipStream_t s, const RoundArgs& a);
void launch_counters_clear(hipStream_t s, const RoundArgs& a);

struct SelectArgs {
    const float* X;
    const float* obs;
    int32_t n_obs;
    const uint8_t* goal;
    const int32_t* p_head;
    const int32_t* p_parent;
    const int32_t* p_pop;
    const double* p_cost;
    const uint8_t* p_state;
    int32_t n_plans;
    int32_t* goal_ids;     // [kMaxGoal]
    int32_t* front_ids;    // [kMaxFront]
    int32_t* paths;        // [kMaxFront][S_max+1] node sequences
    int32_t* path_len;     // [kMaxFront]
    double* wp;            // [kMaxFront][S_max+1][3] nominal waypoints
    int32_t* wp_len;       // [kMaxFront] steps
    int32_t* mc_counts;    // [kMaxFront]
    const float* noise_mc; // [S_max][6][M]
    int32_t M;
    int32_t S_max;
    double dt;
    double r_steer;
    double Acl[4];
    double L[4];
    int32_t estimator;           // 0 LQR, 1 LQG (then noise_mc_meas and lqg are used)
    const float* noise_mc_meas;  // [S_max][3][M]
    LqgCoef lqg;
    Ctl* ctl;
    const uint8_t* valid;        // [n_nodes] (k_select_final counts them)
    int32_t n_nodes;
};

// ---- Smooth(p*, alpha) (smooth_ops.hpp) ----
constexpr int kSmoothLevels = 9;           // bisection steps
constexpr int kSmoothRounds = kSmoothLevels / 3;
constexpr int kSmoothCands = 8;            // candidate weights per round

// Device state of one query's Smooth.
struct SmoothState {
    double lo, hi;            // bisection interval (lo: certified side)
    double T_p, tau_q;        // plan and optimal-connection durations
    double plan_cost;         // cost of p*
    double qc[12];            // optimal connection cubic, per axis (c0, c1, c2, c3)
    double beta, cost;        // result
    int32_t E;                // edges of p* (0: nothing to smooth)
    int32_t f_best;           // front index of p* (-1: none)
    int32_t done;             // search finished
    int32_t lo_cnt, lo_K;     // MC count and steps of the blend at lo
    int32_t count, steps;     // result
    int32_t cnt[kSmoothCands], K[kSmoothCands];
};

struct SmoothBuf {
    SmoothState* st;
    double* e_coef;           // [S_max][3][4] edge cubics of p*
    double* e_t0;             // [S_max + 1] edge start times, e_t0[E] = T_p
    double* wp;               // [kSmoothCands][S_max + 1][3] candidate waypoints
    double* out_wp;           // [S_max + 1][3] waypoints of the result
};

void launch_smooth(hipStream_t s, const SelectArgs& a, const SmoothBuf& b, int f_best,
                   const double* plan_cost, double alpha, int plan_count, int plan_steps);

// Grid barrier state of the single-launch Explore (zeroed before launch).
struct CoopSync {
    unsigned* arrive;          // [n_blocks] last barrier each workgroup reached
    unsigned* release;         // last barrier workgroup 0 released
    int* fail;                 // set when a wait ran out of patience
    unsigned n_blocks;
    unsigned long long patience;   // longest barrier wait, 100 MHz ticks
};

struct CoopArgs {
    CoopSync sync;
    unsigned long long* xa;    // [grid] exchanged chunk totals (zero at launch)
    unsigned long long* xb;    // [grid]
    int32_t* b_deg;            // group degrees (scatter output)
    int32_t* open_cur;         // open list read by the first round
    int32_t* open_next;
    int64_t cap_pairs;
};

// Single-launch Explore (every workgroup resident: the grid is sized by the
// occupancy query).
// ra_dev: two round-argument blocks in device memory, open lists
// (open_cur -> open_next) and (open_next -> open_cur).
hipError_t launch_explore_coop(hipStream_t s, const RoundArgs* ra_dev, const CoopArgs& ca, int N,
                               int blocks);
int coop_max_blocks(int N);

// One query of the batched engine: its round and selection state plus the
// graph-build buffers and inputs, all in device memory.
struct BatchQuery {
    RoundArgs ra[2];           // round arguments: open lists (a -> b) and (b -> a)
    SelectArgs s;
    const float* samples;      // [n][6] caller's device array
    const float* obs_src;      // [n_obs][6] caller's device array
    const float* noise;        // [S_max][6][N] caller's device array
    const float* noise_meas;   // [S_max][3][N] caller's device array (LQG only)
    int32_t estimator;         // 0 LQR, 1 LQG
    LqgCoef lqg;
    float x_init[6];
    float goal_box[6];
    double Acl[4], L[4];
    double alpha;
    double r_steer, r_conn;
    int32_t N, n_nodes, words;
    int32_t cap_pairs, cap_edges;
    int32_t bad;               // input / capacity errors (bit flags)
    int32_t gcount[4];         // graph-build work-list counters (zero on upload)
    int32_t use_rm;            // 1: the graph comes from `rm` (cached roadmap)
    RoadmapDev rm;
    float* X;
    float* obs;
    uint8_t* valid;
    uint8_t* goal;
    uint32_t* ebits;
    int32_t* wstart;           // pass 2: CSR slot of each bit-matrix word's first edge
    int32_t* deg;
    int32_t* row_ptr;
    int32_t* col;
    int32_t* esrc;
    double* etau;
    double* ecost;
    int32_t* b_deg;
    int32_t* open_a;
    int32_t* open_b;
    double* dev_scratch;       // deviation-table chunk states
    SmoothBuf sm;              // Smooth(p*, alpha) state and buffers
    unsigned* team_sync;       // [64 + kMaxTeam] team barrier words (release, fail, arrivals)
    unsigned long long* team_tot;   // [2 * kMaxTeam] team exchange words (zeroed per batch)
};

constexpr int kMaxTeam = 64;   // workgroups planning one batched query

// Schedule of the persistent Explore kernel: entry e plans query query[e]
// with the workgroups holding slots off[e] .. off[e + 1] - 1.
struct BatchSched {
    const int32_t* query;      // [n_entries]
    const int32_t* off;        // [n_entries + 1]
    int32_t n_entries;
    int32_t total;             // off[n_entries]
};

// Per-query outcome written by the batched engine.
struct BatchOut {
    int32_t status, n_goal, n_front, best, best_plan, best_pop, best_mc, best_len;
    double best_cost, best_cp_mc;
    int32_t n_plans, n_edges, rounds, final_i, err, bad;
    long long partial_plans;
    double smooth_beta, smooth_cost;
    int32_t smooth_count, smooth_steps;
};

// The persistent Explore runs once per particle count present: group g
// plans the queries of its schedule with `blocks` workgroups of the kernel
// for N (counters: one queue counter per group).
constexpr int kBatchGroups = 4;   // N = 32, 64, 128, 256
struct BatchGroup {
    int N;
    int blocks;
    BatchSched sch;
};
void launch_batch(hipStream_t s, BatchQuery* qs_dev, int q, int N_max, int max_nodes, int S_max,
                  int M, int words, int explore_threads, int* counters, BatchOut* out,
                  const BatchGroup* groups, int n_groups, bool smooth);
// Workgroups of the batched Explore kernel for N that fit on one CU at once.
int batch_explore_per_cu(int N, int threads);

// P_goal and its front; scratch: an int per plan (free after Explore), blk:
// the scan's block scratch.
void launch_select_front(hipStream_t s, const SelectArgs& a, int32_t* scratch, int32_t* blk);
// n_paths < 0: the front just built (its size read on the device).
void launch_waypoints(hipStream_t s, const SelectArgs& a, int32_t n_paths);
void launch_mc(hipStream_t s, const SelectArgs& a, int32_t n_paths);
// Alg. 5's bisection over the certified front, on the device: fills the
// sel_* fields and n_valid of the control block.
void launch_select_final(hipStream_t s, const SelectArgs& a, double alpha);

}  // namespace pump

// A roadmap owned by the caller (pump_roadmap_create): device arrays, the
// radii it was built with and its sample count.
struct pump_roadmap {
    pump::RoadmapDev d;
    float* X = nullptr;
    int32_t *row_ptr = nullptr, *col = nullptr, *esrc = nullptr;
    double *tau = nullptr, *cost = nullptr, *bbox = nullptr;
    float r_steer = 0.0f, r_conn = 0.0f;
    int32_t n = 0;
    float ms_build = 0.0f;
};
