// C ABI of the batched engine: many planning queries of uneven size planned
// by one HIP graph launch, with an autotuner for the persistent kernel's
// shape.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <string>
#include <type_traits>
#include <vector>

#include "host_consts.hpp"
#include "pump_internal.hpp"

using namespace pump;

namespace {

constexpr int kBatchFrontHost = kMaxFront;

struct Slot {
    // per-query buffers (sized for the batch's maxima)
    float *X, *obs, *D, *cloud, *gcloud;
    uint8_t *valid, *goal, *p_state, *o_inB, *c_flag;
    uint32_t *ebits, *p_mask, *c_mask;
    int32_t *wstart, *deg, *row_ptr, *col, *esrc, *p_head, *p_parent, *p_edge, *p_step, *p_pop, *p_round;
    int32_t *open_a, *open_b, *o_keep, *b_ids, *b_off, *b_deg;
    int32_t *c_head, *c_parent, *c_edge, *c_step, *c_pop, *c_pos;
    SimTask* tasks;
    int32_t *goal_ids, *front_ids, *paths, *path_len, *wp_len, *mc_counts;
    double *etau, *ecost, *p_cost, *c_cost, *wp, *dev_scratch;
    unsigned* team_sync;
    unsigned long long* team_tot;
    unsigned long long* stair;
    SmoothState* sm_st;
    double *sm_coef, *sm_t0, *sm_wp, *sm_out;
    Ctl* ctl;
};

}  // namespace

struct pump_batch {
    pump_config cfg;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int max_q = 0, words = 0, n_cu = 0;
    size_t arena_bytes = 0;
    std::vector<Slot> slots;
    std::vector<void*> allocs;
    BatchQuery* qs_dev = nullptr;
    BatchOut* out_dev = nullptr;
    int* order_dev = nullptr;      // query of each schedule entry
    int* off_dev = nullptr;        // first slot of each entry (+ total)
    int* counter = nullptr;
    std::vector<BatchQuery> qs;
    std::vector<BatchOut> outs;
    std::vector<const pump_roadmap*> rms;   // per query (pump_batch_set_roadmaps)
    std::string err;
};

namespace {

int bfail(pump_batch* b, int code, const std::string& m) {
    if (b) b->err = m;
    return code;
}

#define BCHK(call)                                                                     \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return bfail(b, PUMP_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

}  // namespace

extern "C" {

int pump_batch_destroy(pump_batch* b) {
    if (!b) return PUMP_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (void* p : b->allocs)
        if (p) (void)hipFree(p);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return PUMP_OK;
}

int pump_batch_create(const pump_config* cfg_in, int32_t max_queries, void* hip_stream,
                      pump_batch** out) {
    if (!out || !cfg_in || max_queries < 1 || max_queries > 4096) return PUMP_E_ARG;
    *out = nullptr;
    const pump_config& cfg = *cfg_in;
    const int N = cfg.n_particles;
    if (!(N == 32 || N == 64 || N == 128 || N == 256)) return PUMP_E_ARG;
    if (cfg.cp_model != 0 && cfg.cp_model != 1) return PUMP_E_ARG;
    if (cfg.estimator != 0 && cfg.estimator != 1) return PUMP_E_ARG;
    if (cfg.smooth != 0 && cfg.smooth != 1) return PUMP_E_ARG;
    if (cfg.max_nodes < 2 || cfg.max_nodes > 65535 || cfg.max_obstacles > kMaxObs ||
        cfg.max_steps < 1 || cfg.max_steps > 4096 || cfg.mc_particles < 1)
        return PUMP_E_ARG;
    if (ceil((double)cfg.r_conn / (double)cfg.dt) > kMaxWaypoints) return PUMP_E_ARG;
    if (cfg.cap_pairs < 1 || cfg.cap_pairs > (1ll << 26) || cfg.cap_plans < 1 ||
        cfg.cap_plans > (1ll << 26) || cfg.cap_edges < 1 || cfg.cap_edges > (1ll << 31) - 1)
        return PUMP_E_ARG;
    pump_batch* b = new pump_batch();
    b->cfg = cfg;
    b->max_q = max_queries;
    if (hip_stream) {
        b->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreate(&b->stream) != hipSuccess) { delete b; return PUMP_E_HIP; }
        b->own_stream = true;
    }
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        pump_batch_destroy(b);
        return PUMP_E_HIP;
    }
    b->n_cu = prop.multiProcessorCount;
    const size_t nn = (size_t)cfg.max_nodes, S = (size_t)cfg.max_steps;
    const size_t P = (size_t)cfg.cap_plans, Q = (size_t)cfg.cap_pairs, E = (size_t)cfg.cap_edges;
    const size_t W = (size_t)N / 32;
    b->words = (int)(((nn + 63) / 64) * 2);
    // One arena holds every slot (same layout per slot, 256-byte aligned
    // arrays) and the batch descriptors; slots are sized for the largest
    // query the configuration admits.
    size_t off = 0;
    auto take = [&](auto** p, size_t n) {
        off = (off + 255) & ~(size_t)255;
        *p = reinterpret_cast<std::remove_reference_t<decltype(*p)>>(off);
        off += std::max<size_t>(n, 1) * sizeof(**p);
    };
    Slot lay{};
    take(&lay.X, nn * 6); take(&lay.obs, (size_t)kMaxObs * 6); take(&lay.D, (S + 1) * 3 * N);
    take(&lay.cloud, (S + 1) * 6);
    take(&lay.dev_scratch, (size_t)kDevScratchPer * ((S + 15) / 16) * 3 * N); take(&lay.gcloud, 8); take(&lay.valid, nn); take(&lay.goal, nn);
    take(&lay.ebits, nn * b->words); take(&lay.wstart, nn * b->words); take(&lay.deg, nn + 1); take(&lay.row_ptr, nn + 2);
    take(&lay.col, E); take(&lay.esrc, E); take(&lay.etau, E); take(&lay.ecost, E);
    take(&lay.p_head, P); take(&lay.p_parent, P); take(&lay.p_edge, P); take(&lay.p_step, P);
    take(&lay.p_pop, P); take(&lay.p_round, P); take(&lay.p_cost, P); take(&lay.p_mask, P * W);
    take(&lay.p_state, P); take(&lay.stair, nn * (N + 1)); take(&lay.open_a, P);
    take(&lay.open_b, P); take(&lay.o_keep, P); take(&lay.o_inB, P); take(&lay.b_ids, P + 1);
    take(&lay.b_off, P + 1); take(&lay.b_deg, P + 1); take(&lay.c_head, Q); take(&lay.c_parent, Q);
    take(&lay.c_edge, Q); take(&lay.c_step, Q); take(&lay.c_pop, Q); take(&lay.c_pos, Q);
    take(&lay.tasks, Q); take(&lay.c_cost, Q); take(&lay.c_mask, Q * W); take(&lay.c_flag, Q);
    take(&lay.goal_ids, (size_t)kMaxGoal); take(&lay.front_ids, kBatchFrontHost);
    take(&lay.paths, (size_t)kBatchFrontHost * (S + 1)); take(&lay.path_len, kBatchFrontHost);
    take(&lay.wp_len, kBatchFrontHost); take(&lay.mc_counts, kBatchFrontHost);
    take(&lay.wp, (size_t)kBatchFrontHost * (S + 1) * 3); take(&lay.ctl, 1);
    take(&lay.team_sync, (size_t)64 + kMaxTeam); take(&lay.team_tot, (size_t)2 * kMaxTeam);
    take(&lay.sm_st, 1); take(&lay.sm_coef, S * 12); take(&lay.sm_t0, S + 1);
    take(&lay.sm_wp, (size_t)kSmoothCands * (S + 1) * 3); take(&lay.sm_out, (S + 1) * 3);
    const size_t slot_bytes = (off + 255) & ~(size_t)255;
    off = slot_bytes * (size_t)max_queries;
    size_t o_qs, o_out, o_order, o_counter, o_off;
    {
        BatchQuery* t0; BatchOut* t1; int* t2; int* t3;
        take(&t0, (size_t)max_queries); o_qs = (size_t)t0;
        take(&t1, (size_t)max_queries); o_out = (size_t)t1;
        take(&t2, (size_t)max_queries); o_order = (size_t)t2;
        int* t4;
        take(&t4, (size_t)max_queries + kBatchGroups); o_off = (size_t)t4;
        take(&t3, kBatchGroups); o_counter = (size_t)t3;
    }
    b->arena_bytes = off;
    char* base = nullptr;
    if (hipMalloc((void**)&base, off) != hipSuccess) {
        pump_batch_destroy(b);
        return PUMP_E_HIP;
    }
    b->allocs.push_back(base);
    b->slots.resize(max_queries);
    for (int i = 0; i < max_queries; ++i) {
        char* sb = base + slot_bytes * (size_t)i;
        Slot& d = b->slots[i];
        // rebase every member of the layout onto this slot
        static_assert(sizeof(Slot) % sizeof(void*) == 0, "Slot holds pointers only");
        const uintptr_t* src = reinterpret_cast<const uintptr_t*>(&lay);
        uintptr_t* dst = reinterpret_cast<uintptr_t*>(&d);
        for (size_t k = 0; k < sizeof(Slot) / sizeof(void*); ++k)
            dst[k] = reinterpret_cast<uintptr_t>(sb) + src[k];
    }
    b->qs_dev = reinterpret_cast<BatchQuery*>(base + o_qs);
    b->out_dev = reinterpret_cast<BatchOut*>(base + o_out);
    b->order_dev = reinterpret_cast<int*>(base + o_order);
    b->off_dev = reinterpret_cast<int*>(base + o_off);
    b->counter = reinterpret_cast<int*>(base + o_counter);
    *out = b;
    return PUMP_OK;
}

int pump_batch_plan(pump_batch* b, const pump_problem* probs, const int32_t* n_particles, int32_t q,
                    const pump_batch_tuning* tune, pump_result* out) {
    if (!b || !probs || !n_particles || q < 1) return PUMP_E_ARG;
    if (q > b->max_q) return bfail(b, PUMP_E_ARG, "more queries than max_queries");
    const pump_config& cfg = b->cfg;
    pump_batch_tuning t;
    if (tune) t = *tune;
    else { t.explore_threads = 256; t.blocks_per_cu = 2; t.order = 1; t.use_graph = 1; t.team_scale = 64; }
    if (t.explore_threads != 256 ||
        t.blocks_per_cu < 1 || t.blocks_per_cu > 8 || t.team_scale < 0 || t.team_scale > 256)
        return bfail(b, PUMP_E_ARG, "bad tuning");
    b->qs.assign(q, BatchQuery());
    int N_max = 0, max_nodes = 0;
    std::vector<double> work(q);
    for (int i = 0; i < q; ++i) {
        const pump_problem& pr = probs[i];
        const int N = n_particles[i];
        if (pr.mem != PUMP_MEM_DEVICE) return bfail(b, PUMP_E_ARG, "batched inputs must be device memory");
        if (!(N == 32 || N == 64 || N == 128 || N == 256) || N > cfg.n_particles)
            return bfail(b, PUMP_E_ARG, "query " + std::to_string(i) + ": particle count");
        if (pr.n < 1 || pr.n + 1 > cfg.max_nodes || pr.n_obs < 0 || pr.n_obs > cfg.max_obstacles)
            return bfail(b, PUMP_E_ARG, "query " + std::to_string(i) + ": sizes");
        if (!(pr.alpha > 0.0f && pr.alpha < 1.0f) || !(pr.sigma >= 0.0f) || !pr.samples ||
            !pr.noise || !pr.noise_mc || (pr.n_obs > 0 && !pr.obstacles))
            return bfail(b, PUMP_E_ARG, "query " + std::to_string(i) + ": arguments");
        if (cfg.estimator == 1 && (!(pr.sigma_meas > 0.0f) || !std::isfinite(pr.sigma_meas) ||
                                   !pr.noise_meas || !pr.noise_mc_meas))
            return bfail(b, PUMP_E_ARG, "query " + std::to_string(i) +
                                            ": LQG needs sigma_meas > 0, noise_meas and noise_mc_meas");
        const Slot& s = b->slots[i];
        BatchQuery& Q = b->qs[i];
        memset(&Q, 0, sizeof(Q));
        const double alpha = (double)pr.alpha;
        const double eta = cfg.eta > 0.0f ? (double)cfg.eta : eta_rule(alpha);
        double K[2];
        tracking_constants((double)cfg.dt, (double)cfg.q_pos, (double)cfg.q_vel, (double)cfg.r_track,
                           (double)pr.sigma, K, Q.Acl, Q.L);
        Q.alpha = alpha;
        Q.r_steer = (double)cfg.r_steer;
        Q.r_conn = (double)cfg.r_conn;
        Q.N = N;
        Q.n_nodes = pr.n + 1;
        Q.words = b->words;
        Q.cap_pairs = (int32_t)cfg.cap_pairs;
        Q.cap_edges = (int32_t)std::min<int64_t>(cfg.cap_edges, (1ll << 31) - 1);
        Q.samples = pr.samples;
        Q.obs_src = reinterpret_cast<const float*>(pr.obstacles);
        Q.noise = pr.noise;
        Q.estimator = cfg.estimator;
        if (cfg.estimator == 1) {
            Q.noise_meas = pr.noise_meas;
            lqg_constants((double)cfg.dt, (double)cfg.q_pos, (double)cfg.q_vel,
                          (double)cfg.r_track, (double)pr.sigma, (double)pr.sigma_meas, Q.lqg.m,
                          Q.lqg.e);
        }
        for (int k = 0; k < 6; ++k) Q.x_init[k] = pr.x_init[k];
        for (int k = 0; k < 3; ++k) { Q.goal_box[k] = pr.goal.lo[k]; Q.goal_box[3 + k] = pr.goal.hi[k]; }
        Q.dev_scratch = s.dev_scratch;
        Q.team_sync = s.team_sync;
        Q.team_tot = s.team_tot;
        Q.sm = SmoothBuf{s.sm_st, s.sm_coef, s.sm_t0, s.sm_wp, s.sm_out};
        const pump_roadmap* rm = i < (int)b->rms.size() ? b->rms[i] : nullptr;
        if (rm) {
            if (rm->n != pr.n)
                return bfail(b, PUMP_E_ARG, "query " + std::to_string(i) + ": roadmap has " +
                                                std::to_string(rm->n) + " samples");
            Q.use_rm = 1;
            Q.rm = rm->d;
        }
        Q.X = s.X; Q.obs = s.obs; Q.valid = s.valid; Q.goal = s.goal; Q.ebits = s.ebits;
        Q.wstart = s.wstart; Q.deg = s.deg; Q.row_ptr = s.row_ptr; Q.col = s.col; Q.esrc = s.esrc; Q.etau = s.etau;
        Q.ecost = s.ecost; Q.b_deg = s.b_deg; Q.open_a = s.open_a; Q.open_b = s.open_b;
        RoundArgs& a = Q.ra[0];
        a.X = s.X; a.goal = s.goal; a.obs = s.obs; a.n_obs = pr.n_obs; a.D = s.D; a.cloud = s.cloud;
        a.gcloud = s.gcloud; a.S_max = cfg.max_steps; a.dt = (double)cfg.dt;
        cp_thresholds(alpha, eta, N, &a.c_cut, &a.c_min);
        a.h = (double)cfg.lambda * (double)cfg.r_conn;
        a.preprune = cfg.preprune;
        a.cp_model = cfg.cp_model;
        a.row_ptr = s.row_ptr; a.col = s.col; a.etau = s.etau; a.ecost = s.ecost;
        a.p_head = s.p_head; a.p_parent = s.p_parent; a.p_edge = s.p_edge; a.p_step = s.p_step;
        a.p_pop = s.p_pop; a.p_round = s.p_round; a.p_cost = s.p_cost; a.p_mask = s.p_mask;
        a.p_state = s.p_state; a.cap_plans = cfg.cap_plans; a.stair = s.stair; a.stair_w = N + 1;
        a.open_in = s.open_a; a.open_out = s.open_b; a.o_inB = s.o_inB; a.o_keep = s.o_keep;
        a.b_ids = s.b_ids; a.b_off = s.b_off; a.c_head = s.c_head; a.c_parent = s.c_parent;
        a.c_edge = s.c_edge; a.c_step = s.c_step; a.c_pop = s.c_pop; a.c_cost = s.c_cost;
        a.c_mask = s.c_mask; a.c_flag = s.c_flag; a.c_pos = s.c_pos; a.tasks = s.tasks; a.ctl = s.ctl;
        Q.ra[1] = Q.ra[0];
        Q.ra[1].open_in = s.open_b;
        Q.ra[1].open_out = s.open_a;
        SelectArgs& sa = Q.s;
        sa.X = s.X; sa.obs = s.obs; sa.n_obs = pr.n_obs; sa.goal = s.goal; sa.p_head = s.p_head;
        sa.p_parent = s.p_parent; sa.p_pop = s.p_pop; sa.p_cost = s.p_cost; sa.p_state = s.p_state;
        sa.goal_ids = s.goal_ids; sa.front_ids = s.front_ids; sa.paths = s.paths;
        sa.path_len = s.path_len; sa.wp = s.wp; sa.wp_len = s.wp_len; sa.mc_counts = s.mc_counts;
        sa.noise_mc = pr.noise_mc; sa.M = cfg.mc_particles; sa.S_max = cfg.max_steps; sa.dt = (double)cfg.dt;
        sa.r_steer = (double)cfg.r_steer;
        for (int k = 0; k < 4; ++k) { sa.Acl[k] = Q.Acl[k]; sa.L[k] = Q.L[k]; }
        sa.estimator = Q.estimator;
        sa.noise_mc_meas = cfg.estimator == 1 ? pr.noise_mc_meas : nullptr;
        sa.lqg = Q.lqg;
        sa.ctl = s.ctl;
        N_max = std::max(N_max, N);
        max_nodes = std::max(max_nodes, Q.n_nodes);
        work[i] = (double)Q.n_nodes * Q.n_nodes * sqrt((double)N);
    }
    // Schedules of the persistent Explore kernels, one per particle count:
    // entries in input order or largest first; entry i gets a team of
    // workgroups in proportion to its share of its group's estimated work
    // (team_scale / 4 times the proportional share; 0 = one workgroup per
    // query).  Teams need every workgroup of a launch resident at once, so
    // each launch is capped by its kernel's occupancy.
    std::vector<int> order, off;
    order.reserve(q);
    off.reserve(q + kBatchGroups);
    BatchGroup groups[kBatchGroups];
    int n_groups = 0;
    const int Ns[kBatchGroups] = {256, 128, 64, 32};
    for (int gi = 0; gi < kBatchGroups; ++gi) {
        std::vector<int> mem;
        for (int i = 0; i < q; ++i)
            if (b->qs[i].N == Ns[gi]) mem.push_back(i);
        if (mem.empty()) continue;
        int per_cu = t.blocks_per_cu;
        const int fit = batch_explore_per_cu(Ns[gi], t.explore_threads);
        if (fit > 0 && per_cu > fit) per_cu = fit;
        const int grid = std::max(1, b->n_cu * per_cu);
        if (t.order == 1)
            std::stable_sort(mem.begin(), mem.end(), [&](int x, int y) { return work[x] > work[y]; });
        double wsum = 0.0;
        for (int i : mem) wsum += work[i];
        const int team_cap = std::min(kMaxTeam, grid);
        BatchGroup& G = groups[n_groups++];
        G.N = Ns[gi];
        const int e0 = (int)order.size(), f0 = (int)off.size();
        off.push_back(0);
        for (int i : mem) {
            int size = 1;
            if (t.team_scale > 0 && wsum > 0.0) {
                const double share = 0.25 * t.team_scale * grid * work[i] / wsum;
                size = (int)std::min<double>(std::max(1.0, floor(share + 0.5)), (double)team_cap);
            }
            order.push_back(i);
            off.push_back(off.back() + size);
        }
        G.sch.query = b->order_dev + e0;
        G.sch.off = b->off_dev + f0;
        G.sch.n_entries = (int)mem.size();
        G.sch.total = off.back();
        G.blocks = std::max(1, std::min(G.sch.total, grid));
    }
    b->outs.assign(q, BatchOut());
    memset(b->outs.data(), 0, sizeof(BatchOut) * q);
    BCHK(hipMemcpyAsync(b->qs_dev, b->qs.data(), sizeof(BatchQuery) * q, hipMemcpyHostToDevice, b->stream));
    BCHK(hipMemcpyAsync(b->out_dev, b->outs.data(), sizeof(BatchOut) * q, hipMemcpyHostToDevice, b->stream));
    BCHK(hipMemcpyAsync(b->order_dev, order.data(), sizeof(int) * order.size(), hipMemcpyHostToDevice,
                        b->stream));
    BCHK(hipMemcpyAsync(b->off_dev, off.data(), sizeof(int) * off.size(), hipMemcpyHostToDevice,
                        b->stream));
    auto t0 = std::chrono::steady_clock::now();
    if (t.use_graph) {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        BCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        launch_batch(b->stream, b->qs_dev, q, N_max, max_nodes, cfg.max_steps, cfg.mc_particles,
                     b->words, t.explore_threads, b->counter, b->out_dev, groups, n_groups,
                     cfg.smooth != 0);
        BCHK(hipStreamEndCapture(b->stream, &graph));
        BCHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        BCHK(hipGraphLaunch(exec, b->stream));
        BCHK(hipStreamSynchronize(b->stream));
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
    } else {
        launch_batch(b->stream, b->qs_dev, q, N_max, max_nodes, cfg.max_steps, cfg.mc_particles,
                     b->words, t.explore_threads, b->counter, b->out_dev, groups, n_groups,
                     cfg.smooth != 0);
    }
    BCHK(hipGetLastError());
    BCHK(hipMemcpyAsync(b->outs.data(), b->out_dev, sizeof(BatchOut) * q, hipMemcpyDeviceToHost, b->stream));
    std::vector<Ctl> ctls(q);
    for (int i = 0; i < q; ++i)
        BCHK(hipMemcpyAsync(&ctls[i], b->slots[i].ctl, sizeof(Ctl), hipMemcpyDeviceToHost, b->stream));
    BCHK(hipStreamSynchronize(b->stream));
    const float ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    int worst = PUMP_OK;
    for (int i = 0; i < q; ++i) {
        const BatchOut& o = b->outs[i];
        pump_result r;
        memset(&r, 0, sizeof(r));
        r.status = o.status;
        r.n_goal_plans = o.n_goal;
        r.n_front = o.n_front;
        r.best = o.best;
        r.best_plan = o.best_plan;
        r.best_pop = o.best_pop;
        r.best_mc_count = o.best_mc;
        r.best_len = o.best_len;
        r.best_cost = o.best_cost;
        r.best_cp_mc = o.best_cp_mc;
        r.partial_plans = o.partial_plans;
        r.simulated = ctls[i].simulated;
        r.preprune = ctls[i].preprune;
        r.inserted = ctls[i].inserted;
        r.survivors = ctls[i].n_plans - 1;
        r.dropped_steps = ctls[i].dropped_steps;
        r.flagged = ctls[i].flagged;
        r.sim_waypoints = ctls[i].sim_waypoints;
        r.sim_box_tests = ctls[i].sim_box_tests;
        r.rounds = o.rounds;
        r.final_i = ctls[i].i;
        r.n_plans = ctls[i].n_plans;
        r.n_edges = o.n_edges;
        r.c_cut = b->qs[i].ra[0].c_cut;
        r.c_min = b->qs[i].ra[0].c_min;
        r.smooth_beta = o.smooth_beta;
        r.smooth_cost = o.smooth_cost;
        r.smooth_mc_count = o.smooth_count;
        r.smooth_steps = o.smooth_steps;
        r.ms_total = ms;
        if (out) out[i] = r;
        if (o.status < 0 && worst == PUMP_OK) {
            worst = o.status;
            b->err = "query " + std::to_string(i) + ": status " + std::to_string(o.status);
        }
    }
    return worst;
}

int pump_batch_get_path(pump_batch* b, int32_t query, int32_t plan, int32_t* nodes, int32_t cap,
                        int32_t* len) {
    if (!b || !nodes || !len || query < 0 || query >= (int)b->qs.size()) return PUMP_E_ARG;
    const Slot& s = b->slots[query];
    Ctl c;
    BCHK(hipMemcpy(&c, s.ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
    if (plan < 0 || plan >= c.n_plans) return bfail(b, PUMP_E_ARG, "plan id out of range");
    std::vector<int32_t> par(c.n_plans), head(c.n_plans);
    BCHK(hipMemcpy(par.data(), s.p_parent, (size_t)c.n_plans * 4, hipMemcpyDeviceToHost));
    BCHK(hipMemcpy(head.data(), s.p_head, (size_t)c.n_plans * 4, hipMemcpyDeviceToHost));
    std::vector<int32_t> rev;
    for (int p = plan; p >= 0; p = par[p]) {
        rev.push_back(head[p]);
        if ((int)rev.size() > c.n_plans) return bfail(b, PUMP_E_STATE, "parent cycle");
    }
    if ((int)rev.size() > cap) return bfail(b, PUMP_E_ARG, "output too small");
    *len = (int32_t)rev.size();
    for (size_t i = 0; i < rev.size(); ++i) nodes[i] = rev[rev.size() - 1 - i];
    return PUMP_OK;
}

int pump_batch_tune(pump_batch* b, const pump_problem* probs, const int32_t* n_particles, int32_t q,
                    pump_batch_tuning* best, double* best_ms, const char* json_path) {
    if (!b || !probs || !n_particles || !best) return PUMP_E_ARG;
    const int threads[1] = {256};
    const int per_cu[3] = {1, 2, 4};
    const int scales[3] = {16, 64, 256};
    std::vector<pump_result> ref(q), cur(q);
    double bms = 1e30;
    pump_batch_tuning bt{256, 2, 1, 1, 64};
    std::string js = "{\"candidates\": [";
    bool first = true;
    bool have_ref = false;
    for (int th : threads)
        for (int pc : per_cu)
            for (int sc : scales) {
                pump_batch_tuning t{th, pc, 1, 1, sc};
                int r = pump_batch_plan(b, probs, n_particles, q, &t, cur.data());
                if (r < 0) return r;
                // timed run
                auto t0 = std::chrono::steady_clock::now();
                r = pump_batch_plan(b, probs, n_particles, q, &t, cur.data());
                const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
                if (r < 0) return r;
                if (!have_ref) {
                    ref = cur;
                    have_ref = true;
                } else {
                    // the shape of the kernel must not change any result
                    for (int i = 0; i < q; ++i)
                        if (cur[i].status != ref[i].status || cur[i].best_plan != ref[i].best_plan ||
                            cur[i].best_cost != ref[i].best_cost ||
                            cur[i].partial_plans != ref[i].partial_plans)
                            return bfail(b, PUMP_E_STATE, "tuning changed a result");
                }
                char buf[200];
                snprintf(buf, sizeof(buf),
                         "%s{\"threads\": %d, \"blocks_per_cu\": %d, \"team_scale\": %d, \"ms\": %.3f}",
                         first ? "" : ", ", th, pc, sc, ms);
                js += buf;
                first = false;
                if (ms < bms) { bms = ms; bt = t; }
            }
    char buf[200];
    snprintf(buf, sizeof(buf),
             "], \"best\": {\"threads\": %d, \"blocks_per_cu\": %d, \"team_scale\": %d, \"ms\": %.3f}}",
             bt.explore_threads, bt.blocks_per_cu, bt.team_scale, bms);
    js += buf;
    if (json_path) {
        FILE* f = fopen(json_path, "w");
        if (f) { fputs(js.c_str(), f); fclose(f); }
    }
    *best = bt;
    if (best_ms) *best_ms = bms;
    return PUMP_OK;
}

const char* pump_batch_last_error(const pump_batch* b) { return b ? b->err.c_str() : ""; }

}  // extern "C"

int pump_batch_set_roadmaps(pump_batch* b, const pump_roadmap* const* rms, int32_t n) {
    if (!b || n < 0 || (n > 0 && !rms)) return PUMP_E_ARG;
    std::vector<const pump_roadmap*> v(rms, rms + n);
    for (int i = 0; i < n; ++i) {
        const pump_roadmap* rm = v[i];
        if (!rm) continue;
        if (rm->r_steer != b->cfg.r_steer || rm->r_conn != b->cfg.r_conn)
            return bfail(b, PUMP_E_ARG, "roadmap " + std::to_string(i) + ": radii differ from the batch's");
        if (rm->n + 1 > b->cfg.max_nodes)
            return bfail(b, PUMP_E_ARG, "roadmap " + std::to_string(i) + ": more samples than max_nodes - 1");
    }
    b->rms = std::move(v);
    return PUMP_OK;
}
