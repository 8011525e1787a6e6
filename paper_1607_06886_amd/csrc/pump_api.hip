// C ABI of libpump: context, problem setup, the Explore loop and
// PlanSelection (Alg. 2-5).  Host code only orchestrates; every step of the
// planner runs in the kernels of kernels_*.hip.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "host_consts.hpp"
#include "pump_internal.hpp"

using namespace pump;

// Words of the single launch's barrier allocation (see pump_ctx::coop_sync).
constexpr size_t kCoopSyncWords = 64 + 4096 + 4 * 4096;

struct pump_ctx {
    pump_config cfg;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int N = 0, W = 0;
    int words_per_row = 0;  // edge bit-matrix row length (u32)
    // problem
    float* X = nullptr;
    uint8_t* valid = nullptr;
    uint8_t* goal = nullptr;
    float* obs = nullptr;
    float* noise_buf = nullptr;
    float* noise_mc_buf = nullptr;
    const float* noise = nullptr;
    const float* noise_mc = nullptr;
    float* noise_meas_buf = nullptr;     // LQG only
    float* noise_mc_meas_buf = nullptr;  // LQG only
    const float* noise_meas = nullptr;
    const float* noise_mc_meas = nullptr;
    LqgCoef lqg;
    float* D = nullptr;
    double* dev_scratch = nullptr;  // deviation-table chunk states
    float* cloud = nullptr;
    float* gcloud = nullptr;
    int32_t* dev_ints = nullptr;  // [0] n_nodes, [1] bad-input flag
    // graph
    uint32_t* ebits = nullptr;
    int32_t* wstart = nullptr;  // pass 2: CSR slot of each bit-matrix word's first edge
    int32_t* deg = nullptr;
    int32_t* row_ptr = nullptr;
    int32_t* col = nullptr;
    int32_t* esrc = nullptr;
    double* etau = nullptr;
    double* ecost = nullptr;
    // plans
    int32_t *p_head = nullptr, *p_parent = nullptr, *p_edge = nullptr, *p_step = nullptr,
            *p_pop = nullptr, *p_round = nullptr;
    double* p_cost = nullptr;
    uint32_t* p_mask = nullptr;
    uint8_t* p_state = nullptr;
    unsigned long long* stair = nullptr;
    int32_t *open_a = nullptr, *open_b = nullptr, *o_keep = nullptr;
    uint8_t* o_inB = nullptr;
    int32_t *b_ids = nullptr, *b_off = nullptr, *b_deg = nullptr;
    // candidates
    int32_t *c_head = nullptr, *c_parent = nullptr, *c_edge = nullptr, *c_step = nullptr,
            *c_pop = nullptr, *c_pos = nullptr;
    SimTask* tasks = nullptr;          // simulation queue records
    double* c_cost = nullptr;
    uint32_t* c_mask = nullptr;
    uint8_t* c_flag = nullptr;
    int32_t* blk = nullptr;
    long long* part = nullptr;      // [kPartSlots][kPartK] counter partials
    // grid barrier and exchange words: release word, failure flag (words 0-63),
    // arrival words [4096], then the 64-bit exchange words [2][coop_blocks]
    unsigned* coop_sync = nullptr;
    int coop_blocks = 0;            // resident workgroups of the single-launch Explore
    int explore_mode = 0;           // 0: one launch per phase, 1: single launch, 2: by graph size
    unsigned long long patience = kDefaultPatience;   // single launch's barrier waits (100 MHz ticks)
    long long fallbacks = 0;        // single launches that timed out and were redone per phase
    RoundArgs* ra_dev = nullptr;    // [2] round arguments of the single launch
    RoundArgs* ra_h = nullptr;      // [2] pinned staging
    Ctl* ctl = nullptr;
    Ctl* ctl_h = nullptr;  // pinned mirror
    int32_t* stage_h = nullptr;   // pinned: [0] n_nodes up; [4..9) flags, counters and edges down
    float* xinit_h = nullptr;     // pinned: x_init on its way to node 0
    // selection
    int32_t *goal_ids = nullptr, *front_ids = nullptr, *paths = nullptr, *path_len = nullptr,
            *wp_len = nullptr, *mc_counts = nullptr;
    double* wp = nullptr;
    // Smooth(p*, alpha)
    SmoothBuf sm{nullptr, nullptr, nullptr, nullptr, nullptr};
    int last_best = -1;        // front index of the last p* (-1: none)
    int last_steps = 0;        // tracking steps of the trajectory returned last
    bool last_smoothed = false;
    const pump_roadmap* rm = nullptr;  // cached Near connections (pump_set_roadmap)
    // query state
    int n_nodes = 0, n_obs = 0, M = 0, S_max = 0;
    double alpha = 0, eta = 0, alpha_min = 0, alpha_max = 0, h = 0, dt = 0;
    int c_cut = 0, c_min = 0;
    double Acl[4] = {0, 0, 0, 0}, L[4] = {0, 0, 0, 0}, K[2] = {0, 0};
    int n_edges = 0, n_valid = 0;
    bool have_setup = false, have_explore = false, explore_done = false;
    int32_t* open_cur = nullptr;
    int32_t* open_next = nullptr;
    long long partial_plans = 0;
    int32_t last_pairs = 0;
    int32_t last_chunks = 1;        // chunks the last round ran in (1: in one piece)
    long long chunked_rounds = 0;   // rounds of this Explore run in chunks
    int rounds = 0;
    float ms_setup = 0, ms_explore = 0, ms_select = 0;
    // 0/4 setup begin/end, 1/2 Explore, 2/3 selection, 5/6 pump_plan
    hipEvent_t ev[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    bool setup_time_pending = false;   // ms_setup not yet read from ev[0], ev[4]
    std::string err;
    // per-kernel timing
    bool timing = false;
    double t_ms[PUMP_TIMING_KINDS] = {0};
    long long t_n[PUMP_TIMING_KINDS] = {0};
    struct Pend { int kind; hipEvent_t a, b; };
    std::vector<Pend> pending;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
};

namespace {

int fail(pump_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

#define HIPCHK(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(ctx, PUMP_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <class T>
hipError_t dalloc(T** p, size_t n) {
    if (n == 0) n = 1;
    return hipMalloc((void**)p, n * sizeof(T));
}

RoundArgs round_args(pump_ctx* c) {
    RoundArgs a;
    memset(&a, 0, sizeof(a));
    a.X = c->X;
    a.goal = c->goal;
    a.obs = c->obs;
    a.n_obs = c->n_obs;
    a.D = c->D;
    a.cloud = c->cloud;
    a.gcloud = c->gcloud;
    a.S_max = c->S_max;
    a.dt = c->dt;
    a.c_cut = c->c_cut;
    a.c_min = c->c_min;
    a.h = c->h;
    a.preprune = c->cfg.preprune;
    a.cp_model = c->cfg.cp_model;
    a.row_ptr = c->row_ptr;
    a.col = c->col;
    a.etau = c->etau;
    a.ecost = c->ecost;
    a.p_head = c->p_head;
    a.p_parent = c->p_parent;
    a.p_edge = c->p_edge;
    a.p_step = c->p_step;
    a.p_pop = c->p_pop;
    a.p_round = c->p_round;
    a.p_cost = c->p_cost;
    a.p_mask = c->p_mask;
    a.p_state = c->p_state;
    a.cap_plans = c->cfg.cap_plans;
    a.stair = c->stair;
    a.stair_w = c->N + 1;
    a.open_in = c->open_cur;
    a.open_out = c->open_next;
    a.o_inB = c->o_inB;
    a.o_keep = c->o_keep;
    a.b_ids = c->b_ids;
    a.b_off = c->b_off;
    a.c_head = c->c_head;
    a.c_parent = c->c_parent;
    a.c_edge = c->c_edge;
    a.c_step = c->c_step;
    a.c_pop = c->c_pop;
    a.c_cost = c->c_cost;
    a.c_mask = c->c_mask;
    a.c_flag = c->c_flag;
    a.c_pos = c->c_pos;
    a.tasks = c->tasks;
    a.part = c->part;
    a.ctl = c->ctl;
    return a;
}

SelectArgs select_args(pump_ctx* c) {
    SelectArgs a;
    memset(&a, 0, sizeof(a));
    a.X = c->X;
    a.obs = c->obs;
    a.n_obs = c->n_obs;
    a.goal = c->goal;
    a.p_head = c->p_head;
    a.p_parent = c->p_parent;
    a.p_pop = c->p_pop;
    a.p_cost = c->p_cost;
    a.p_state = c->p_state;
    a.n_plans = c->ctl_h->n_plans;
    a.goal_ids = c->goal_ids;
    a.front_ids = c->front_ids;
    a.paths = c->paths;
    a.path_len = c->path_len;
    a.wp = c->wp;
    a.wp_len = c->wp_len;
    a.mc_counts = c->mc_counts;
    a.noise_mc = c->noise_mc;
    a.M = c->M;
    a.S_max = c->S_max;
    a.dt = c->dt;
    a.r_steer = (double)c->cfg.r_steer;
    for (int k = 0; k < 4; ++k) { a.Acl[k] = c->Acl[k]; a.L[k] = c->L[k]; }
    a.estimator = c->cfg.estimator;
    a.noise_mc_meas = c->noise_mc_meas;
    a.lqg = c->lqg;
    a.ctl = c->ctl;
    a.valid = c->valid;
    a.n_nodes = c->n_nodes;
    return a;
}

// Timing brackets: tbeg/tend around a launch group when timing is on.
void tbeg(pump_ctx* c, int kind) {
    if (!c->timing) return;
    if (c->pool.empty()) {
        hipEvent_t a = nullptr, b = nullptr;
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
        c->pool.push_back({a, b});
    }
    auto pr = c->pool.back();
    c->pool.pop_back();
    (void)hipEventRecord(pr.first, c->stream);
    c->pending.push_back({kind, pr.first, pr.second});
}

void tend(pump_ctx* c) {
    if (!c->timing || c->pending.empty()) return;
    (void)hipEventRecord(c->pending.back().b, c->stream);
}

// After a stream synchronisation: accumulate the finished brackets.
void tresolve(pump_ctx* c) {
    if (c->setup_time_pending &&
        hipEventElapsedTime(&c->ms_setup, c->ev[0], c->ev[4]) == hipSuccess)
        c->setup_time_pending = false;
    for (auto& p : c->pending) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            c->t_ms[p.kind] += ms;
            c->t_n[p.kind] += 1;
        }
        c->pool.push_back({p.a, p.b});
    }
    c->pending.clear();
}

int read_ctl(pump_ctx* ctx) {
    HIPCHK(hipMemcpyAsync(ctx->ctl_h, ctx->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    tresolve(ctx);
    return PUMP_OK;
}

bool finite6(const float* x) {
    for (int k = 0; k < 6; ++k)
        if (!std::isfinite(x[k])) return false;
    return true;
}

}  // namespace

extern "C" {

void pump_config_default(pump_config* c) {
    if (!c) return;
    memset(c, 0, sizeof(*c));
    c->n_particles = 128;
    c->max_nodes = 4001;
    c->max_obstacles = 64;
    c->max_steps = 512;
    c->mc_particles = 10000;
    c->preprune = 1;
    c->dt = 0.05f;
    c->q_pos = 100.0f;
    c->q_vel = 10.0f;
    c->r_track = 1.0f;
    c->r_steer = 0.1f;
    c->r_conn = 1.0f;
    c->eta = 0.0f;
    c->lambda = 0.5f;
    c->cp_model = 0;
    c->estimator = 0;
    c->smooth = 0;
    c->reserved_ = 0;
    c->cap_edges = 4 << 20;
    c->cap_plans = 1 << 20;
    c->cap_pairs = 4 << 20;
}

const char* pump_status_str(int s) {
    switch (s) {
        case PUMP_OK: return "ok";
        case PUMP_INFEASIBLE: return "infeasible: no plan of the front certified";
        case PUMP_NO_GOAL_PLAN: return "no plan reached the goal region";
        case PUMP_E_ARG: return "invalid argument";
        case PUMP_E_CAPACITY: return "capacity exceeded";
        case PUMP_E_HIP: return "HIP runtime error";
        case PUMP_E_STATE: return "call out of order";
        default: return "unknown status";
    }
}

const char* pump_last_error(const pump_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

int pump_destroy(pump_ctx* ctx) {
    if (!ctx) return PUMP_OK;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    void* ptrs[] = {ctx->X, ctx->valid, ctx->goal, ctx->obs, ctx->noise_buf, ctx->noise_mc_buf,
                    ctx->noise_meas_buf, ctx->noise_mc_meas_buf,
                    ctx->D, ctx->cloud, ctx->gcloud, ctx->dev_ints, ctx->ebits, ctx->wstart, ctx->deg,
                    ctx->row_ptr, ctx->col, ctx->esrc, ctx->etau, ctx->ecost, ctx->p_head, ctx->p_parent,
                    ctx->p_edge, ctx->p_step, ctx->p_pop, ctx->p_round, ctx->p_cost, ctx->p_mask,
                    ctx->p_state, ctx->stair, ctx->open_a, ctx->open_b, ctx->o_keep, ctx->o_inB,
                    ctx->b_ids, ctx->b_off, ctx->b_deg, ctx->c_head, ctx->c_parent, ctx->c_edge,
                    ctx->c_step, ctx->c_pop, ctx->c_pos, ctx->tasks, ctx->c_cost, ctx->c_mask, ctx->c_flag,
                    ctx->blk, ctx->part, ctx->ctl, ctx->goal_ids, ctx->front_ids, ctx->paths,
                    ctx->path_len, ctx->wp_len, ctx->mc_counts, ctx->wp, ctx->sm.st,
                    ctx->sm.e_coef, ctx->sm.e_t0, ctx->sm.wp, ctx->sm.out_wp, ctx->coop_sync,
                    ctx->ra_dev};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (ctx->ctl_h) (void)hipHostFree(ctx->ctl_h);
    if (ctx->ra_h) (void)hipHostFree(ctx->ra_h);
    if (ctx->stage_h) (void)hipHostFree(ctx->stage_h);
    if (ctx->xinit_h) (void)hipHostFree(ctx->xinit_h);
    for (auto& e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& p : ctx->pending) ctx->pool.push_back({p.a, p.b});
    for (auto& p : ctx->pool) {
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return PUMP_OK;
}

int pump_create(const pump_config* cfg_in, void* hip_stream, pump_ctx** out) {
    if (!out) return PUMP_E_ARG;
    *out = nullptr;
    pump_config cfg;
    if (cfg_in) cfg = *cfg_in; else pump_config_default(&cfg);
    const int N = cfg.n_particles;
    if (!(N == 32 || N == 64 || N == 128 || N == 256)) return PUMP_E_ARG;
    if (cfg.max_nodes < 2 || cfg.max_nodes > 65535) return PUMP_E_ARG;
    if (cfg.cp_model != 0 && cfg.cp_model != 1) return PUMP_E_ARG;
    if (cfg.estimator != 0 && cfg.estimator != 1) return PUMP_E_ARG;
    if (cfg.smooth != 0 && cfg.smooth != 1) return PUMP_E_ARG;
    if (cfg.max_obstacles < 0 || cfg.max_obstacles > kMaxObs) return PUMP_E_ARG;
    if (cfg.max_steps < 1 || cfg.max_steps > 4096 || cfg.mc_particles < 1) return PUMP_E_ARG;
    if (!(cfg.dt > 0) || !(cfg.r_conn > 0) || !(cfg.lambda > 0) || !(cfg.r_steer > 0) ||
        !(cfg.r_track > 0) || !(cfg.q_pos >= 0) || !(cfg.q_vel >= 0))
        return PUMP_E_ARG;
    if (ceil((double)cfg.r_conn / (double)cfg.dt) > kMaxWaypoints) return PUMP_E_ARG;
    if (cfg.cap_pairs < 1 || cfg.cap_pairs > (1ll << 26) || cfg.cap_plans < 1 ||
        cfg.cap_plans > (1ll << 26) || cfg.cap_edges < 1 || cfg.cap_edges > (1ll << 31) - 1)
        return PUMP_E_ARG;
    pump_ctx* ctx = new pump_ctx();
    ctx->cfg = cfg;
    ctx->N = N;
    ctx->W = N / 32;
    if (hip_stream) {
        ctx->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreate(&ctx->stream) != hipSuccess) { delete ctx; return PUMP_E_HIP; }
        ctx->own_stream = true;
    }
    const size_t nn = (size_t)cfg.max_nodes;
    const size_t S = (size_t)cfg.max_steps;
    const size_t M = (size_t)cfg.mc_particles;
    const size_t P = (size_t)cfg.cap_plans;
    const size_t Q = (size_t)cfg.cap_pairs;
    const size_t E = (size_t)cfg.cap_edges;
    ctx->words_per_row = (int)(((nn + 63) / 64) * 2);
    bool ok = true;
    auto A = [&](hipError_t e) { ok = ok && (e == hipSuccess); };
    A(dalloc(&ctx->X, nn * 6));
    A(dalloc(&ctx->valid, nn));
    A(dalloc(&ctx->goal, nn));
    A(dalloc(&ctx->obs, (size_t)kMaxObs * 6));
    A(dalloc(&ctx->noise_buf, S * 6 * N));
    A(dalloc(&ctx->noise_mc_buf, S * 6 * M));
    A(dalloc(&ctx->D, (S + 1) * 3 * N));
    if (cfg.estimator == 1) {
        A(dalloc(&ctx->noise_meas_buf, S * 3 * N));
        A(dalloc(&ctx->noise_mc_meas_buf, S * 3 * M));
    }
    A(dalloc(&ctx->dev_scratch, (size_t)kDevScratchPer * ((S + 15) / 16) * 3 * N));
    A(dalloc(&ctx->cloud, (S + 1) * 6));
    A(dalloc(&ctx->gcloud, 8));
    A(dalloc(&ctx->dev_ints, 8));
    A(dalloc(&ctx->ebits, nn * ctx->words_per_row));
    A(dalloc(&ctx->wstart, nn * ctx->words_per_row));
    A(dalloc(&ctx->deg, nn + 1));
    A(dalloc(&ctx->row_ptr, nn + 2));
    A(dalloc(&ctx->col, E));
    A(dalloc(&ctx->esrc, E));
    A(dalloc(&ctx->etau, E));
    A(dalloc(&ctx->ecost, E));
    A(dalloc(&ctx->p_head, P));
    A(dalloc(&ctx->p_parent, P));
    A(dalloc(&ctx->p_edge, P));
    A(dalloc(&ctx->p_step, P));
    A(dalloc(&ctx->p_pop, P));
    A(dalloc(&ctx->p_round, P));
    A(dalloc(&ctx->p_cost, P));
    A(dalloc(&ctx->p_mask, P * ctx->W));
    A(dalloc(&ctx->p_state, P));
    A(dalloc(&ctx->stair, nn * (N + 1)));
    A(dalloc(&ctx->open_a, P));
    A(dalloc(&ctx->open_b, P));
    A(dalloc(&ctx->o_keep, P));
    A(dalloc(&ctx->o_inB, P));
    A(dalloc(&ctx->b_ids, P + 1));
    A(dalloc(&ctx->b_off, P + 1));
    A(dalloc(&ctx->b_deg, P + 1));
    A(dalloc(&ctx->c_head, Q));
    A(dalloc(&ctx->c_parent, Q));
    A(dalloc(&ctx->c_edge, Q));
    A(dalloc(&ctx->c_step, Q));
    A(dalloc(&ctx->c_pop, Q));
    A(dalloc(&ctx->c_pos, Q));
    A(dalloc(&ctx->tasks, Q));
    A(dalloc(&ctx->c_cost, Q));
    A(dalloc(&ctx->c_mask, Q * ctx->W));
    A(dalloc(&ctx->c_flag, Q));
    A(dalloc(&ctx->blk, (size_t)2 * 65536));
    A(dalloc(&ctx->part, (size_t)kPartSlots * kPartK));
    A(hipMemset(ctx->part, 0, sizeof(long long) * kPartSlots * kPartK));
    {
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess) ctx->coop_blocks = coop_max_blocks(N);
        // one workgroup per CU (PUMP_SINGLE_LAUNCH_WG_PER_CU may raise it):
        // each barrier costs a cache write-back and invalidation per
        // workgroup, which outweighs the extra waves of a second workgroup
        int per_cu = 1;
        if (const char* e = getenv("PUMP_SINGLE_LAUNCH_WG_PER_CU")) per_cu = atoi(e) >= 1 ? atoi(e) : 1;
        int n_cu = 0;
        if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            n_cu > 0 && ctx->coop_blocks > per_cu * n_cu)
            ctx->coop_blocks = per_cu * n_cu;
        if (ctx->coop_blocks > 4096) ctx->coop_blocks = 4096;
        ctx->explore_mode = ctx->coop_blocks > 0 ? 2 : 0;
    }
    A(dalloc(&ctx->coop_sync, (size_t)kCoopSyncWords));
    A(dalloc(&ctx->ra_dev, 2));
    A(hipHostMalloc((void**)&ctx->ra_h, 2 * sizeof(RoundArgs), hipHostMallocDefault));
    A(dalloc(&ctx->ctl, 1));
    A(dalloc(&ctx->goal_ids, (size_t)kMaxGoal));
    A(dalloc(&ctx->front_ids, (size_t)kMaxFront));
    A(dalloc(&ctx->paths, (size_t)kMaxFront * (S + 1)));
    A(dalloc(&ctx->path_len, (size_t)kMaxFront));
    A(dalloc(&ctx->wp_len, (size_t)kMaxFront));
    A(dalloc(&ctx->mc_counts, (size_t)kMaxFront));
    A(dalloc(&ctx->sm.st, 1));
    A(dalloc(&ctx->sm.e_coef, S * 12));
    A(dalloc(&ctx->sm.e_t0, S + 1));
    A(dalloc(&ctx->sm.wp, (size_t)kSmoothCands * (S + 1) * 3));
    A(dalloc(&ctx->sm.out_wp, (S + 1) * 3));
    A(dalloc(&ctx->wp, (size_t)kMaxFront * (S + 1) * 3));
    A(hipHostMalloc((void**)&ctx->ctl_h, sizeof(Ctl), hipHostMallocDefault));
    A(hipHostMalloc((void**)&ctx->stage_h, 16 * sizeof(int32_t), hipHostMallocDefault));
    A(hipHostMalloc((void**)&ctx->xinit_h, 8 * sizeof(float), hipHostMallocDefault));
    for (auto& e : ctx->ev) A(hipEventCreate(&e));
    if (!ok) {
        pump_destroy(ctx);
        return PUMP_E_HIP;
    }
    memset(ctx->ctl_h, 0, sizeof(Ctl));
    *out = ctx;
    return PUMP_OK;
}

int pump_setup(pump_ctx* ctx, const pump_problem* pr) {
    if (!ctx || !pr) return PUMP_E_ARG;
    ctx->have_setup = ctx->have_explore = ctx->explore_done = false;
    const pump_config& cfg = ctx->cfg;
    if (pr->n < 1 || pr->n + 1 > cfg.max_nodes) return fail(ctx, PUMP_E_ARG, "n out of range for max_nodes");
    if (ctx->rm && pr->n != ctx->rm->n)
        return fail(ctx, PUMP_E_ARG, "the problem has " + std::to_string(pr->n) + " samples, the roadmap " +
                                         std::to_string(ctx->rm->n));
    if (pr->n_obs < 0 || pr->n_obs > cfg.max_obstacles) return fail(ctx, PUMP_E_ARG, "n_obs exceeds max_obstacles");
    if (!pr->samples || (pr->n_obs > 0 && !pr->obstacles) || !pr->noise || !pr->noise_mc)
        return fail(ctx, PUMP_E_ARG, "null input pointer");
    if (!(pr->alpha > 0.0f && pr->alpha < 1.0f)) return fail(ctx, PUMP_E_ARG, "alpha must lie in (0, 1)");
    if (!(pr->sigma >= 0.0f) || !std::isfinite(pr->sigma)) return fail(ctx, PUMP_E_ARG, "sigma must be finite and >= 0");
    if (cfg.estimator == 1) {
        if (!(pr->sigma_meas > 0.0f) || !std::isfinite(pr->sigma_meas))
            return fail(ctx, PUMP_E_ARG, "LQG needs a finite sigma_meas > 0");
        if (!pr->noise_meas || !pr->noise_mc_meas)
            return fail(ctx, PUMP_E_ARG, "LQG needs noise_meas and noise_mc_meas");
    }
    if (!finite6(pr->x_init)) return fail(ctx, PUMP_E_ARG, "x_init not finite");
    for (int k = 0; k < 3; ++k) {
        if (fabsf(pr->x_init[k]) > 16.0f) return fail(ctx, PUMP_E_ARG, "x_init outside [-16, 16]");
        if (!(pr->goal.lo[k] <= pr->goal.hi[k])) return fail(ctx, PUMP_E_ARG, "goal box empty");
    }
    if (pr->mem != PUMP_MEM_HOST && pr->mem != PUMP_MEM_DEVICE) return fail(ctx, PUMP_E_ARG, "mem flag");
    const hipMemcpyKind kind = pr->mem == PUMP_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    if (pr->mem == PUMP_MEM_HOST) {
        for (int o = 0; o < pr->n_obs; ++o) {
            const pump_aabb& b = pr->obstacles[o];
            for (int k = 0; k < 3; ++k) {
                if (!std::isfinite(b.lo[k]) || !std::isfinite(b.hi[k]) || !(b.lo[k] <= b.hi[k]) ||
                    fabsf(b.lo[k]) > 16.0f || fabsf(b.hi[k]) > 16.0f)
                    return fail(ctx, PUMP_E_ARG, "obstacle box invalid or outside [-16, 16]");
            }
            bool in = true;
            for (int k = 0; k < 3; ++k) in = in && pr->x_init[k] >= b.lo[k] && pr->x_init[k] <= b.hi[k];
            if (in) return fail(ctx, PUMP_E_ARG, "x_init lies in an obstacle");
        }
    }
    const int N = ctx->N;
    ctx->n_nodes = pr->n + 1;
    ctx->n_obs = pr->n_obs;
    ctx->M = cfg.mc_particles;
    ctx->S_max = cfg.max_steps;
    ctx->dt = (double)cfg.dt;
    ctx->alpha = (double)pr->alpha;
    ctx->eta = cfg.eta > 0.0f ? (double)cfg.eta : eta_rule(ctx->alpha);
    ctx->alpha_min = ctx->alpha / ctx->eta;
    ctx->alpha_max = ctx->eta * ctx->alpha;
    cp_thresholds(ctx->alpha, ctx->eta, N, &ctx->c_cut, &ctx->c_min);
    ctx->h = (double)cfg.lambda * (double)cfg.r_conn;
    // tracking constants (eq. (2) for the double integrator; LQR)
    tracking_constants(ctx->dt, (double)cfg.q_pos, (double)cfg.q_vel, (double)cfg.r_track,
                       (double)pr->sigma, ctx->K, ctx->Acl, ctx->L);
    memset(&ctx->lqg, 0, sizeof(ctx->lqg));
    if (cfg.estimator == 1)
        lqg_constants(ctx->dt, (double)cfg.q_pos, (double)cfg.q_vel, (double)cfg.r_track,
                      (double)pr->sigma, (double)pr->sigma_meas, ctx->lqg.m, ctx->lqg.e);

    HIPCHK(hipEventRecord(ctx->ev[0], ctx->stream));
    // uploads: x_init is node 0, sample i is node i + 1
    // (small uploads go through pinned buffers, so the copies stay asynchronous;
    //  the previous query's copies from them finished at its last wait)
    memcpy(ctx->xinit_h, pr->x_init, 6 * sizeof(float));
    HIPCHK(hipMemcpyAsync(ctx->X, ctx->xinit_h, 6 * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->X + 6, pr->samples, (size_t)pr->n * 6 * sizeof(float), kind, ctx->stream));
    if (pr->n_obs > 0)
        HIPCHK(hipMemcpyAsync(ctx->obs, pr->obstacles, (size_t)pr->n_obs * 6 * sizeof(float), kind, ctx->stream));
    if (pr->mem == PUMP_MEM_HOST) {
        HIPCHK(hipMemcpyAsync(ctx->noise_buf, pr->noise, (size_t)ctx->S_max * 6 * N * sizeof(float),
                              hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(hipMemcpyAsync(ctx->noise_mc_buf, pr->noise_mc,
                              (size_t)ctx->S_max * 6 * ctx->M * sizeof(float), hipMemcpyHostToDevice,
                              ctx->stream));
        ctx->noise = ctx->noise_buf;
        ctx->noise_mc = ctx->noise_mc_buf;
        if (cfg.estimator == 1) {
            HIPCHK(hipMemcpyAsync(ctx->noise_meas_buf, pr->noise_meas,
                                  (size_t)ctx->S_max * 3 * N * sizeof(float),
                                  hipMemcpyHostToDevice, ctx->stream));
            HIPCHK(hipMemcpyAsync(ctx->noise_mc_meas_buf, pr->noise_mc_meas,
                                  (size_t)ctx->S_max * 3 * ctx->M * sizeof(float),
                                  hipMemcpyHostToDevice, ctx->stream));
            ctx->noise_meas = ctx->noise_meas_buf;
            ctx->noise_mc_meas = ctx->noise_mc_meas_buf;
        }
    } else {
        ctx->noise = pr->noise;
        ctx->noise_mc = pr->noise_mc;
        if (cfg.estimator == 1) {
            ctx->noise_meas = pr->noise_meas;
            ctx->noise_mc_meas = pr->noise_mc_meas;
        }
    }
    float gb[6] = {pr->goal.lo[0], pr->goal.lo[1], pr->goal.lo[2],
                   pr->goal.hi[0], pr->goal.hi[1], pr->goal.hi[2]};
    tbeg(ctx, 0);
    if (cfg.estimator == 1)
        launch_deviation_table_lqg(ctx->stream, ctx->noise, ctx->noise_meas, ctx->D, ctx->cloud,
                                   ctx->gcloud, N, ctx->S_max, ctx->lqg, ctx->dev_scratch);
    else
        launch_deviation_table(ctx->stream, ctx->noise, ctx->D, ctx->cloud, ctx->gcloud, N,
                               ctx->S_max, ctx->Acl, ctx->L, ctx->dev_scratch);
    tend(ctx);
    HIPCHK(hipMemsetAsync(ctx->dev_ints, 0, 8 * sizeof(int32_t), ctx->stream));
    launch_mark_valid(ctx->stream, ctx->X, ctx->n_nodes, ctx->obs, ctx->n_obs, gb, ctx->valid, ctx->goal,
                      ctx->dev_ints + 1);
    HIPCHK(hipMemsetAsync(ctx->deg, 0, (size_t)(ctx->n_nodes + 1) * sizeof(int32_t), ctx->stream));
    // pass-1 work lists: the near list in the edge arrays (free until pass 2),
    // the exact queue in two Explore candidate arrays (free until Explore)
    const GraphWork gw{ctx->esrc, ctx->col, ctx->etau, ctx->c_pop, ctx->c_pos, ctx->dev_ints + 2,
                       (int32_t)std::min<int64_t>(cfg.cap_edges, (1ll << 31) - 1),
                       (int32_t)cfg.cap_pairs};
    tbeg(ctx, 1);
    if (ctx->rm)
        launch_rm_query(ctx->stream, ctx->X, ctx->valid, ctx->n_nodes, ctx->obs, ctx->n_obs,
                        (double)cfg.r_steer, (double)cfg.r_conn, ctx->rm->d, ctx->ebits,
                        ctx->words_per_row, ctx->deg, ctx->dev_ints + 1, gw);
    else
        launch_graph_mark(ctx->stream, ctx->X, ctx->valid, ctx->n_nodes, ctx->obs, ctx->n_obs,
                          (double)cfg.r_steer, (double)cfg.r_conn, ctx->ebits, ctx->deg,
                          ctx->words_per_row, gw);
    tend(ctx);
    const int32_t nn = ctx->n_nodes;
    ctx->stage_h[0] = nn;
    HIPCHK(hipMemcpyAsync(ctx->dev_ints, ctx->stage_h, sizeof(int32_t), hipMemcpyHostToDevice,
                          ctx->stream));
    // the scan's total is the edge count, written to row_ptr[n_nodes] and to
    // dev_ints[4], so one read-back brings it with the flags and counters
    scan_exclusive(ctx->stream, ctx->deg, ctx->row_ptr, ctx->dev_ints, nn, ctx->row_ptr + nn,
                   ctx->blk, ctx->dev_ints + 4);
    HIPCHK(hipMemcpyAsync(ctx->stage_h + 4, ctx->dev_ints, 5 * sizeof(int32_t),
                          hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    const int32_t* flags = ctx->stage_h + 4;
    if (flags[1] & 1) return fail(ctx, PUMP_E_ARG, "a sample or obstacle is not finite or lies outside [-16, 16]");
    if (flags[1] & 2) return fail(ctx, PUMP_E_ARG, "x_init lies in an obstacle");
    if (flags[1] & 4) return fail(ctx, PUMP_E_ARG, "the samples differ from the roadmap's");
    if ((long long)flags[2] > cfg.cap_edges)
        return fail(ctx, PUMP_E_CAPACITY, "near connections " + std::to_string(flags[2]) +
                                              " exceed cap_edges");
    if ((long long)flags[3] > cfg.cap_pairs)
        return fail(ctx, PUMP_E_CAPACITY, "exact box tests " + std::to_string(flags[3]) +
                                              " exceed cap_pairs");
    ctx->n_edges = flags[4];
    if ((long long)ctx->n_edges > cfg.cap_edges)
        return fail(ctx, PUMP_E_CAPACITY, "graph edges " + std::to_string(ctx->n_edges) +
                                              " exceed cap_edges");
    tbeg(ctx, 2);
    if (ctx->rm) {
        launch_graph_cols(ctx->stream, ctx->n_nodes, ctx->ebits, ctx->row_ptr, ctx->col, ctx->esrc,
                          ctx->words_per_row);
        launch_rm_fill(ctx->stream, ctx->X, ctx->n_nodes, (double)cfg.r_steer, ctx->row_ptr, ctx->col,
                       ctx->esrc, ctx->rm->d, ctx->etau, ctx->ecost, ctx->n_edges);
    } else {
        launch_graph_fill_near(ctx->stream, ctx->X, ctx->n_nodes, (double)cfg.r_steer, ctx->ebits,
                               ctx->row_ptr, ctx->col, ctx->esrc, ctx->etau, ctx->ecost, ctx->wstart,
                               ctx->words_per_row, ctx->n_edges, gw);
    }
    tend(ctx);
    // no wait here: the setup time is read at the next synchronisation
    HIPCHK(hipEventRecord(ctx->ev[4], ctx->stream));
    HIPCHK(hipGetLastError());
    ctx->setup_time_pending = true;
    ctx->have_setup = true;
    return PUMP_OK;
}

// Root plan and empty staircases.  Without `sync` (pump_plan with the
// single-launch Explore, which reads the loop state on the device) the host
// does not wait for the root's state.
static int explore_begin(pump_ctx* ctx, bool sync) {
    if (!ctx) return PUMP_E_ARG;
    if (!ctx->have_setup) return fail(ctx, PUMP_E_STATE, "pump_setup first");
    ctx->open_cur = ctx->open_b;
    ctx->open_next = ctx->open_a;
    RoundArgs a = round_args(ctx);
    // (also clears the control block and the single launch's barrier words)
    launch_explore_init(ctx->stream, a, ctx->n_nodes, ctx->N, ctx->coop_sync,
                        (int)(64 + 4096 + 4 * (size_t)ctx->coop_blocks));  // writes open_next
    launch_counters_clear(ctx->stream, a);   // (partials a failed round may have left)
    std::swap(ctx->open_cur, ctx->open_next);
    HIPCHK(hipGetLastError());
    ctx->partial_plans = 0;
    ctx->rounds = 0;
    ctx->last_chunks = 1;
    ctx->chunked_rounds = 0;
    ctx->ms_explore = 0.0f;
    ctx->have_explore = true;
    ctx->explore_done = false;
    if (sync) {
        int r = read_ctl(ctx);
        if (r) return r;
        ctx->explore_done = ctx->ctl_h->done != 0;
    }
    return PUMP_OK;
}

int pump_explore_begin(pump_ctx* ctx) { return explore_begin(ctx, true); }

int pump_explore_round(pump_ctx* ctx, int32_t* done) {
    if (!ctx) return PUMP_E_ARG;
    if (!ctx->have_explore) return fail(ctx, PUMP_E_STATE, "pump_explore_begin first");
    if (ctx->explore_done) {
        if (done) *done = 1;
        return PUMP_OK;
    }
    const int32_t n_pairs = ctx->ctl_h->n_pairs;
    const int32_t n_open = ctx->ctl_h->n_open;
    RoundArgs a = round_args(ctx);
    const long long slots = ctx->cfg.cap_pairs;
    if ((long long)n_pairs <= slots) {
        tbeg(ctx, 3);
        launch_expand(ctx->stream, a, ctx->N, n_pairs, 1);
        tend(ctx);
        tbeg(ctx, 18);
        launch_expand(ctx->stream, a, ctx->N, n_pairs, 2);
        tend(ctx);
        tbeg(ctx, 4);
        launch_prune(ctx->stream, a, ctx->N, n_pairs, n_open);
        tend(ctx);
        tbeg(ctx, 5);
        launch_compact(ctx->stream, a, ctx->N, n_pairs, n_open, ctx->blk);
        tend(ctx);
        ctx->last_chunks = 1;
    } else {
        // more pairs than candidate slots: the round in chunks of cap_pairs
        // pairs, in two passes (kernels_explore.hip)
        a.chunked = 1;
        int chunks = 0;
        for (int pass = 0; pass < 2; ++pass) {
            a.quiet = pass;
            if (pass == 1) {
                tbeg(ctx, 5);
                launch_open_compact(ctx->stream, a, n_open, ctx->blk);
                tend(ctx);
            }
            for (long long q0 = 0; q0 < n_pairs; q0 += slots) {
                const int32_t n = (int32_t)std::min<long long>(slots, (long long)n_pairs - q0);
                a.q0 = (int32_t)q0;
                launch_chunk_begin(ctx->stream, a, n);
                tbeg(ctx, 3);
                launch_expand(ctx->stream, a, ctx->N, n, 1);
                tend(ctx);
                tbeg(ctx, 18);
                launch_expand(ctx->stream, a, ctx->N, n, 2);
                tend(ctx);
                if (pass == 0) {
                    tbeg(ctx, 4);
                    launch_stair_update(ctx->stream, a, n);
                    tend(ctx);
                    ++chunks;
                } else {
                    tbeg(ctx, 5);
                    launch_chunk_compact(ctx->stream, a, ctx->N, n, ctx->blk);
                    tend(ctx);
                }
            }
        }
        launch_chunks_finalize(ctx->stream, a);
        a.chunked = 0;
        a.q0 = 0;
        a.quiet = 0;
        ctx->last_chunks = chunks;
        ctx->chunked_rounds += 1;
    }
    launch_counters_reduce(ctx->stream, a);
    long long upper = std::min<long long>((long long)n_open + n_pairs, ctx->cfg.cap_plans);
    tbeg(ctx, 6);
    launch_next_group(ctx->stream, a, (int32_t)upper, ctx->b_deg, ctx->blk);
    tend(ctx);
    HIPCHK(hipGetLastError());
    int r = read_ctl(ctx);
    if (r) return r;
    ctx->partial_plans += n_pairs;
    ctx->last_pairs = n_pairs;
    ctx->rounds += 1;
    std::swap(ctx->open_cur, ctx->open_next);
    if (ctx->ctl_h->err == 3) return fail(ctx, PUMP_E_STATE, "open plans without a finite cost");
    if (ctx->ctl_h->err)
        return fail(ctx, PUMP_E_CAPACITY,
                    "plan store needs " +
                        std::to_string((long long)ctx->ctl_h->n_plans + ctx->ctl_h->n_surv) +
                        " plans, over cap_plans");
    if (ctx->rounds > (1 << 24)) return fail(ctx, PUMP_E_STATE, "Explore did not terminate");
    ctx->explore_done = ctx->ctl_h->done != 0;
    if (done) *done = ctx->explore_done ? 1 : 0;
    return PUMP_OK;
}

// Remaining rounds in one launch (see kernels_coop.hip).
// The single launch in two halves: enqueue, and the bookkeeping once the
// control block has been read back.
static int explore_single_enqueue(pump_ctx* ctx) {
    RoundArgs a = round_args(ctx);
    CoopArgs ca;
    ca.sync.release = ctx->coop_sync;
    ca.sync.fail = reinterpret_cast<int*>(ctx->coop_sync + 1);
    ca.sync.arrive = ctx->coop_sync + 64;
    ca.sync.n_blocks = (unsigned)ctx->coop_blocks;
    ca.sync.patience = ctx->patience;
    ca.xa = reinterpret_cast<unsigned long long*>(ctx->coop_sync + 64 + 4096);
    ca.xb = ca.xa + ctx->coop_blocks;
    ca.b_deg = ctx->b_deg;
    ca.open_cur = ctx->open_cur;
    ca.open_next = ctx->open_next;
    ca.cap_pairs = ctx->cfg.cap_pairs;
    // (the barrier words were cleared by explore_begin)
    tbeg(ctx, 9);
    ctx->ra_h[0] = a;
    ctx->ra_h[0].open_in = ctx->open_cur;
    ctx->ra_h[0].open_out = ctx->open_next;
    ctx->ra_h[1] = a;
    ctx->ra_h[1].open_in = ctx->open_next;
    ctx->ra_h[1].open_out = ctx->open_cur;
    HIPCHK(hipMemcpyAsync(ctx->ra_dev, ctx->ra_h, 2 * sizeof(RoundArgs), hipMemcpyHostToDevice,
                          ctx->stream));
    HIPCHK(launch_explore_coop(ctx->stream, ctx->ra_dev, ca, ctx->N, ctx->coop_blocks));
    tend(ctx);
    return PUMP_OK;
}

static int explore_single_finish(pump_ctx* ctx) {
    const Ctl* c = ctx->ctl_h;
    if (ctx->timing) {
        // the real-time counter runs at 100 MHz
        for (int k = 0; k < 8; ++k) {
            ctx->t_ms[10 + k] += 1e-5 * (double)c->phase_ticks[k];
            ctx->t_n[10 + k] += c->rounds;
        }
    }
    ctx->partial_plans += c->partial;
    ctx->rounds += c->rounds;
    if (c->open_final) std::swap(ctx->open_cur, ctx->open_next);
    if (c->err == 4)
        return fail(ctx, PUMP_E_CAPACITY, "round pairs " + std::to_string(c->n_pairs) +
                                              " exceed cap_pairs");
    if (c->err == 3) return fail(ctx, PUMP_E_STATE, "open plans without a finite cost");
    if (c->err == 5) return fail(ctx, PUMP_E_STATE, "grid barrier timed out");
    if (c->err == 6) return fail(ctx, PUMP_E_STATE, "Explore did not terminate");
    // (2 is the selection's code for an oversized front, set when the
    // selection already ran behind the launch)
    if (c->err && c->err != 2)
        return fail(ctx, PUMP_E_CAPACITY,
                    "plan store needs " + std::to_string((long long)c->n_plans + c->n_surv) +
                        " plans, over cap_plans");
    ctx->explore_done = true;
    return PUMP_OK;
}

// The single launch gave up in a way the per-phase rounds do not: a barrier
// wait ran out of patience (its workgroups were not all resident), or a
// round had more pairs than candidate slots (the per-phase rounds run such a
// round in chunks).
static bool single_needs_fallback(const pump_ctx* ctx, int r) {
    return (r == PUMP_E_STATE && ctx->ctl_h->err == 5) ||
           (r == PUMP_E_CAPACITY && ctx->ctl_h->err == 4);
}

static int explore_single_launch(pump_ctx* ctx) {
    int r = explore_single_enqueue(ctx);
    if (r == PUMP_OK) r = read_ctl(ctx);
    if (r == PUMP_OK) r = explore_single_finish(ctx);
    return r;
}

// Mode 2 picks per query: the single launch holds every phase in one kernel
// at two waves per SIMD and meets at grid barriers, which pays on graphs of
// a few million edges or less (one query then is a short chain of dependent
// steps); on larger graphs the particle simulation dominates and its own
// kernel, at four waves per SIMD with dynamically scheduled workgroups, is
// faster than the single launch despite a host round trip per round
// (indoor 20,000-sample query: 13.3 against 19.3 ms; 4,000-sample query:
// 1.38 against 1.24 ms).  The half-space model's particle work is heavy at
// any size (4,000-sample query: 9.2 ms per phase against 11.3 ms in one
// launch), so with it the per-phase kernels are taken throughout.
constexpr long long kPerPhaseEdges = 4ll << 20;

static int effective_mode(const pump_ctx* ctx) {
    if (ctx->explore_mode != 2) return ctx->explore_mode;
    if (ctx->cfg.cp_model == 1) return 0;
    return (long long)ctx->n_edges >= kPerPhaseEdges ? 0 : 1;
}

int pump_explore_run(pump_ctx* ctx) {
    if (!ctx) return PUMP_E_ARG;
    if (!ctx->have_explore) return fail(ctx, PUMP_E_STATE, "pump_explore_begin first");
    HIPCHK(hipEventRecord(ctx->ev[1], ctx->stream));
    if (effective_mode(ctx) == 1 && !ctx->explore_done) {
        int r = explore_single_launch(ctx);
        if (single_needs_fallback(ctx, r)) {
            // redo Explore with one launch per phase
            ctx->fallbacks += 1;
            r = explore_begin(ctx, true);
            int32_t done = ctx->explore_done ? 1 : 0;
            while (r == PUMP_OK && !done) r = pump_explore_round(ctx, &done);
        }
        if (r) return r;
    } else {
        int32_t done = ctx->explore_done ? 1 : 0;
        while (!done) {
            int r = pump_explore_round(ctx, &done);
            if (r) return r;
        }
    }
    HIPCHK(hipEventRecord(ctx->ev[2], ctx->stream));
    HIPCHK(hipEventSynchronize(ctx->ev[2]));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, ctx->ev[1], ctx->ev[2]));
    ctx->ms_explore = ms;
    return PUMP_OK;
}

int pump_set_explore_mode(pump_ctx* ctx, int32_t mode) {
    if (!ctx || mode < 0 || mode > 2) return PUMP_E_ARG;
    if (mode != 0 && ctx->coop_blocks <= 0)
        return fail(ctx, PUMP_E_ARG, "the single-launch Explore does not fit on this device");
    ctx->explore_mode = mode;
    return PUMP_OK;
}

int pump_set_barrier_patience(pump_ctx* ctx, double ms) {
    if (!ctx || !(ms > 0.0) || !(ms <= 600000.0)) return PUMP_E_ARG;
    ctx->patience = (unsigned long long)(ms * 1e5);   // 100 MHz ticks
    if (ctx->patience < 1) ctx->patience = 1;
    return PUMP_OK;
}

int pump_get_chunked_rounds(pump_ctx* ctx, int64_t* n) {
    if (!ctx || !n) return PUMP_E_ARG;
    *n = ctx->chunked_rounds;
    return PUMP_OK;
}

int pump_get_explore_fallbacks(pump_ctx* ctx, int64_t* n) {
    if (!ctx || !n) return PUMP_E_ARG;
    *n = ctx->fallbacks;
    return PUMP_OK;
}

int pump_get_explore_mode(pump_ctx* ctx, int32_t* mode, int32_t* blocks) {
    if (!ctx) return PUMP_E_ARG;
    if (mode) *mode = ctx->explore_mode;
    if (blocks) *blocks = ctx->coop_blocks;
    return PUMP_OK;
}

static void fill_counters(pump_ctx* ctx, pump_result* o) {
    const Ctl* c = ctx->ctl_h;
    o->partial_plans = ctx->partial_plans;
    o->simulated = c->simulated;
    o->preprune = c->preprune;
    o->inserted = c->inserted;
    o->survivors = c->n_plans - 1;
    o->dropped_steps = c->dropped_steps;
    o->flagged = c->flagged;
    o->sim_waypoints = c->sim_waypoints;
    o->sim_box_tests = c->sim_box_tests;
    o->rounds = ctx->rounds;
    o->final_i = c->i;
    o->n_plans = c->n_plans;
    o->n_edges = ctx->n_edges;
    o->c_cut = ctx->c_cut;
    o->c_min = ctx->c_min;
    o->ms_setup = ctx->ms_setup;
    o->ms_explore = ctx->ms_explore;
    o->ms_select = ctx->ms_select;
}

// PlanSelection.  With explore_pending the single-launch Explore was only
// enqueued: the selection kernels follow it on the stream (reading the plan
// count on the device) and its bookkeeping runs after the one read-back.
static int select_impl(pump_ctx* ctx, pump_result* out, bool explore_pending) {
    pump_result res;
    memset(&res, 0, sizeof(res));
    res.best = -1;
    res.best_plan = -1;
    ctx->last_best = -1;
    ctx->last_smoothed = false;
    HIPCHK(hipEventRecord(ctx->ev[2], ctx->stream));
    SelectArgs a = select_args(ctx);
    if (explore_pending) a.n_plans = -1;
    // the whole of Alg. 5 on the device (front, waypoints, Monte Carlo,
    // bisection), then one read-back of the control block
    tbeg(ctx, 7);
    launch_select_front(ctx->stream, a, ctx->o_keep, ctx->blk);
    tend(ctx);
    launch_waypoints(ctx->stream, a, -1);
    tbeg(ctx, 8);
    launch_mc(ctx->stream, a, -1);
    tend(ctx);
    launch_select_final(ctx->stream, a, ctx->alpha);
    HIPCHK(hipGetLastError());
    int r = read_ctl(ctx);
    if (r) return r;
    if (explore_pending) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, ctx->ev[1], ctx->ev[2]) == hipSuccess) ctx->ms_explore = ms;
        r = explore_single_finish(ctx);
        if (r) return r;
    }
    const Ctl* c = ctx->ctl_h;
    if (c->err == 2) return fail(ctx, PUMP_E_CAPACITY, "Pareto front exceeds 256 plans");
    if (c->n_goal > kMaxGoal) return fail(ctx, PUMP_E_CAPACITY, "P_goal exceeds 65536 plans");
    if (c->sel_bad_wp) return fail(ctx, PUMP_E_STATE, "front plan longer than max_steps");
    res.n_goal_plans = c->n_goal;
    res.n_front = c->n_front;
    res.status = c->sel_status;
    if (res.status == PUMP_OK) {
        const int m = c->sel_best + 1;   // 1-based, as in Alg. 5
        res.best = m - 1;
        res.best_plan = c->sel_plan;
        res.best_mc_count = c->sel_mc;
        res.best_cp_mc = (double)c->sel_mc / (double)ctx->M;
        res.best_len = c->sel_len;
        res.best_cost = c->sel_cost;
        res.best_pop = c->sel_pop;
        ctx->last_best = m - 1;
        res.smooth_beta = 0.0;
        res.smooth_cost = res.best_cost;
        res.smooth_mc_count = res.best_mc_count;
        res.smooth_steps = c->sel_steps;
        ctx->last_steps = c->sel_steps;
        if (ctx->cfg.smooth) {
            tbeg(ctx, 17);
            launch_smooth(ctx->stream, a, ctx->sm, m - 1, ctx->p_cost + c->sel_plan, ctx->alpha,
                          c->sel_mc, c->sel_steps);
            tend(ctx);
            HIPCHK(hipGetLastError());
            SmoothState st;
            HIPCHK(hipMemcpyAsync(&st, ctx->sm.st, sizeof(st), hipMemcpyDeviceToHost, ctx->stream));
            HIPCHK(hipStreamSynchronize(ctx->stream));
            res.smooth_beta = st.beta;
            res.smooth_cost = st.cost;
            res.smooth_mc_count = st.count;
            res.smooth_steps = st.steps;
            ctx->last_steps = st.steps;
            ctx->last_smoothed = true;
        }
    }
    HIPCHK(hipEventRecord(ctx->ev[3], ctx->stream));
    HIPCHK(hipEventSynchronize(ctx->ev[3]));
    HIPCHK(hipEventElapsedTime(&ctx->ms_select, ctx->ev[2], ctx->ev[3]));
    fill_counters(ctx, &res);
    res.n_valid_nodes = ctx->ctl_h->n_valid;
    if (out) *out = res;
    return res.status;
}

int pump_select(pump_ctx* ctx, pump_result* out) {
    if (!ctx) return PUMP_E_ARG;
    if (!ctx->have_explore || !ctx->explore_done) return fail(ctx, PUMP_E_STATE, "explore not finished");
    return select_impl(ctx, out, false);
}

int pump_plan(pump_ctx* ctx, const pump_problem* pr, pump_result* out) {
    if (!ctx || !pr) return PUMP_E_ARG;
    hipEvent_t t0 = ctx->ev[5], t1 = ctx->ev[6];
    HIPCHK(hipEventRecord(t0, ctx->stream));
    int r = pump_setup(ctx, pr);
    // with the single-launch Explore the host enqueues Explore and the
    // selection back to back and waits once, at the end
    const bool one_wait = r == PUMP_OK && effective_mode(ctx) == 1;
    if (r == PUMP_OK) r = explore_begin(ctx, !one_wait);
    pump_result res;
    memset(&res, 0, sizeof(res));
    if (one_wait) {
        if (r == PUMP_OK) {
            HIPCHK(hipEventRecord(ctx->ev[1], ctx->stream));
            r = explore_single_enqueue(ctx);
        }
        if (r == PUMP_OK) r = select_impl(ctx, &res, true);
        if (single_needs_fallback(ctx, r)) {
            // Explore again from the root with one launch per phase, then
            // select
            ctx->fallbacks += 1;
            memset(&res, 0, sizeof(res));
            r = explore_begin(ctx, true);
            const int mode = ctx->explore_mode;
            ctx->explore_mode = 0;
            if (r == PUMP_OK) r = pump_explore_run(ctx);
            ctx->explore_mode = mode;
            if (r == PUMP_OK) r = pump_select(ctx, &res);
        }
    } else {
        if (r == PUMP_OK) r = pump_explore_run(ctx);
        if (r == PUMP_OK) r = pump_select(ctx, &res);
    }
    HIPCHK(hipEventRecord(t1, ctx->stream));
    HIPCHK(hipEventSynchronize(t1));
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, t0, t1);
    res.ms_total = ms;
    if (out) *out = res;
    return r;
}

int pump_set_roadmap(pump_ctx* ctx, const pump_roadmap* rm) {
    if (!ctx) return PUMP_E_ARG;
    if (rm && (rm->r_steer != ctx->cfg.r_steer || rm->r_conn != ctx->cfg.r_conn))
        return fail(ctx, PUMP_E_ARG, "roadmap radii differ from the context's");
    if (rm && rm->n + 1 > ctx->cfg.max_nodes)
        return fail(ctx, PUMP_E_ARG, "roadmap holds more samples than max_nodes - 1");
    ctx->rm = rm;
    ctx->have_setup = ctx->have_explore = ctx->explore_done = false;
    return PUMP_OK;
}

int pump_sample_halton(int32_t n, int32_t n_goal, const float* lo, const float* hi,
                       const pump_aabb* goal, int64_t start, float* out, void* hip_stream) {
    if (n < 1 || n_goal < 0 || n_goal > n || !lo || !hi || !out || (n_goal > 0 && !goal))
        return PUMP_E_ARG;
    if (start < 0 || start + (int64_t)n >= (1ll << 31)) return PUMP_E_ARG;
    for (int d = 0; d < 6; ++d)
        if (!std::isfinite(lo[d]) || !std::isfinite(hi[d]) || !(lo[d] <= hi[d])) return PUMP_E_ARG;
    float glo[6], ghi[6];
    for (int d = 0; d < 6; ++d) {
        glo[d] = d < 3 && goal ? goal->lo[d] : lo[d];
        ghi[d] = d < 3 && goal ? goal->hi[d] : hi[d];
    }
    if (goal)
        for (int d = 0; d < 3; ++d)
            if (!std::isfinite(glo[d]) || !std::isfinite(ghi[d]) || !(glo[d] <= ghi[d])) return PUMP_E_ARG;
    hipStream_t s = (hipStream_t)hip_stream;
    const int32_t n_box = n - n_goal;
    if (launch_halton(s, start, n_box, lo, hi, out) != hipSuccess) return PUMP_E_HIP;
    if (launch_halton(s, start + n_box, n_goal, glo, ghi, out + (size_t)n_box * 6) != hipSuccess)
        return PUMP_E_HIP;
    return hipStreamSynchronize(s) == hipSuccess ? PUMP_OK : PUMP_E_HIP;
}

int pump_get_smooth_path(pump_ctx* ctx, double* wp, int32_t cap_steps, int32_t* steps) {
    if (!ctx || !wp) return PUMP_E_ARG;
    if (ctx->last_best < 0) return fail(ctx, PUMP_E_STATE, "no certified plan from the last selection");
    if (steps) *steps = ctx->last_steps;
    if (cap_steps < ctx->last_steps) return fail(ctx, PUMP_E_CAPACITY, "cap_steps below the trajectory's steps");
    const double* src = ctx->last_smoothed ? ctx->sm.out_wp
                                           : ctx->wp + (size_t)ctx->last_best * (ctx->S_max + 1) * 3;
    HIPCHK(hipMemcpy(wp, src, (size_t)(ctx->last_steps + 1) * 3 * sizeof(double), hipMemcpyDeviceToHost));
    return PUMP_OK;
}

int pump_set_timing(pump_ctx* ctx, int32_t on) {
    if (!ctx) return PUMP_E_ARG;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    tresolve(ctx);
    ctx->timing = on != 0;
    for (int k = 0; k < PUMP_TIMING_KINDS; ++k) { ctx->t_ms[k] = 0.0; ctx->t_n[k] = 0; }
    return PUMP_OK;
}

int pump_get_timing(pump_ctx* ctx, double* ms, int64_t* launches, int32_t n) {
    if (!ctx || n < 0) return PUMP_E_ARG;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    tresolve(ctx);
    for (int k = 0; k < n && k < PUMP_TIMING_KINDS; ++k) {
        if (ms) ms[k] = ctx->t_ms[k];
        if (launches) launches[k] = ctx->t_n[k];
    }
    return PUMP_OK;
}

int pump_get_deviation(pump_ctx* ctx, float* out, int64_t cap) {
    if (!ctx || !out) return PUMP_E_ARG;
    if (!ctx->have_setup) return fail(ctx, PUMP_E_STATE, "pump_setup first");
    size_t n = (size_t)(ctx->S_max + 1) * 3 * ctx->N;
    if ((int64_t)n > cap) return fail(ctx, PUMP_E_ARG, "output too small");
    HIPCHK(hipMemcpy(out, ctx->D, n * sizeof(float), hipMemcpyDeviceToHost));
    return PUMP_OK;
}

int pump_get_graph(pump_ctx* ctx, int32_t* row_ptr, int32_t* col, double* tau, double* cost,
                   uint8_t* valid, int64_t cap_edges, int64_t* n_edges) {
    if (!ctx) return PUMP_E_ARG;
    if (!ctx->have_setup) return fail(ctx, PUMP_E_STATE, "pump_setup first");
    if (n_edges) *n_edges = ctx->n_edges;
    if (row_ptr) HIPCHK(hipMemcpy(row_ptr, ctx->row_ptr, (ctx->n_nodes + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (valid) HIPCHK(hipMemcpy(valid, ctx->valid, ctx->n_nodes, hipMemcpyDeviceToHost));
    if ((col || tau || cost) && cap_edges < ctx->n_edges) return fail(ctx, PUMP_E_ARG, "output too small");
    if (col) HIPCHK(hipMemcpy(col, ctx->col, (size_t)ctx->n_edges * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (tau) HIPCHK(hipMemcpy(tau, ctx->etau, (size_t)ctx->n_edges * sizeof(double), hipMemcpyDeviceToHost));
    if (cost) HIPCHK(hipMemcpy(cost, ctx->ecost, (size_t)ctx->n_edges * sizeof(double), hipMemcpyDeviceToHost));
    return PUMP_OK;
}

int pump_get_plans(pump_ctx* ctx, int32_t* head, int32_t* parent, int32_t* edge, double* cost,
                   int32_t* step, int32_t* pop, int32_t* round, uint8_t* state, uint32_t* mask,
                   int64_t cap, int64_t* n_plans) {
    if (!ctx) return PUMP_E_ARG;
    if (!ctx->have_explore) return fail(ctx, PUMP_E_STATE, "pump_explore_begin first");
    const size_t n = (size_t)ctx->ctl_h->n_plans;
    if (n_plans) *n_plans = (int64_t)n;
    if ((head || parent || edge || cost || step || pop || round || state || mask) && (int64_t)n > cap)
        return fail(ctx, PUMP_E_ARG, "output too small");
    if (head) HIPCHK(hipMemcpy(head, ctx->p_head, n * 4, hipMemcpyDeviceToHost));
    if (parent) HIPCHK(hipMemcpy(parent, ctx->p_parent, n * 4, hipMemcpyDeviceToHost));
    if (edge) HIPCHK(hipMemcpy(edge, ctx->p_edge, n * 4, hipMemcpyDeviceToHost));
    if (cost) HIPCHK(hipMemcpy(cost, ctx->p_cost, n * 8, hipMemcpyDeviceToHost));
    if (step) HIPCHK(hipMemcpy(step, ctx->p_step, n * 4, hipMemcpyDeviceToHost));
    if (pop) HIPCHK(hipMemcpy(pop, ctx->p_pop, n * 4, hipMemcpyDeviceToHost));
    if (round) HIPCHK(hipMemcpy(round, ctx->p_round, n * 4, hipMemcpyDeviceToHost));
    if (state) HIPCHK(hipMemcpy(state, ctx->p_state, n, hipMemcpyDeviceToHost));
    if (mask) HIPCHK(hipMemcpy(mask, ctx->p_mask, n * ctx->W * 4, hipMemcpyDeviceToHost));
    return PUMP_OK;
}

int pump_get_candidates(pump_ctx* ctx, uint8_t* flag, int32_t* pop, int32_t* parent, int32_t* head,
                        double* cost, uint32_t* mask, int64_t cap, int64_t* n_pairs) {
    if (!ctx) return PUMP_E_ARG;
    if (!ctx->have_explore) return fail(ctx, PUMP_E_STATE, "pump_explore_begin first");
    // the pair count of the round just run is the previous round's n_pairs;
    // kept as the number the caller saw before the round
    if (ctx->last_chunks > 1)
        return fail(ctx, PUMP_E_STATE, "the last round ran in " + std::to_string(ctx->last_chunks) +
                                           " chunks; its candidates are not kept");
    const int32_t n = ctx->last_pairs;
    if (n_pairs) *n_pairs = n;
    if ((int64_t)n > cap && (flag || pop || parent || head || cost || mask))
        return fail(ctx, PUMP_E_ARG, "output too small");
    if (flag) HIPCHK(hipMemcpy(flag, ctx->c_flag, (size_t)n, hipMemcpyDeviceToHost));
    if (pop) HIPCHK(hipMemcpy(pop, ctx->c_pop, (size_t)n * 4, hipMemcpyDeviceToHost));
    if (parent) HIPCHK(hipMemcpy(parent, ctx->c_parent, (size_t)n * 4, hipMemcpyDeviceToHost));
    if (head) HIPCHK(hipMemcpy(head, ctx->c_head, (size_t)n * 4, hipMemcpyDeviceToHost));
    if (cost) HIPCHK(hipMemcpy(cost, ctx->c_cost, (size_t)n * 8, hipMemcpyDeviceToHost));
    if (mask) HIPCHK(hipMemcpy(mask, ctx->c_mask, (size_t)n * ctx->W * 4, hipMemcpyDeviceToHost));
    return PUMP_OK;
}

int pump_get_front(pump_ctx* ctx, int32_t* plan_ids, int32_t* mc_counts, int32_t cap, int32_t* n_front) {
    if (!ctx) return PUMP_E_ARG;
    const int nf = ctx->ctl_h->n_front;
    if (n_front) *n_front = nf;
    if ((plan_ids || mc_counts) && nf > cap) return fail(ctx, PUMP_E_ARG, "output too small");
    if (plan_ids && nf) HIPCHK(hipMemcpy(plan_ids, ctx->front_ids, nf * 4, hipMemcpyDeviceToHost));
    if (mc_counts && nf) HIPCHK(hipMemcpy(mc_counts, ctx->mc_counts, nf * 4, hipMemcpyDeviceToHost));
    return PUMP_OK;
}

int pump_get_path(pump_ctx* ctx, int32_t plan, int32_t* nodes, int32_t cap, int32_t* len) {
    if (!ctx || !nodes || !len) return PUMP_E_ARG;
    if (!ctx->have_explore) return fail(ctx, PUMP_E_STATE, "pump_explore_begin first");
    const int n = ctx->ctl_h->n_plans;
    if (plan < 0 || plan >= n) return fail(ctx, PUMP_E_ARG, "plan id out of range");
    std::vector<int32_t> par(n), head(n);
    HIPCHK(hipMemcpy(par.data(), ctx->p_parent, (size_t)n * 4, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(head.data(), ctx->p_head, (size_t)n * 4, hipMemcpyDeviceToHost));
    std::vector<int32_t> rev;
    for (int q = plan; q >= 0; q = par[q]) {
        rev.push_back(head[q]);
        if ((int)rev.size() > n) return fail(ctx, PUMP_E_STATE, "parent cycle");
    }
    if ((int)rev.size() > cap) return fail(ctx, PUMP_E_ARG, "output too small");
    *len = (int32_t)rev.size();
    for (size_t i = 0; i < rev.size(); ++i) nodes[i] = rev[rev.size() - 1 - i];
    return PUMP_OK;
}

int pump_mc_path(pump_ctx* ctx, const int32_t* nodes, int32_t len, int32_t* count) {
    if (!ctx || !nodes || !count) return PUMP_E_ARG;
    if (!ctx->have_setup) return fail(ctx, PUMP_E_STATE, "pump_setup first");
    if (len < 1 || len > ctx->S_max + 1 || nodes[0] != 0) return fail(ctx, PUMP_E_ARG, "bad path");
    for (int i = 0; i < len; ++i)
        if (nodes[i] < 0 || nodes[i] >= ctx->n_nodes) return fail(ctx, PUMP_E_ARG, "node out of range");
    HIPCHK(hipMemcpyAsync(ctx->paths, nodes, (size_t)len * 4, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->path_len, &len, 4, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemsetAsync(ctx->mc_counts, 0, 4, ctx->stream));
    SelectArgs a = select_args(ctx);
    launch_waypoints(ctx->stream, a, 1);
    launch_mc(ctx->stream, a, 1);
    HIPCHK(hipGetLastError());
    int32_t wl = 0;
    HIPCHK(hipMemcpyAsync(&wl, ctx->wp_len, 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(count, ctx->mc_counts, 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (wl < 0) return fail(ctx, PUMP_E_ARG, "path longer than max_steps");
    return PUMP_OK;
}

}  // extern "C"
