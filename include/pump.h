/*
 * pump.h -- C ABI of libpump, an MI355X (gfx950) implementation of the hot
 * path of PUMP (Parallel Uncertainty-aware Multiobjective Planning; Ichter,
 * Schmerling, Agha-mohammadi, Pavone, arXiv 1607.06886).
 *
 * The planning problem is the stochastic kinodynamic motion planning problem
 * of Sec. II, eq. (3): find the lowest-cost nominal trajectory from x_init to a
 * goal region whose collision probability (CP) under an LQ tracking controller
 * (full-state LQR, or LQG with a Kalman estimate) and Gaussian process (and
 * measurement) noise is at most alpha.  The robot is the 6-D double
 * integrator of Sec. V-A; obstacles are unions of axis-aligned boxes (Sec. V-C).
 * pump_plan() runs Alg. 2: BuildGraph (Alg. 3), Explore (Alg. 4), PlanSelection
 * (Alg. 5).
 *
 * Conventions for every call:
 *   - A state is 6 floats (px, py, pz, vx, vy, vz).  Positions must lie within
 *     [-16, 16] on every axis.
 *   - Every function returns a status code (PUMP_OK, a positive algorithmic
 *     outcome, or a negative error) unless stated otherwise; on a negative
 *     code pump_last_error() describes the failure.
 *   - The caller owns every buffer it passes.  The library never keeps a
 *     caller pointer after a call returns.  Pointers flagged PUMP_MEM_DEVICE
 *     are read on the context's HIP stream; calls return only after their
 *     device work has finished.
 *   - The context owns its device workspace (allocated once in pump_create,
 *     sized by the pump_config capacities) and every result it reports; those
 *     stay valid until the next call on the same context.  A context is used
 *     by one host thread at a time.
 *   - Same inputs, configuration and build give bit-identical outputs.
 */
#ifndef PUMP_H
#define PUMP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes.  Positive values are outcomes of the algorithm, not errors. */
#define PUMP_OK            0
#define PUMP_INFEASIBLE    1   /* Alg. 5: no plan of the front is certified (MC > alpha) */
#define PUMP_NO_GOAL_PLAN  2   /* Explore ended with no plan reaching the goal region */
#define PUMP_E_ARG        -1   /* invalid argument (see pump_last_error) */
#define PUMP_E_CAPACITY   -2   /* a workspace capacity was exceeded; pump_last_error names it */
#define PUMP_E_HIP        -3   /* a HIP runtime call failed */
#define PUMP_E_STATE      -4   /* call out of order (e.g. a round before setup) */

#define PUMP_MEM_HOST      0
#define PUMP_MEM_DEVICE    1

/* A closed axis-aligned box {p : lo <= p <= hi} (Sec. V-C: obstacles are
 * unions of such boxes). */
typedef struct pump_aabb {
    float lo[3];
    float hi[3];
} pump_aabb;

/* Planner configuration.  Fill with pump_config_default() and override.
 * The paper fixes N = 128, eta and lambda (Sec. V-A); the other model
 * parameters are left open by the paper and default to the values below. */
typedef struct pump_config {
    int32_t n_particles;   /* N exploration particles: 32, 64, 128 or 256          */
    int32_t max_nodes;     /* capacity: samples + 1 (x_init is node 0)              */
    int32_t max_obstacles; /* capacity: obstacle boxes, <= 256                      */
    int32_t max_steps;     /* S_max: tracking steps a plan may span; also the step
                              extent of both noise arrays                          */
    int32_t mc_particles;  /* M certification particles (Alg. 5 MC(p))             */
    int32_t preprune;      /* 1: skip simulating a pair whose parent cp_hat already
                              makes it dominated (exact; results unchanged)       */
    float dt;              /* tracking step of eq. (2), default 0.05                */
    float q_pos, q_vel;    /* LQR state weights per axis, default 100, 10           */
    float r_track;         /* LQR input weight, default 1                           */
    float r_steer;         /* control-effort weight r_u in the cost c, default 0.1  */
    float r_conn;          /* connection radius r_n of Near (Alg. 3), default 1.0   */
    float eta;             /* CP approximation factor of Alg. 2; 0 = 2 above 1%,
                              10 at 0.1%, log-linear between                      */
    float lambda;          /* group cost factor of Alg. 4, default 0.5             */
    int32_t cp_model;      /* exploration collision model of a particle at a
                              waypoint: 0 (default) position inside a closed box;
                              1 Half-Space Monte Carlo (Sec. III-B): deviation
                              beyond a plane of the waypoint's local convex
                              region, planes made perpendicular to the nominal
                              velocity (eq. (7)).  Certification (MC(p)) is the
                              same for both.                                   */
    int32_t estimator;     /* tracking controller of eq. (2): 0 (default) LQR on
                              the true deviation (no measurement noise); 1 LQG:
                              the LQR gain acts on a steady-state Kalman
                              estimate built from a position measurement
                              dy = C dx + w, C = [I 0], W = sigma_meas^2 / dt
                              per axis.  Exploration particles and MC(p) both
                              follow the chosen controller.                   */
    int32_t smooth;        /* Alg. 5's final Smooth(p*, alpha): 0 (default) the
                              identity; 1 blend p* with the optimal connection
                              x_init -> p*.head (weight beta, normalised time,
                              both boundary states kept), beta = 1 tried first,
                              then 9 bisection steps re-certified by MC over
                              the blend's tracking grid; the cheaper certified
                              blend replaces p* (pump_result.smooth_*,
                              pump_get_smooth_path).                           */
    int32_t reserved_;     /* zero                                               */
    int64_t cap_edges;     /* capacity: graph edges                                 */
    int64_t cap_plans;     /* capacity: plan records over a whole query             */
    int64_t cap_pairs;     /* capacity: candidate slots ((plan, neighbour) pairs
                              held at once) and BuildGraph's exact queue.  A
                              round of Explore with more pairs runs in chunks
                              of cap_pairs pairs (pump_explore_round), with the
                              same result; the batched engine fails such a
                              query with PUMP_E_CAPACITY.                      */
} pump_config;

/* One planning query: Alg. 2's inputs plus the noise the particle models
 * consume.  `samples`, `obstacles`, `noise` and `noise_mc` live in host or
 * device memory as `mem` says.
 *   samples   [n][6]          SampleFree(n) states (Alg. 3); a sample whose
 *                             position lies in an obstacle is dropped
 *   obstacles [n_obs]         closed boxes
 *   noise     [S_max][6][N]   standard normals for the exploration particles;
 *                             component 2a and 2a+1 drive axis a at step s
 *   noise_mc  [S_max][6][M]   standard normals for certification
 * alpha in (0, 1) is the CP bound of eq. (3); sigma is the process-noise
 * intensity (V_c = sigma^2 I in eq. (1)).
 * With cfg.estimator = 1 (LQG) three more fields are read (ignored otherwise):
 *   sigma_meas > 0            measurement-noise intensity (W_c = sigma_meas^2 I
 *                             in eq. (1))
 *   noise_meas    [S_max][3][N]  standard normals of the exploration
 *                             particles' measurements; row s, component a is
 *                             the axis-a measurement taken after step s
 *   noise_mc_meas [S_max][3][M]  the same for certification
 * in the memory space `mem` names, like the other arrays. */
typedef struct pump_problem {
    const float* samples;
    int32_t n;
    const pump_aabb* obstacles;
    int32_t n_obs;
    float x_init[6];
    pump_aabb goal;          /* X_goal: closed position box, velocity free */
    float alpha;
    float sigma;
    const float* noise;
    const float* noise_mc;
    int32_t mem;             /* PUMP_MEM_HOST or PUMP_MEM_DEVICE */
    float sigma_meas;
    const float* noise_meas;
    const float* noise_mc_meas;
} pump_problem;

/* Outcome of a query (Alg. 2 output plus counters). */
typedef struct pump_result {
    int32_t status;          /* PUMP_OK, PUMP_INFEASIBLE or PUMP_NO_GOAL_PLAN */
    int32_t n_goal_plans;    /* |P_goal| (Alg. 4 return)                      */
    int32_t n_front;         /* Pareto front of P_goal (cost, cp_hat)         */
    int32_t best;            /* index of p* in the sorted front, -1 if none  */
    int32_t best_plan;       /* plan id of p* (see pump_get_plans), -1       */
    int32_t best_pop;        /* invalid exploration particles of p*           */
    int32_t best_mc_count;   /* certification particles of p* that collide    */
    int32_t best_len;        /* nodes on p* including x_init                  */
    double best_cost;        /* c of p*                                        */
    double best_cp_mc;       /* MC(p*) = best_mc_count / M                     */
    int64_t partial_plans;   /* (plan, neighbour) pairs formed in Explore     */
    int64_t simulated;       /* pairs whose particles were propagated         */
    int64_t preprune;        /* pairs resolved as dominated before simulation */
    int64_t inserted;        /* pairs passing the CP cutoff and not pre-pruned*/
    int64_t survivors;       /* plans added to the plan store                 */
    int64_t dropped_steps;   /* pairs dropped for exceeding S_max             */
    int64_t flagged;         /* particle decisions within 1e-5 of a box face,
                                over the pairs that pass the CP cutoff         */
    int32_t rounds;          /* Explore iterations with a non-empty group     */
    int32_t final_i;         /* group index i at exit                          */
    int32_t n_plans;         /* plan records created                          */
    int32_t n_edges;         /* graph edges                                    */
    int32_t n_valid_nodes;   /* nodes not inside an obstacle                   */
    int32_t c_cut;           /* keep a pair iff pop < c_cut (= ceil(alpha_max N)) */
    int32_t c_min;           /* goal stop iff pop < c_min (= ceil(alpha_min N))   */
    int32_t pad;
    float ms_setup;          /* deviation table + graph build (Alg. 3)        */
    float ms_explore;        /* Alg. 4                                          */
    float ms_select;         /* Alg. 5                                          */
    float ms_total;          /* whole pump_plan call                            */
    int64_t sim_waypoints;   /* (pair, waypoint) particle tests: each covers the N
                                particles at a waypoint whose cloud meets a box;
                                a pair stops at the waypoint where its count
                                reaches c_cut                                  */
    int64_t sim_box_tests;   /* (pair, waypoint, box) tests, each over N particles */
    /* Smooth(p*, alpha) with cfg.smooth = 1 (else beta 0 and p*'s figures):  */
    double smooth_beta;      /* blend weight returned (0: p* kept)            */
    double smooth_cost;      /* cost of the returned trajectory               */
    int32_t smooth_mc_count; /* its certification count (of M)                */
    int32_t smooth_steps;    /* its tracking steps                            */
} pump_result;

typedef struct pump_ctx pump_ctx;

/* Defaults: N = 128, dt = 0.05, q = (100, 10), r_track = 1, r_steer = 0.1,
 * r_conn = 1, eta = 0 (rule), lambda = 0.5, M = 10000, S_max = 512,
 * preprune = 1, capacities for 4001 nodes / 64 obstacles. */
void pump_config_default(pump_config* cfg);

/* Create a context on the current HIP device.  `hip_stream` is a
 * hipStream_t to run on, or NULL for a stream the context creates.  All
 * device memory is allocated here.  Errors: PUMP_E_ARG for an unsupported
 * configuration, PUMP_E_HIP if allocation fails (*out is then NULL). */
int pump_create(const pump_config* cfg, void* hip_stream, pump_ctx** out);

/* Free the context and its device memory.  NULL is accepted. */
int pump_destroy(pump_ctx* ctx);

/* Alg. 2 end to end: setup (deviation table, BuildGraph), Explore,
 * PlanSelection.  Fills *out (which may be NULL).  Returns the status. */
int pump_plan(pump_ctx* ctx, const pump_problem* prob, pump_result* out);

/* Step hooks (the same work pump_plan does, one stage at a time). */
/* Upload the problem, compute the tracking constants, the particle deviation
 * table and BuildGraph (Alg. 3). */
int pump_setup(pump_ctx* ctx, const pump_problem* prob);
/* Alg. 4 initialisation: P_open = B = {root}, i = 0. */
int pump_explore_begin(pump_ctx* ctx);
/* One iteration of Alg. 4's while loop; *done = 1 once the loop test fails
 * (no open plan, or a goal plan of the group has cp_hat < alpha_min).
 * A round whose pairs (sum of the group's out-degrees) exceed cap_pairs runs
 * in chunks of cap_pairs pairs and two passes: the first expands each chunk
 * and enters its candidates into the dominance staircases, the second
 * expands each chunk again and keeps the candidates the final staircases do
 * not dominate.  RemoveDominated depends only on the final staircases, so
 * the plan store is the one the round in one piece makes (same plan ids);
 * the counters of pump_result count the first pass.
 * pump_get_chunked_rounds reports how many rounds of the current Explore ran
 * in chunks. */
int pump_explore_round(pump_ctx* ctx, int32_t* done);
int pump_get_chunked_rounds(pump_ctx* ctx, int64_t* n);
/* Rounds until done. */
int pump_explore_run(pump_ctx* ctx);
/* Alg. 5 on the explored plans; fills *out (status and p*). */
int pump_select(pump_ctx* ctx, pump_result* out);

/* Readers (host output buffers; sizes in elements). */
/* Particle deviation table D[s][a][j] (position part), (S_max+1)*3*N floats. */
int pump_get_deviation(pump_ctx* ctx, float* out, int64_t cap);
/* Graph: row_ptr [n+2] (node v's neighbours are col[row_ptr[v]..row_ptr[v+1]),
 * sorted), col/tau/cost [n_edges]; valid [n+1] (node not in an obstacle).
 * Any pointer may be NULL. */
int pump_get_graph(pump_ctx* ctx, int32_t* row_ptr, int32_t* col, double* tau,
                   double* cost, uint8_t* valid, int64_t cap_edges, int64_t* n_edges);
/* Plan store: for plans 0..n-1 their head node, parent plan (-1 for the root),
 * graph edge (-1 for the root), cost, tracking steps, pop (invalid particles),
 * group index of the round that created them, state (0 open, 1 closed,
 * 2 removed by RemoveDominated) and particle bits (N/32 words per plan, bit j
 * of word j/32 = particle j invalid).  Any pointer may be NULL. */
int pump_get_plans(pump_ctx* ctx, int32_t* head, int32_t* parent, int32_t* edge,
                   double* cost, int32_t* step, int32_t* pop, int32_t* round,
                   uint8_t* state, uint32_t* mask, int64_t cap, int64_t* n_plans);
/* Candidates of the last round, one per (plan, neighbour) pair in pair order:
 * flag (0 dropped, 1 kept and not dominated, 2 kept but dominated),
 * pop (-1 pre-pruned before simulation, -2 over S_max; a cut pair's pop is
 * some value >= c_cut, as its simulation stops once the count reaches c_cut),
 * and for kept ones parent plan, head, cost and particle bits.  Any pointer
 * may be NULL.
 * PUMP_E_STATE if that round ran in chunks (its candidates are not kept). */
int pump_get_candidates(pump_ctx* ctx, uint8_t* flag, int32_t* pop, int32_t* parent,
                        int32_t* head, double* cost, uint32_t* mask, int64_t cap,
                        int64_t* n_pairs);
/* The sorted Pareto front of P_goal used by Alg. 5: plan ids and the MC
 * certification counts (out of M). */
int pump_get_front(pump_ctx* ctx, int32_t* plan_ids, int32_t* mc_counts, int32_t cap,
                   int32_t* n_front);
/* Node sequence (x_init first) of a plan. */
int pump_get_path(pump_ctx* ctx, int32_t plan, int32_t* nodes, int32_t cap, int32_t* len);
/* MC(p) (Sec. IV) for an arbitrary node sequence (nodes[0] must be 0):
 * number of the M certification particles whose path meets an obstacle. */
int pump_mc_path(pump_ctx* ctx, const int32_t* nodes, int32_t len, int32_t* count);
/* Nominal tracking waypoints of the trajectory pump_select returned last:
 * the Smooth(p*, alpha) blend (cfg.smooth = 1, smooth_beta > 0) or p* itself;
 * (*steps + 1) positions [*steps + 1][3] (FP64, host memory) go to `wp`,
 * which holds cap_steps + 1 of them.  PUMP_E_STATE if the last selection
 * certified no plan, PUMP_E_CAPACITY if cap_steps < *steps. */
int pump_get_smooth_path(pump_ctx* ctx, double* wp, int32_t cap_steps, int32_t* steps);

/* Cached roadmap (Alg. 3's obstacle-independent part; the paper caches
 * neighbours and edge controls offline, Sec. V-A).  pump_roadmap_create runs
 * Near and the optimal connections (tau*, c*) over every ordered pair of the
 * n samples, with no obstacles, and keeps each connection with its nominal
 * position range.  A context given the roadmap (pump_set_roadmap) builds a
 * query's graph by testing only the cached connections against the query's
 * obstacles, plus the connections to and from its x_init; the graph equals
 * the one pump_setup builds from scratch.  `samples` [n][6] is host or device
 * memory as `mem` says; cfg supplies r_steer, r_conn, max_nodes (n + 1 at
 * most) and cap_edges.  The roadmap owns its device memory; it is used on
 * the context's stream and must outlive its use.  Errors: PUMP_E_ARG (sizes,
 * non-finite samples or outside [-16, 16]), PUMP_E_CAPACITY (more than
 * cap_edges connections), PUMP_E_HIP. */
typedef struct pump_roadmap pump_roadmap;
int pump_roadmap_create(const pump_config* cfg, const float* samples, int32_t n, int32_t mem,
                        void* hip_stream, pump_roadmap** out);
int pump_roadmap_destroy(pump_roadmap* rm);
/* Sample count, cached connections and build time (ms) of a roadmap. */
int pump_roadmap_info(const pump_roadmap* rm, int32_t* n, int64_t* n_edges, float* ms_build);
/* Use `rm` (NULL: none) for the graph of later pump_setup / pump_plan calls
 * on ctx.  PUMP_E_ARG if its radii differ from the context's or it holds
 * more samples than max_nodes - 1.  pump_setup then fails with PUMP_E_ARG if
 * the problem's samples differ from the roadmap's (compared bit for bit). */
int pump_set_roadmap(pump_ctx* ctx, const pump_roadmap* rm);

/* SampleFree(n) (Alg. 3) with the Halton sequence the paper samples with
 * (Sec. V-A).  Writes n states [n][6] (FP32) to device memory `out` on
 * `hip_stream` (NULL: the null stream) and returns once they are written.
 * Point i of the sequence has coordinate d = lo + (hi - lo) * phi_b(i) with
 * phi_b the radical inverse in base b = 2, 3, 5, 7, 11, 13 for
 * (px, py, pz, vx, vy, vz).  The first n - n_goal states are points
 * start .. over the box [lo, hi]; the last n_goal continue the sequence with
 * positions over `goal` and velocities over [lo, hi] (Alg. 3 asks for at least
 * one sample from X_goal; `goal` may be NULL when n_goal = 0).  Samples that
 * fall in obstacles are dropped by pump_setup as usual.  PUMP_E_ARG for n < 1,
 * n_goal outside [0, n], an empty or non-finite box, or start + n >= 2^31. */
int pump_sample_halton(int32_t n, int32_t n_goal, const float* lo, const float* hi,
                       const pump_aabb* goal, int64_t start, float* out, void* hip_stream);

/* Per-kernel timing.  When on, every launch of the kernels below is
 * bracketed by HIP events on the context's stream and the elapsed times are
 * accumulated per kind:
 *   0 deviation table   1 graph pass 1 (all pairs)   2 graph pass 2 (fill)
 *   3 expand, pair stage (per-phase mode)   4 prune (staircase update + mark)
 *   5 compact (scans + scatter)   6 next group (min, flags, scans)
 *   7 front selection   8 MC certification   9 Explore as one launch
 *   10..16 phases of the single-launch Explore as seen by its first
 *   workgroup (expand, simulate, staircase, marks, scans + compaction,
 *   next group, group scatter + pair offsets; each includes its barrier;
 *   "launches" counts rounds)   17 Smooth (all of its launches)
 *   18 expand, particle stage (per-phase mode)
 * pump_set_timing(ctx, on) switches it and clears the totals;
 * pump_get_timing copies min(n, PUMP_TIMING_KINDS) totals (ms) and launch
 * counts (either pointer may be NULL). */
#define PUMP_TIMING_KINDS 19
int pump_set_timing(pump_ctx* ctx, int32_t on);
int pump_get_timing(pump_ctx* ctx, double* ms, int64_t* launches, int32_t n);

/* How pump_explore_run (and so pump_plan) runs Alg. 4's loop: mode 1 runs all
 * remaining rounds in one launch whose workgroups (all resident at once) meet
 * at grid-wide barriers; mode 0 launches each phase of each round separately
 * and reads the loop state back after every round (as pump_explore_round
 * always does); mode 2 (the default where the single launch fits) chooses
 * per query from the graph's edge count: the single launch below 4 * 2^20
 * edges, per-phase launches from there on, where the particle simulation's
 * own kernel is faster, and per-phase launches at any size with the
 * half-space model (cp_model 1).  All modes build the same plan store.  get
 * reports the configured mode and the workgroups of the single launch. */
int pump_set_explore_mode(pump_ctx* ctx, int32_t mode);
int pump_get_explore_mode(pump_ctx* ctx, int32_t* mode, int32_t* blocks);

/* Patience of the single launch's barrier waits, in milliseconds (default
 * 4000; 0 < ms <= 600000, else PUMP_E_ARG).  A workgroup that waits longer
 * (its team members were not all resident together, e.g. because other work
 * held compute units) makes every workgroup leave the launch; pump_plan and
 * pump_explore_run then redo Explore from the root with one launch per phase
 * (mode 0 for that call only), which gives the same plan store, and count
 * the event.  They do the same when a round of the single launch has more
 * pairs than cap_pairs (the per-phase rounds run it in chunks).  pump_get_explore_fallbacks reports how many times that
 * happened on this context. */
int pump_set_barrier_patience(pump_ctx* ctx, double ms);
int pump_get_explore_fallbacks(pump_ctx* ctx, int64_t* n);

/* ---------------------------------------------------------------------------
 * Learned sampling proposal.  The paper draws SampleFree(n) uniformly (Alg. 3;
 * Halton in Sec. V-A); a learned proposal only changes that sample set (half
 * learned, half uniform), and every plan is still certified by MC(p) in
 * Alg. 5.  Network: condition vector of 396 floats (start state 6, goal box
 * centre 3 and half-size 3, then up to 64 obstacle boxes as lo xyz, hi xyz,
 * zero padded) -> 4 hidden layers of 256 with ReLU -> 208 outputs: 16 mixture
 * logits, then 16 x 6 means, then 16 x 6 log standard deviations (clamped to
 * [-4, 2]) of a diagonal Gaussian mixture over the 6-D state.  Weights are
 * kept as FP32 masters with BF16 copies; matrix products take BF16 operands
 * with FP32 accumulation.  Parameters are one flat FP32 array: for each layer
 * W [out][in] row-major, then b [out].
 * Array arguments are host or device memory as `mem` says; every call returns
 * after its device work has finished.  Errors: PUMP_E_ARG (sizes), PUMP_E_HIP.
 * ------------------------------------------------------------------------- */
typedef struct pump_mlp pump_mlp;
#define PUMP_MLP_IN  396
#define PUMP_MLP_OUT 208

/* Create a network workspace for batches up to max_batch rows. */
int pump_mlp_create(int32_t max_batch, void* hip_stream, pump_mlp** out);
int pump_mlp_destroy(pump_mlp* m);
/* Number of parameters (352464). */
int pump_mlp_num_params(void);
/* Load FP32 parameters from the host (resets the Adam moments) / read them. */
int pump_mlp_set_params(pump_mlp* m, const float* params, int64_t n);
int pump_mlp_get_params(pump_mlp* m, float* params, int64_t n);
/* Checkpoint and resume of training: the FP32 parameters, Adam's first and
 * second moment estimates (each [n] host arrays, n = pump_mlp_num_params())
 * and the step counter t.  set restores all four (the BF16 copies are
 * refreshed), so training resumed from a saved state takes exactly the
 * steps the uninterrupted run would.  pump_mlp_set_params instead resets the
 * moments and t to zero. */
int pump_mlp_get_state(pump_mlp* m, float* params, float* m1, float* m2, int64_t n, int32_t* t);
int pump_mlp_set_state(pump_mlp* m, const float* params, const float* m1, const float* m2,
                       int64_t n, int32_t t);
/* One Adam step (Kingma and Ba; beta1 0.9, beta2 0.999, eps 1e-8, bias
 * corrections at step t + 1) on the given gradient vector grads [n] (host or
 * device per mem) instead of the network's own; the training step's update. */
int pump_mlp_adam_step(pump_mlp* m, const float* grads, int64_t n, float lr, int32_t mem);
/* out [B][208] = network outputs for cond [B][396]. */
int pump_mlp_forward(pump_mlp* m, const float* cond, int32_t B, float* out, int32_t mem);
/* Mean mixture negative log-likelihood of target states [B][6] and its
 * gradient (flat, same layout as the parameters; grads may be NULL). */
int pump_mlp_loss_grad(pump_mlp* m, const float* cond, const float* target, int32_t B,
                       float* loss, float* grads, int32_t mem);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) on the mean NLL of the batch. */
int pump_mlp_train_step(pump_mlp* m, const float* cond, const float* target, int32_t B,
                        float lr, float* loss, int32_t mem);
/* Condition vectors [q][396] from device arrays: x_init [q][6], goal boxes
 * [q][6] (lo xyz, hi xyz), boxes [q][max_boxes_in][6], n_obs [q]. */
int pump_mlp_condition(pump_mlp* m, const float* x_init, const float* goal, const float* boxes,
                       const int32_t* n_obs, int32_t q, int32_t max_boxes_in, float* cond);
/* n draws per query from the mixture: the component is chosen by inverse CDF
 * of softmax(logits) at u [q][n] (uniform in [0, 1)), the state is
 * mean + exp(log-std) * eps [q][n][6] (standard normals), clamped to the
 * state box (positions [0, 1], velocities [-0.5, 0.5]); out [q][n][6]. */
int pump_mlp_sample(pump_mlp* m, const float* cond, int32_t q, const float* u, const float* eps,
                    int32_t n, float* out, int32_t mem);
/* pump_mlp_sample for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same draws, bit for bit, with no allocation or free on the call.  With
 * host memory (mem != PUMP_MEM_DEVICE) u, eps and out are staged through a
 * static per-GPU array of 2^21 floats that the library holds until the
 * process ends, so q * n * 13 must not exceed 2^21 (q * n <= 161319 draws);
 * larger requests return PUMP_E_CAPACITY with the limit in the message.
 * Every call on one GPU shares that array: calls that overlap on one GPU (from
 * several threads or streams) race and must be serialised by the caller.
 * Device memory needs no staging and has no limit beyond pump_mlp_sample's. */
int pump_mlp_sample_noalloc(pump_mlp* m, const float* cond, int32_t q, const float* u,
                            const float* eps, int32_t n, float* out, int32_t mem);
const char* pump_mlp_last_error(const pump_mlp* m);

/* -------------------------------------------------------------------------
 * Batched engine.  Many independent queries (Alg. 2 each: BuildGraph, Explore,
 * PlanSelection), of uneven sizes, planned by one sequence of device launches
 * with no host round trip between them, captured in one HIP graph.  Setup
 * and selection run as batched kernels with the query index as a grid
 * dimension; Explore runs in one persistent kernel whose workgroups take
 * slots of a device queue; the workgroups holding a query's slots form a
 * team that runs all of its rounds, meeting at barriers (one workgroup for a
 * small query, several for a large one).  Each query's results equal those of pump_plan on
 * the same inputs (same per-element code, same orders).  Selection certifies
 * at most 32 Pareto-front plans per query (a larger front makes that query
 * report PUMP_E_CAPACITY).
 * ------------------------------------------------------------------------- */
typedef struct pump_batch pump_batch;

/* Shape of the persistent Explore kernel (every shape gives the same results). */
typedef struct pump_batch_tuning {
    int32_t explore_threads; /* threads per workgroup: 256 */
    int32_t blocks_per_cu;   /* 1..8 persistent workgroups per compute unit */
    int32_t order;           /* 0: queue in input order; 1: largest query first */
    int32_t use_graph;       /* 1: capture the launches in a HIP graph and launch it */
    int32_t team_scale;      /* workgroups per query: 0 = one; 1..256: k/4 times the
                                query's share of the estimated work (samples^2 x
                                sqrt(particles)) of all workgroups, at most 64
                                workgroups per team */
} pump_batch_tuning;

/* Allocate per-query workspaces for up to max_queries queries, each sized by
 * *cfg (n_particles is the largest particle count a query may use, max_nodes
 * the largest n + 1, and so on).  hip_stream NULL creates a private stream.
 * Errors: PUMP_E_ARG (unsupported configuration), PUMP_E_HIP (allocation). */
int pump_batch_create(const pump_config* cfg, int32_t max_queries, void* hip_stream,
                      pump_batch** out);
int pump_batch_destroy(pump_batch* b);
/* Plan q queries.  probs[i] must have mem == PUMP_MEM_DEVICE (every array on
 * the device, read only, kept alive until the call returns); n_particles[i]
 * is that query's N (32/64/128/256, at most cfg.n_particles; noise arrays are
 * [S_max][6][N] for that N).  tune may be NULL (256 threads, 2 per CU,
 * largest first, graph on, team_scale 64).  out[i] receives query i's result; the returned
 * code is PUMP_OK or the first negative per-query status.  ms_total holds the
 * wall time of the whole batch. */
int pump_batch_plan(pump_batch* b, const pump_problem* probs, const int32_t* n_particles,
                    int32_t q, const pump_batch_tuning* tune, pump_result* out);
/* Cached roadmaps for the queries of later pump_batch_plan calls: query i
 * (i < n) builds its graph from rms[i] (NULL: from scratch), as
 * pump_set_roadmap does for a context; n = 0 clears them.  PUMP_E_ARG if a
 * roadmap's radii differ from the batch configuration's or it holds more
 * than max_nodes - 1 samples; at plan time a query whose sample count
 * differs from its roadmap's fails the call, one whose samples differ gets
 * PUMP_E_ARG as its own status.  The roadmaps must outlive their use. */
int pump_batch_set_roadmaps(pump_batch* b, const pump_roadmap* const* rms, int32_t n);
/* Node ids (x_init = 0, sample k = k + 1) of plan `plan` of query `query`
 * from the last pump_batch_plan call, root first. */
int pump_batch_get_path(pump_batch* b, int32_t query, int32_t plan, int32_t* nodes, int32_t cap,
                        int32_t* len);
/* Autotuner: time every persistent-kernel shape (threads x workgroups per CU x
 * team scale, largest first, graph on) on these queries, check that every shape returns the same
 * per-query results, write the timings as JSON to json_path (if not NULL)
 * and return the fastest shape and its time. */
int pump_batch_tune(pump_batch* b, const pump_problem* probs, const int32_t* n_particles,
                    int32_t q, pump_batch_tuning* best, double* best_ms, const char* json_path);
const char* pump_batch_last_error(const pump_batch* b);

/* Status text for a code, and the last error message of a context. */
const char* pump_status_str(int status);
const char* pump_last_error(const pump_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* PUMP_H */
