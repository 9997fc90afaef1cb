/*
 * kpx.h -- C ABI of the Kino-PAX+ planner hot path on AMD Instinct MI355X
 * (gfx950): the per-iteration select -> propagate -> prune -> insert cycle of
 * "Kino-PAX+: Near-Optimal Massively Parallel Kinodynamic Sampling-based
 * Motion Planner" (arXiv 2602.02846), Alg. 1-4 and App. A.
 *
 * Conventions
 *   - Plain C types only.  "host" pointers are CPU memory owned by the caller
 *     and only read or written during the call; "device" pointers are GPU
 *     memory.  No call keeps a pointer the caller passed in, except the
 *     optional workspace given to kpx_create (used until kpx_destroy).
 *   - Every call returns a status: 0 = KPX_OK, > 0 informational, < 0 error.
 *     No exception or abort crosses this boundary.  kpx_last_error() gives a
 *     message for the last failing call on a handle.
 *   - A handle is not thread-safe; all its GPU work runs in order on one HIP
 *     stream (the caller's, or the default stream when NULL is passed).
 *   - Node status codes: 0 = active (V_A), 1 = inactive (V_I),
 *     2 = terminal (V_T); V_U is the per-iteration survivor mask (Sec. IV).
 *   - Beside the planner: batches of independent queries (kpx_batch_*), the
 *     adaptive decomposition (kpx_refine), and the differentiable quadrotor
 *     edge rollout with its gradient (kpx_diff_*), also used to polish the
 *     planner's inserted edges (kpx_set_polish).
 */
#ifndef KPX_H
#define KPX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KPX_MAX_STATE 12
#define KPX_MAX_CONTROL 4
#define KPX_MAX_BOXES 1024

/* status codes */
#define KPX_OK 0
#define KPX_FULL 1               /* the tree cannot take another iteration (App. A, t_e) */
#define KPX_ERR_ARG (-1)         /* invalid argument, size or NULL pointer */
#define KPX_ERR_INVALID_START (-2) /* x_init is not in the (planning) valid set */
#define KPX_ERR_OOM (-3)         /* device memory or workspace too small */
#define KPX_ERR_DEVICE (-4)      /* a HIP runtime call failed */
#define KPX_ERR_BUFFER (-5)      /* a caller buffer is too small */
#define KPX_ERR_STATE (-6)       /* call not valid in the handle's current state */

/* robot models (Sec. V): double integrator, nonlinear quadrotor, Dubins airplane */
#define KPX_DI6 0
#define KPX_QUAD12 1
#define KPX_DUBINS6 2

/* trajectory cost satisfying Assumption 1 */
#define KPX_COST_TIME 0          /* duration; stored as the total integer RK4 step count */
#define KPX_COST_PATH_LENGTH 1   /* length of the position path; stored as float32 bits */

#define KPX_ACTIVE 0
#define KPX_INACTIVE 1
#define KPX_TERMINAL 2

/*
 * Problem 1 (Sec. III): dynamics x' = f(x, u) (Eq. 1), compact state and
 * control sets, the valid set (workspace, state bounds, box obstacles),
 * x_init in the valid set, a goal set inside it, and the cost.
 *
 *   state layouts    DI6     p(3) v(3)
 *                    QUAD12  p(3) roll pitch yaw  v(3, world frame)  body rates(3)
 *                    DUBINS6 x y z yaw pitch speed
 *   control layouts  DI6 acceleration(3); QUAD12 thrust, torque(3);
 *                    DUBINS6 yaw rate, pitch rate, acceleration
 *   dyn_params       QUAD12: mass, Ixx, Iyy, Izz, gravity; unused otherwise
 *   boxes            host, n_boxes x 6 floats (lo x y z, hi x y z); copied
 *   margin           planning clearance: boxes grow and workspace, state
 *                    bounds and goal radius shrink by it (0 allowed)
 *   goal             closed ball over the position coordinates
 * Unused trailing entries of the fixed-size arrays are ignored.  State bounds
 * may be +-INFINITY.
 */
typedef struct kpx_problem {
    int32_t dynamics;
    int32_t cost;
    float dyn_params[8];
    float x_init[KPX_MAX_STATE];
    float x_lo[KPX_MAX_STATE];
    float x_hi[KPX_MAX_STATE];
    float u_lo[KPX_MAX_CONTROL];
    float u_hi[KPX_MAX_CONTROL];
    float ws_lo[3];
    float ws_hi[3];
    const float* boxes;
    int32_t n_boxes;
    float margin;
    float goal_center[3];
    float goal_radius;
} kpx_problem;

/*
 * Algorithm parameters (Alg. 1 inputs, App. A sizing).
 *   dt, steps_min..steps_max  one expansion integrates n RK4 steps of size dt,
 *                             n uniform in [steps_min, steps_max] (duration in (0, T_prop]);
 *                             1 <= steps_min <= steps_max <= 32767
 *   grid, vel_sign_bins       region decomposition R: grid[a] cells per
 *                             position axis over the workspace, times 8
 *                             velocity-sign classes when vel_sign_bins = 1
 *                             (DI6 and QUAD12 only)
 *   n_select                  at most this many active nodes are expanded per
 *                             iteration, taken in region order from a rotating cursor
 *   samples_per_node          K (the branching factor lambda); 0 selects the
 *                             uncapped form of Sec. VI-A / App. A: every active
 *                             node (up to n_select) with lambda =
 *                             max(1, floor(n_select / |selected|)) samples, so that
 *                             n_select is the size of the candidate buffer
 *   tree_cap                  t_e: capacity of the tree
 *   i_max                     inactivity threshold I_max (0..254)
 *   seed, query_id            Philox4x32-10 key and counter field
 *   refine_max                the largest total factor per axis by which
 *                             kpx_refine may later divide the grid cells
 *                             (0 or 1: never); region arrays are sized for it
 */
typedef struct kpx_params {
    float dt;
    int32_t steps_min;
    int32_t steps_max;
    int32_t grid[3];
    int32_t vel_sign_bins;
    int32_t n_select;
    int32_t samples_per_node;
    int32_t i_max;
    int64_t tree_cap;
    uint64_t seed;
    uint32_t query_id;
    uint32_t refine_max;
} kpx_params;

typedef struct kpx_handle kpx_handle;

/* Device counters after the last completed iteration. */
typedef struct kpx_counters {
    int64_t n_tree;                    /* nodes in T */
    int64_t iteration;                 /* completed iterations */
    int64_t cursor;                    /* region the next selection starts from */
    int64_t n_select;                  /* nodes expanded in the last iteration */
    int64_t n_valid;                   /* valid expansions in the last iteration */
    int64_t n_survivors;               /* nodes added in the last iteration */
    int64_t substeps;                  /* RK4 substeps integrated in the last iteration */
    int64_t first_solution_iteration;  /* -1 until a goal node exists */
    uint64_t solution_key;             /* (cost field << 32) | tree index; all ones = none */
    int32_t full;                      /* 1 once the capacity pre-check failed */
    int32_t samples_per_node;          /* samples per node in the last iteration */
} kpx_counters;

typedef struct kpx_solution_info {
    int32_t found;
    int32_t n_edges;
    int64_t tree_index;
    uint32_t cost_field;               /* TIME: steps; PATH_LENGTH: float32 bits */
    uint32_t reserved;
    double cost;                       /* TIME: steps * dt seconds; PATH_LENGTH: length */
    int64_t first_solution_iteration;
    int64_t n_tree;
    int64_t iteration;
} kpx_solution_info;

/* Host buffers for kpx_snapshot; any pointer may be NULL (not copied).
 * Per-node arrays hold at least `capacity` entries; state and control are
 * component-major: state[k * capacity + i] is component k of node i. */
typedef struct kpx_tree_view {
    int64_t capacity;
    float* state;        /* KPX_MAX_STATE x capacity */
    float* control;      /* KPX_MAX_CONTROL x capacity */
    int32_t* steps;
    int32_t* parent;     /* -1 for the root */
    uint32_t* cost;      /* cost field */
    int32_t* cell;
    uint8_t* status;
    uint8_t* icount;
    uint64_t* cell_table;  /* n_cells keys: (cost field << 32) | owner; all ones = never reached */
    int64_t cell_table_len;
} kpx_tree_view;

/* Host buffers for kpx_read_dump: the last iteration's expansions, one entry
 * per slot s = r * K + j (r-th selected node, j-th sample, K the samples per
 * node of that iteration).  Any pointer may be
 * NULL.  state and control are component-major with leading dimension `capacity`. */
typedef struct kpx_dump_view {
    int64_t capacity;
    int32_t* parent;
    float* control;        /* KPX_MAX_CONTROL x capacity */
    int32_t* steps;
    float* state;          /* end state, KPX_MAX_STATE x capacity (valid slots) */
    int32_t* first_invalid;/* 0 when valid, else the first invalid substep (1-based);
                            * -1: obstacle test skipped (kpx_set_cost_first) */
    int32_t* cell;         /* -1 when invalid */
    uint64_t* key;         /* (cost field << 32) | (n_tree + s); all ones when invalid */
    uint8_t* goal;
    uint8_t* survivor;
    /* edge polish (kpx_set_polish): one entry per node the iteration inserted,
     * in insertion order (kpx_counters.n_survivors entries; zeros with polish
     * off) */
    int32_t* polish_first_invalid; /* first invalid step of the polished edge, 0 when valid */
    int32_t* polish_cell;          /* region of the polished edge's end state, -1 when invalid */
    uint8_t* polish_goal;          /* 1 when that end state lies in the goal set */
    uint8_t* polish_accepted;      /* 1 when the polished edge replaced the node's edge */
} kpx_dump_view;

/* One record per completed iteration (ring of kpx_stats_capacity entries). */
typedef struct kpx_iter_stats {
    int64_t iteration;
    int64_t n_tree;           /* after the iteration */
    int32_t n_select;
    int32_t n_valid;
    int32_t n_survivors;
    int32_t samples_per_node;
    int64_t substeps;
    uint64_t solution_key;
    uint64_t t_begin;         /* device wall clock ticks (kpx_clock_rate_khz) */
    uint64_t t_end;
    int64_t n_live;           /* regions a tree node still owned after propagate (the
                               * owners prune examines) */
} kpx_iter_stats;

/* Bytes of device workspace kpx_create needs for this problem.  Pure host
 * computation.  Returns KPX_ERR_ARG for invalid sizes. */
int kpx_workspace_bytes(const kpx_problem* prob, const kpx_params* prm, size_t* out_bytes);

/* Validates the problem and parameters (Problem 1; capacity >= 1 + the most
 * survivors one iteration can add), copies them, allocates the tree, region
 * table and per-iteration buffers on the device (or carves them from
 * `workspace`, a device buffer of `workspace_bytes` >= kpx_workspace_bytes,
 * which the caller keeps alive until kpx_destroy), and runs the initialisation of Alg. 1:
 * root = x_init (active), every region at infinite cost except the root's,
 * which holds (0, root), no solution.  hip_stream: a hipStream_t or NULL.
 * Errors: KPX_ERR_ARG, KPX_ERR_INVALID_START (checked on the host before any
 * GPU call), KPX_ERR_OOM, KPX_ERR_DEVICE.  *out is NULL on error. */
int kpx_create(const kpx_problem* prob, const kpx_params* prm, void* hip_stream, void* workspace,
               size_t workspace_bytes, kpx_handle** out);

/* Enqueues n_iters iterations of Alg. 1's loop body (Propagate, PruneNodes,
 * UpdateTree, each preceded by the selection of the nodes to expand) on the
 * handle's stream and returns without waiting.  Counts stay on the device.
 * Once the capacity pre-check fails the iterations do nothing; the host
 * learns this at the next kpx_sync / kpx_counters / kpx_solution, after
 * which kpx_iterate returns KPX_FULL.  n_iters >= 0. */
int kpx_iterate(kpx_handle* h, int32_t n_iters);

/* Waits for the handle's stream; returns KPX_FULL if the tree is full, else KPX_OK. */
int kpx_sync(kpx_handle* h);

/* Waits and copies the device counters to *out (host). */
int kpx_counters_read(kpx_handle* h, kpx_counters* out);

/* Waits, then returns the best goal node's trajectory (Alg. 4).  A root that
 * lies in the goal set (planning radius: goal radius minus the margin) is the
 * solution from the start: cost 0, no edge, first_solution_iteration 0.
 * Layout:
 * states (n_edges + 1) x KPX_MAX_STATE row-major starting at x_init,
 * controls n_edges x KPX_MAX_CONTROL, steps n_edges (host buffers, may be NULL).
 * If capacity_edges < n_edges only *info is filled and KPX_ERR_BUFFER is returned. */
int kpx_solution(kpx_handle* h, kpx_solution_info* info, float* states, float* controls,
                 int32_t* steps, int32_t capacity_edges);

/* Waits and copies the tree, region table and counters to host buffers.
 * KPX_ERR_BUFFER when view->capacity < n_tree or cell_table_len < n_cells. */
int kpx_snapshot(kpx_handle* h, kpx_tree_view* view, kpx_counters* counters);

/* Records every expansion of the following iterations for kpx_read_dump
 * (enable = 1) or stops recording (0).  Recording costs extra stores only. */
int kpx_set_dump(kpx_handle* h, int32_t enable);

/* Waits and copies the last recorded iteration's expansions; *n_slots gets the
 * slot count (n_select * K).  KPX_ERR_STATE when recording is off;
 * KPX_ERR_BUFFER when view->capacity < n_slots. */
int kpx_read_dump(kpx_handle* h, kpx_dump_view* view, int64_t* n_slots);

/* Propagate in the cost-first form of the App. A remark (enable = 1) or the
 * plain form (0, the default) from the next iteration on.  The form is exact:
 * an edge is integrated with the state and workspace bounds only, and its
 * obstacle test is run (by integrating it again) only when its key
 * (cost << 32 | index) is not above its region's entry in the table at that
 * moment, so the tree, the table, the statuses and the solution are those of
 * the plain form.  What differs is recorded per slot: an edge whose obstacle
 * test was skipped has first_invalid -1 in kpx_read_dump and counts as
 * invalid in n_valid; an edge that leaves the bounds after entering a box
 * reports the bound's substep; kpx_iter_stats.substeps counts the substeps of
 * both passes.  The batched form (kpx_batch_*) always propagates in the plain
 * form.  KPX_ERR_ARG for enable outside 0..1. */
int kpx_set_cost_first(kpx_handle* h, int32_t enable);

/* Brackets the kernels of every following iteration with HIP events on the
 * handle's stream: bit k of kernel_mask (0..15) times kernel k (numbered as
 * in kpx_read_timing); 0 stops.  Each call clears the accumulated times.
 * The edge-polish kernel (kpx_set_polish) is not among them.
 * KPX_ERR_ARG for a mask outside 0..15. */
int kpx_set_timing(kpx_handle* h, int32_t kernel_mask);

/* Times the selected kernels only in every period-th iteration from now on
 * (1, the default: every iteration), so that the events' own cost stays
 * small in long runs.  KPX_ERR_ARG for period < 1. */
int kpx_set_timing_every(kpx_handle* h, int32_t period);

/* Waits and returns, per kernel (0 propagate, 1 prune + survivor flags,
 * 2 insert, 3 close of the iteration + next selection), the summed
 * milliseconds and the number of launches timed since timing was enabled.
 * Only iterations that ran count: those enqueued after the tree filled
 * return at once and their launches are left out. */
int kpx_read_timing(kpx_handle* h, double ms[4], int64_t launches[4]);

/* Number of per-iteration records kept (a ring indexed by iteration). */
int kpx_stats_capacity(const kpx_handle* h, int64_t* out);

/* Waits and copies the records of iterations first .. first + count - 1
 * (each must be among the last kpx_stats_capacity iterations) to out (host). */
int kpx_read_stats(kpx_handle* h, int64_t first, int64_t count, kpx_iter_stats* out);

/* Device wall-clock rate for kpx_iter_stats timestamps, in kHz. */
int kpx_clock_rate_khz(kpx_handle* h, int64_t* out);

/* Diagnostic: evaluates the device Philox4x32-10 block function (the one the
 * expansions use) on n host (counter, key) records of 6 words
 * (c0 c1 c2 c3 k0 k1) and writes 4 words per record to host out. Runs on the
 * current device with its own short-lived buffers. */
int kpx_philox(const uint32_t* counter_key, int64_t n, uint32_t* out);

/* kpx_philox without any allocation, for callers that cannot allocate device
 * memory (tight loops, code that forbids hipMalloc): the same records and
 * results, staged through a buffer the library holds in static device memory
 * (10 * KPX_PHILOX_STATIC_MAX words, 2.5 MiB, kept by each device it runs on
 * until the process ends).  It runs on the current device and the default
 * stream and waits for its copies.  Every call on a device shares that
 * device's buffer: calls that overlap on one device (from several host
 * threads) race.  KPX_ERR_ARG for n > KPX_PHILOX_STATIC_MAX, n < 0 or NULL
 * buffers; KPX_ERR_DEVICE when a runtime call fails. */
#define KPX_PHILOX_STATIC_MAX 65536
int kpx_philox_static(const uint32_t* counter_key, int64_t n, uint32_t* out);

/* Releases what the library allocated (not a caller workspace).  NULL is ok. */
int kpx_destroy(kpx_handle* h);

/* Adaptive decomposition (the paper's remark on non-uniform and adaptive
 * decompositions, Sec. IV, which defers their analysis): between iterations,
 * divides every grid cell of R into factor^3 cells (the grid becomes
 * grid * factor per axis; velocity-sign classes are kept).  Every node's
 * region is recomputed from its state; the region table is rebuilt from the
 * nodes that are not terminal (at most one per old region, so at most one per
 * new one: each stays its region's best); terminal nodes stay terminal; the
 * selection cursor moves to the first new cell of its old cell; the tree is
 * marked full when the larger survivor bound no longer fits; the next
 * iteration's nodes are selected again over the refined regions.
 * KPX_ERR_ARG for factor < 2 or a total factor beyond params.refine_max.
 * Batches made before a refinement refuse to run. */
int kpx_refine(kpx_handle* h, int32_t factor);

/* Edge polish of inserted nodes, an extension past the paper (which cites
 * gradient-based trajectory optimization only as related work, Sec. I-A).
 * With steps > 0, every iteration ends its insertion by polishing each node
 * it inserted: the node's control u takes `steps` projected gradient steps
 *   u <- clamp(u - lr grad L(u, u, u, u), control box)
 * on the loss of the differentiable edges below (all 4 segments tied to u,
 * the margin-grown boxes, the goal centre, the given weights; w_len weighs
 * the edge's path length).  The polished edge, integrated and checked as
 * propagate does, replaces the node's edge when it is valid, ends in the
 * node's region and keeps a goal node in the goal, and, under
 * KPX_COST_PATH_LENGTH, is shorter; a node that enters the goal competes for
 * the solution (Alg. 4).  Under KPX_COST_TIME the node's cost (its step
 * count) does not change; under KPX_COST_PATH_LENGTH the shorter edge lowers
 * the node's cost and its region's key (the node keeps the region and has no
 * descendants yet), and a goal node's solution key.  Statuses do not change. */
typedef struct kpx_polish {
    int32_t steps;           /* 0 = off (also NULL); at most 16 */
    float lr;                /* >= 0 */
    float w_ctrl, w_obst, k_obst, d_safe, w_goal;
    float w_len;             /* weight of the path length in the loss */
    int32_t goal_only;       /* 1: polish only the nodes inserted in the goal set */
} kpx_polish;

/* Sets edge polish for later iterations.  KPX_ERR_ARG unless the handle is a
 * KPX_QUAD12 problem with steps_max <= 64, or for steps outside 0..16,
 * lr < 0, non-finite values or goal_only outside 0..1; KPX_ERR_DEVICE if
 * the kernel cannot get its shared memory.  Handles with polish on cannot be
 * batched. */
int kpx_set_polish(kpx_handle* h, const kpx_polish* p);

/* Static message for a status code. */
const char* kpx_status_string(int status);

/* Message for the last failing call on h (empty string if none). */
const char* kpx_last_error(const kpx_handle* h);

/* ---------------------------------------------------------------- batches
 * Independent queries (handles made by kpx_create, any mix of models, sizes,
 * obstacle sets and capacities) iterated together: each kernel of an
 * iteration is launched once for all the queries of one robot model and
 * cost, each such group on a stream of its own, so that small queries share
 * the GPU.  Every query computes exactly what kpx_iterate would compute for
 * it alone. */
typedef struct kpx_batch kpx_batch;

/* Groups n host-array handles (not copied; the caller keeps them alive and
 * destroys them after the batch).  They must be distinct, share one stream,
 * have run the same number of iterations modulo 2, and have edge polish off.
 * A handle that records its expansions (kpx_set_dump) when the batch is made
 * keeps recording in the batch, and kpx_read_dump reads them after each
 * batched iteration.  KPX_ERR_ARG otherwise;
 * KPX_ERR_OOM / KPX_ERR_DEVICE on allocation or runtime failure. */
int kpx_batch_create(kpx_handle* const* handles, int32_t n, kpx_batch** out);

/* enable = 1: kpx_batch_iterate replays HIP graphs of two iterations
 * (captured on first use on the batch's own stream); 0: plain launches.
 * KPX_ERR_ARG for other values. */
int kpx_batch_set_graph(kpx_batch* b, int32_t enable);

/* Propagate threads per block for the batch's queries of one robot model
 * (KPX_DI6 / KPX_QUAD12 / KPX_DUBINS6): 256 (one wave per SIMD, the default)
 * or 512 (two), the per-query thread count the samples-per-node autotuner
 * also tries.  Results do not depend on it.  Captured graphs are dropped and
 * captured again on the next iterate.  KPX_ERR_ARG for another thread count;
 * a model the batch does not hold is left alone. */
int kpx_batch_set_threads(kpx_batch* b, int32_t dynamics, int32_t threads);

/* Enqueues n_iters iterations of every query, ordered after the work already
 * on the handles' stream and before any later work on it; returns at once.
 * A query whose tree is full stops changing, as with kpx_iterate; each
 * handle's kpx_sync reports it.  KPX_ERR_STATE if a handle was iterated on
 * its own since the batch was made (an odd number of times), turned edge
 * polish on, or switched its recording on or off. */
int kpx_batch_iterate(kpx_batch* b, int32_t n_iters);

/* Waits for the batch's work and releases what the batch allocated (not the
 * handles).  NULL is ok. */
int kpx_batch_destroy(kpx_batch* b);

/* Message for the last failing call on b (empty string if none). */
const char* kpx_batch_last_error(const kpx_batch* b);

/* ------------------------------------------------------ differentiable edges
 * An extension past the paper, which cites gradient-based trajectory
 * optimization only as related work (Sec. I-A): loss and control gradient of
 * quadrotor edges (the Sec. V model and the planner's RK4 integrator), for
 * local refinement of edges.  A batch holds E independent edges, each n RK4 steps of
 * size dt (4 <= n <= 40) from x0 under 4 piecewise-constant control segments,
 * step k using segment j with floor(j n / 4) <= k < floor((j + 1) n / 4).
 * The loss of an edge is
 *   n dt + w_ctrl |u|^2 + w_obst sum_{k=1..n} softplus(k_obst (d_safe - sd(p_k)))
 *        + w_goal |p_n - goal|^2 + w_len l
 * with sd(p) the signed distance of position p to the nearest box (negative
 * inside) and l the length of the position path (the speed integrated by the
 * same RK4 steps, as the planner's KPX_COST_PATH_LENGTH is); the gradient is
 * with respect to the edge's 16 controls.  It is
 * computed by reverse mode through the RK4 steps, in float32.
 *
 * Device arrays are structure-of-arrays over the edges: x0 is 12 x E
 * (component i of edge e at i * E + e), u is 16 x E (control c of segment j
 * at (4 j + c) * E + e), n, loss are E, grad is 16 x E.  An edge with n
 * outside 4..40 gets loss NaN and a zero gradient. */
typedef struct kpx_diff_problem {
    float dyn_params[8];      /* mass, Ixx, Iyy, Izz, gravity (as for KPX_QUAD12) */
    float dt;                 /* RK4 step, > 0 */
    const float* boxes;       /* host, n_boxes x 6 (lo x y z, hi x y z); copied */
    int32_t n_boxes;          /* 0 .. KPX_MAX_BOXES */
    float goal[3];
    float w_ctrl, w_obst, k_obst, d_safe, w_goal;
    float u_lo[4], u_hi[4];   /* control box for kpx_diff_polish's projection */
    float x_lo[12], x_hi[12]; /* state bounds (may be +-INFINITY), for validity */
    float ws_lo[3], ws_hi[3]; /* workspace, for validity */
    float w_len;              /* weight of the path length (finite) */
} kpx_diff_problem;

typedef struct kpx_diff kpx_diff;

/* Copies the problem to the device.  hip_stream (a hipStream_t, NULL for the
 * default stream) orders every later call of the object.  KPX_ERR_ARG for
 * non-positive mass, inertia or dt, u_lo > u_hi, a box with lo > hi, or a
 * box count outside 0 .. KPX_MAX_BOXES;
 * KPX_ERR_OOM / KPX_ERR_DEVICE otherwise.  *out is NULL on error. */
int kpx_diff_create(const kpx_diff_problem* p, void* hip_stream, kpx_diff** out);

/* Enqueues loss (device, E) and, when grad (device, 16 x E) is not NULL, the
 * gradient of E edges (x0, u, n: device, layouts above); returns at once.
 * The inputs are only read.  E = 0 does nothing.  KPX_ERR_ARG for a NULL
 * pointer or E < 0; KPX_ERR_DEVICE if the launch fails. */
int kpx_diff_loss_grad(kpx_diff* d, const float* x0, const float* u, const int32_t* n, int64_t E, float* loss,
                       float* grad);

/* Enqueues `steps` projected gradient steps u <- clamp(u - lr grad, u_lo, u_hi)
 * on every edge, in place on u (device, 16 x E), and writes the loss of the
 * final controls to loss (device, E).  When first_invalid (device, E) is not
 * NULL it receives, for the final controls, the first step k in 1..n whose
 * state x_k leaves the valid set (outside the state bounds or the closed
 * workspace, or inside a closed box), 0 when all are valid, -1 for an
 * unsupported n.  steps = 0 only evaluates the loss (and validity).
 * KPX_ERR_ARG for steps < 0, lr < 0 or NaN, or as kpx_diff_loss_grad. */
int kpx_diff_polish(kpx_diff* d, const float* x0, float* u, const int32_t* n, int64_t E, int32_t steps, float lr,
                    float* loss, int32_t* first_invalid);

/* Waits for the object's work and releases it.  NULL is ok. */
int kpx_diff_destroy(kpx_diff* d);

/* Message for the last failing call on d (empty string if none). */
const char* kpx_diff_last_error(const kpx_diff* d);

#ifdef __cplusplus
}
#endif

#endif /* KPX_H */
