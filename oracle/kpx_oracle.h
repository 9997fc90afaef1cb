/*
 * kpx_oracle.h -- plain, sequential, float64 reference of one Kino-PAX+
 * iteration.  TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the
 * CPU-baseline leg of the benchmark call it; the planner library never does.
 *
 * It follows the paper (arXiv 2602.02846) step by step:
 *   Alg. 1  main loop: Propagate -> PruneNodes -> UpdateTree
 *   Alg. 2  Propagate: sample (u, duration), integrate, validity, region map,
 *           additive cost, region minimum, admission to V_U
 *   Alg. 3  PruneNodes: inactivity counter, reactivation, terminal, ancestor test
 *   Alg. 4  UpdateTree: re-check region minimum, append to T, solution update
 *   App. A  exclusive scan + GraphSearch compaction, append at |T| + rank
 * The readings taken where the paper is silent are listed with each function
 * in kpx_oracle.c.
 *
 * Every constant enters as a float32 value and is widened to float64 here.
 */
#ifndef KPX_ORACLE_H
#define KPX_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORA_MAX_STATE 12
#define ORA_MAX_CONTROL 4

enum { ORA_DI6 = 0, ORA_QUAD12 = 1, ORA_DUBINS6 = 2 };
enum { ORA_COST_TIME = 0, ORA_COST_PATH = 1 };
/* node sets of Sec. IV: V_A, V_I, V_T (V_U is the per-iteration survivor mask) */
enum { ORA_ACTIVE = 0, ORA_INACTIVE = 1, ORA_TERMINAL = 2 };
enum { ORA_OK = 0, ORA_FULL = 1, ORA_ERR_ARG = -1, ORA_ERR_INVALID_START = -2 };

/* Reasons a decision fell within `band` of its threshold (the two sides of
 * the comparison may then legitimately disagree under rounding). */
enum {
    ORA_FLAG_BOX = 1u,        /* a substep within band of an (inflated) box face */
    ORA_FLAG_WORKSPACE = 2u,  /* within band of a workspace face */
    ORA_FLAG_BOUND = 4u,      /* within band of a state bound */
    ORA_FLAG_CELL = 8u,       /* end state within band of a region face */
    ORA_FLAG_VSIGN = 16u,     /* velocity component within band of 0 (sign bins) */
    ORA_FLAG_GOAL = 32u,      /* end state within band of the goal sphere */
    ORA_FLAG_TIE = 64u        /* path-length cost within relative band of a rival */
};

typedef struct {
    int32_t dynamics;          /* ORA_DI6 / ORA_QUAD12 / ORA_DUBINS6 */
    int32_t cost;              /* ORA_COST_TIME / ORA_COST_PATH */
    float dyn_params[8];       /* QUAD12: m, Ixx, Iyy, Izz, g */
    float x_init[ORA_MAX_STATE];
    float x_lo[ORA_MAX_STATE]; /* +-inf = unbounded */
    float x_hi[ORA_MAX_STATE];
    float u_lo[ORA_MAX_CONTROL];
    float u_hi[ORA_MAX_CONTROL];
    float ws_lo[3], ws_hi[3];
    const float* boxes;        /* n_boxes x 6: lo xyz, hi xyz */
    int32_t n_boxes;
    float margin;              /* planning clearance margin */
    float goal_center[3];
    float goal_radius;
    float dt;                  /* RK4 step */
    int32_t steps_min, steps_max;
    int32_t grid[3];
    int32_t vel_sign_bins;
    int32_t n_select, samples_per_node;
    int64_t tree_cap;
    int32_t i_max;
    uint64_t seed;
    uint32_t query_id;
    double band;               /* flag band for decisions (1e-5) */
    /* edge polish of every inserted node (QUAD12; steps 0 = off): projected
     * gradient steps on the node's control of the tied loss of
     * kpx_oracle_diff.h over the margin-grown boxes */
    int32_t polish_steps;
    double polish_lr, polish_w_ctrl, polish_w_obst, polish_k_obst, polish_d_safe, polish_w_goal;
    double polish_w_len;
    int32_t polish_goal_only;  /* 1: only the nodes inserted in the goal set */
} ora_problem;

typedef struct {
    int64_t cap, n_tree;
    double* x;          /* cap x 12 */
    float* u;           /* cap x 4 */
    int32_t* steps;
    int64_t* parent;    /* -1 for the root */
    double* cost;
    int64_t* cell;
    uint8_t* status;
    int32_t* icount;
    int64_t n_cells;
    double* tbl_cost;   /* n_cells; +inf when the region was never reached */
    int64_t* tbl_id;    /* n_cells; -1 when the region was never reached */
    int64_t cursor;     /* region index the next selection starts from */
    int64_t iter;
    double sol_cost;    /* +inf until a goal node exists */
    int64_t sol_id;
    int64_t first_sol_iter;
    int32_t full;
    int64_t last_n_sel, last_n_valid, last_n_surv;
} ora_tree;

typedef struct {
    int64_t cap_slots;
    int64_t n_slots;
    int64_t* parent;
    float* u;               /* cap_slots x 4 */
    int32_t* n;
    double* xn;             /* cap_slots x 12 */
    uint8_t* valid;
    int32_t* first_invalid; /* 0 when valid, else the first invalid substep */
    int32_t* substeps;      /* substeps integrated */
    uint32_t* flags;
    int64_t* cell;          /* -1 when invalid */
    double* cost;           /* cost from the root (parent cost + edge cost) */
    uint8_t* goal;
    uint8_t* survivor;
    int64_t* new_index;     /* tree index when a survivor, else -1 */
    uint8_t* polished;      /* per node inserted, in insertion order: 1 when edge
                             * polish replaced its edge (NULL: not recorded) */
    int64_t substeps_total;
    int64_t k;              /* samples per selected node in this iteration */
} ora_cands;

/* Decisions of an implementation under test.  The oracle adopts one only
 * where its own decision is flagged as within band, and only if it is one of
 * the outcomes that band allows.  Any pointer may be NULL. */
typedef struct {
    const int32_t* first_invalid;
    const int64_t* cell;
    const uint8_t* goal;
    const uint8_t* survivor;
    /* edge polish, per node inserted this iteration (insertion order): the
     * first invalid step of the polished edge (0 when valid) and the region and
     * goal decisions at its end state; each is adopted only where the oracle's
     * own decision of that test is flagged within band */
    const int32_t* polish_first_invalid;
    const int64_t* polish_cell;
    const uint8_t* polish_goal;
    /* ... and whether the polished edge replaced the node's edge, adopted only
     * where the path-length comparison (shorter or not) lies within band */
    const uint8_t* polish_accepted;
} ora_hints;

typedef struct {
    double xn[ORA_MAX_STATE];
    double length;
    int32_t first_invalid;
    int32_t substeps;
    uint32_t flags;
} ora_edge;

typedef struct {
    int32_t ok;
    int32_t starts_at_init;
    int32_t collision_free;
    int32_t within_bounds;
    int32_t reaches_goal;
    int32_t cost_ok;
    int32_t first_bad_edge, first_bad_substep;
    double cost;            /* recomputed: steps (TIME) or length (PATH) */
    double min_clearance;   /* min Chebyshev distance to any box over all substeps */
    double max_gap;         /* max |re-integrated - stored| state gap at edge ends */
    double goal_distance;
} ora_verify_report;

int ora_state_dim(int32_t dynamics);
/* Threads ora_step shares its expansions among: 1 for the plain build, the
 * OpenMP thread count for the timing build (liboracle_omp.so). */
int ora_threads(void);
int ora_control_dim(int32_t dynamics);

void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void ora_philox_many(const uint32_t* counter_key, int64_t n, uint32_t* out);
void ora_sample(const ora_problem* P, uint32_t iter, uint32_t slot, float u[ORA_MAX_CONTROL],
                int32_t* n);

void ora_deriv(const ora_problem* P, const double* z, const double* u, double* zdot);
void ora_rk4_step(const ora_problem* P, double* z, const double* u, double h);
void ora_integrate(const ora_problem* P, const double* x0, const double* u, int32_t n, double h,
                   double* z_out);

int ora_point_status(const ora_problem* P, const double* x, double margin, double band,
                     uint32_t* flags);
int64_t ora_cell_of(const ora_problem* P, const double* x, const int64_t* hint, uint32_t* flags);
int ora_goal_test(const ora_problem* P, const double* x, double radius, const uint8_t* hint,
                  uint32_t* flags);
void ora_propagate_edge(const ora_problem* P, const double* x0, const float* u, int32_t n,
                        int32_t hint_first_invalid, ora_edge* out);

void ora_exclusive_scan(const uint8_t* mask, int64_t n, int64_t* S);
int64_t ora_graph_search(const uint8_t* mask, const int64_t* S, int64_t n, int64_t* I);

int ora_init(const ora_problem* P, ora_tree* T);
int64_t ora_select(const ora_problem* P, const ora_tree* T, int64_t* sel, int64_t* cursor_next);
void ora_prune(const ora_problem* P, ora_tree* T);
int ora_step(const ora_problem* P, ora_tree* T, ora_cands* C, const ora_hints* H);

/* Adaptive decomposition: P already holds the refined grid (factor times the
 * old one per axis) and T's region arrays hold its regions.  Every node's
 * region is recomputed; the region table is rebuilt from the nodes that are
 * not terminal; the cursor moves to the first refined cell of its old cell;
 * the tree is marked full when the survivor bound no longer fits.  hint_cell
 * (optional, per node) is adopted where a region decision is within band. */
int ora_refine(const ora_problem* P, ora_tree* T, int32_t factor, const int64_t* hint_cell);

int ora_verify(const ora_problem* P, int32_t n_edges, const float* controls, const int32_t* steps,
               const float* states, double reported_cost, ora_verify_report* rep);

#ifdef __cplusplus
}
#endif

#endif /* KPX_ORACLE_H */
