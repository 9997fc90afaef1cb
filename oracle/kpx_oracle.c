/*
 * kpx_oracle.c -- plain float64 reference of Kino-PAX+ (arXiv 2602.02846).
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark use this file; the planner library never links it.
 *
 * Deliberately slow and literal: one slot after another, one node after
 * another, O(n) loops, no blocking, no fusion, no reordering.  Each function
 * names the passage of the paper it follows.  Readings taken where the paper
 * is silent are marked "Reading:".
 */
#include "kpx_oracle.h"
#include "kpx_oracle_diff.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int ora_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int ora_state_dim(int32_t dyn)
{
    switch (dyn) {
    case ORA_DI6: return 6;
    case ORA_QUAD12: return 12;
    case ORA_DUBINS6: return 6;
    default: return -1;
    }
}

int ora_control_dim(int32_t dyn)
{
    switch (dyn) {
    case ORA_DI6: return 3;
    case ORA_QUAD12: return 4;
    case ORA_DUBINS6: return 3;
    default: return -1;
    }
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11).  Each round multiplies counter words 0 and 2 by */
/* the two published 32-bit multipliers, and builds the new counter from the */
/* high halves xor-ed with the other two words and the key, and the low      */
/* halves.  The key is advanced by the two published Weyl increments before */
/* every round after the first.                                              */
/* ------------------------------------------------------------------------ */
void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t mul0 = 0xD2511F53u, mul1 = 0xCD9E8D57u;
    const uint32_t weyl0 = 0x9E3779B9u, weyl1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += weyl0;
            k1 += weyl1;
        }
        uint64_t p0 = (uint64_t)mul0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)mul1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* rows of (c0, c1, c2, c3, k0, k1) -> rows of 4 output words */
void ora_philox_many(const uint32_t* counter_key, int64_t n, uint32_t* out)
{
    for (int64_t i = 0; i < n; ++i)
        ora_philox4x32_10(&counter_key[6 * i], &counter_key[6 * i + 4], &out[4 * i]);
}

/* Random control and duration of one expansion (Alg. 2; Alg. 6).
 * Reading: counter = (iteration, slot, query, block), key = (seed low, seed
 * high).  Block b yields words 4b..4b+3.  Control i takes word i; the step
 * count takes word m (m = control dimension).  A word w maps to the uniform
 * (w >> 8) * 2^-24, and control i is fmaf(uniform, hi_i - lo_i, lo_i) in
 * float32 with one rounding.  The duration is n * dt with
 * n = n_min + floor(w_m * (n_max - n_min + 1) / 2^32), the discrete reading of
 * "duration in (0, T_prop]". */
void ora_sample(const ora_problem* P, uint32_t iter, uint32_t slot, float u[ORA_MAX_CONTROL],
                int32_t* n)
{
    uint32_t key[2] = {(uint32_t)(P->seed & 0xFFFFFFFFu), (uint32_t)(P->seed >> 32)};
    uint32_t words[8];
    for (uint32_t b = 0; b < 2; ++b) {
        uint32_t ctr[4] = {iter, slot, P->query_id, b};
        ora_philox4x32_10(ctr, key, &words[4 * b]);
    }
    int m = ora_control_dim(P->dynamics);
    for (int i = 0; i < ORA_MAX_CONTROL; ++i) u[i] = 0.0f;
    for (int i = 0; i < m; ++i) {
        float unit = (float)(words[i] >> 8) * 0x1p-24f;
        float span = P->u_hi[i] - P->u_lo[i];
        u[i] = fmaf(unit, span, P->u_lo[i]);
    }
    uint64_t range = (uint64_t)(P->steps_max - P->steps_min + 1);
    *n = P->steps_min + (int32_t)(((uint64_t)words[m] * range) >> 32);
}

/* ------------------------------------------------------------------------ */
/* Dynamics x' = f(x, u) (Eq. 1).  The paper only cites the models; the     */
/* equations below are the standard forms.  The integrated vector z carries  */
/* the state in z[0..d-1] and the accumulated path length in z[d].           */
/* ------------------------------------------------------------------------ */
void ora_deriv(const ora_problem* P, const double* z, const double* u, double* zdot)
{
    switch (P->dynamics) {
    case ORA_DI6: {
        /* position' = velocity, velocity' = acceleration control */
        for (int i = 0; i < 3; ++i) {
            zdot[i] = z[3 + i];
            zdot[3 + i] = u[i];
        }
        zdot[6] = sqrt(z[3] * z[3] + z[4] * z[4] + z[5] * z[5]);
        break;
    }
    case ORA_QUAD12: {
        /* state: position, ZYX Euler angles (roll phi, pitch theta, yaw psi),
         * world-frame velocity, body rates (p, q, r);
         * control: collective thrust T and body torques. */
        const double mass = P->dyn_params[0];
        const double jx = P->dyn_params[1], jy = P->dyn_params[2], jz = P->dyn_params[3];
        const double grav = P->dyn_params[4];
        const double phi = z[3], theta = z[4], psi = z[5];
        const double vx = z[6], vy = z[7], vz = z[8];
        const double wp = z[9], wq = z[10], wr = z[11];
        const double sphi = sin(phi), cphi = cos(phi);
        const double sth = sin(theta), cth = cos(theta);
        const double spsi = sin(psi), cpsi = cos(psi);
        zdot[0] = vx;
        zdot[1] = vy;
        zdot[2] = vz;
        /* Euler-angle rates from body rates */
        zdot[3] = wp + (sphi * wq + cphi * wr) * (sth / cth);
        zdot[4] = cphi * wq - sphi * wr;
        zdot[5] = (sphi * wq + cphi * wr) / cth;
        /* thrust along the body z axis rotated to the world frame, minus gravity */
        const double acc = u[0] / mass;
        zdot[6] = acc * (cpsi * sth * cphi + spsi * sphi);
        zdot[7] = acc * (spsi * sth * cphi - cpsi * sphi);
        zdot[8] = acc * (cth * cphi) - grav;
        /* Euler's rigid-body equations with a diagonal inertia */
        zdot[9] = (u[1] - (jz - jy) * wq * wr) / jx;
        zdot[10] = (u[2] - (jx - jz) * wp * wr) / jy;
        zdot[11] = (u[3] - (jy - jx) * wp * wq) / jz;
        zdot[12] = sqrt(vx * vx + vy * vy + vz * vz);
        break;
    }
    case ORA_DUBINS6: {
        /* state: x, y, z, yaw psi, pitch gamma, speed v;
         * control: yaw rate, pitch rate, acceleration */
        const double psi = z[3], gam = z[4], v = z[5];
        zdot[0] = v * cos(psi) * cos(gam);
        zdot[1] = v * sin(psi) * cos(gam);
        zdot[2] = v * sin(gam);
        zdot[3] = u[0];
        zdot[4] = u[1];
        zdot[5] = u[2];
        zdot[6] = v;
        break;
    }
    default:
        break;
    }
}

/* Classical four-stage Runge-Kutta step of size h on z = (x, length).
 * Reading: PropagateODE (Alg. 2) is not specified; RK4 with a fixed
 * step dt is used. */
void ora_rk4_step(const ora_problem* P, double* z, const double* u, double h)
{
    const int dim = ora_state_dim(P->dynamics) + 1;
    double k1[ORA_MAX_STATE + 1], k2[ORA_MAX_STATE + 1], k3[ORA_MAX_STATE + 1],
        k4[ORA_MAX_STATE + 1], t[ORA_MAX_STATE + 1];
    ora_deriv(P, z, u, k1);
    for (int i = 0; i < dim; ++i) t[i] = z[i] + 0.5 * h * k1[i];
    ora_deriv(P, t, u, k2);
    for (int i = 0; i < dim; ++i) t[i] = z[i] + 0.5 * h * k2[i];
    ora_deriv(P, t, u, k3);
    for (int i = 0; i < dim; ++i) t[i] = z[i] + h * k3[i];
    ora_deriv(P, t, u, k4);
    for (int i = 0; i < dim; ++i) z[i] += h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
}

void ora_integrate(const ora_problem* P, const double* x0, const double* u, int32_t n, double h,
                   double* z_out)
{
    const int d = ora_state_dim(P->dynamics);
    for (int i = 0; i < d; ++i) z_out[i] = x0[i];
    z_out[d] = 0.0;
    for (int32_t k = 0; k < n; ++k) ora_rk4_step(P, z_out, u, h);
}

/* ------------------------------------------------------------------------ */
/* Valid set (Sec. III): inside the workspace, within the state bounds and   */
/* outside every obstacle.  Reading: the robot is a point at its position    */
/* coordinates, obstacles are closed boxes (touching a face collides), the   */
/* workspace and bounds are closed (touching them is allowed).  For planning */
/* the boxes grow by `margin` and the workspace, bounds and goal shrink by   */
/* it (a clearance margin); verification uses margin 0.                      */
/*                                                                           */
/* Returns bit 0 = invalid (exact float64 decision), bit 1 = the decision is */
/* within `band` of a threshold and no check is violated by more than band.  */
/* ------------------------------------------------------------------------ */
int ora_point_status(const ora_problem* P, const double* x, double margin, double band,
                     uint32_t* flags)
{
    const int d = ora_state_dim(P->dynamics);
    int invalid = 0, clear_violation = 0, near = 0;
    uint32_t fl = 0;
    for (int a = 0; a < 3; ++a) {
        double lo = (double)P->ws_lo[a] + margin, hi = (double)P->ws_hi[a] - margin;
        double s = fmin(x[a] - lo, hi - x[a]);
        if (s < 0.0) invalid = 1;
        if (s < -band) clear_violation = 1;
        else if (fabs(s) <= band) { near = 1; fl |= ORA_FLAG_WORKSPACE; }
    }
    for (int i = 0; i < d; ++i) {
        double blo = (double)P->x_lo[i], bhi = (double)P->x_hi[i];
        if (isfinite(blo)) {
            double s = x[i] - (blo + margin);
            double b = band * fmax(1.0, fabs(blo));
            if (s < 0.0) invalid = 1;
            if (s < -b) clear_violation = 1;
            else if (fabs(s) <= b) { near = 1; fl |= ORA_FLAG_BOUND; }
        }
        if (isfinite(bhi)) {
            double s = (bhi - margin) - x[i];
            double b = band * fmax(1.0, fabs(bhi));
            if (s < 0.0) invalid = 1;
            if (s < -b) clear_violation = 1;
            else if (fabs(s) <= b) { near = 1; fl |= ORA_FLAG_BOUND; }
        }
    }
    for (int k = 0; k < P->n_boxes; ++k) {
        const float* bx = P->boxes + 6 * k;
        /* Chebyshev signed distance to the grown box: <= 0 means inside */
        double dist = -INFINITY;
        for (int a = 0; a < 3; ++a) {
            double lo = (double)bx[a] - margin, hi = (double)bx[3 + a] + margin;
            dist = fmax(dist, fmax(lo - x[a], x[a] - hi));
        }
        if (dist <= 0.0) invalid = 1;
        if (dist < -band) clear_violation = 1;
        else if (fabs(dist) <= band) { near = 1; fl |= ORA_FLAG_BOX; }
    }
    int amb = (!clear_violation && near) ? 1 : 0;
    if (amb && flags) *flags |= fl;
    return invalid | (amb << 1);
}

/* Region of a state (Alg. 2).  Reading: a uniform grid over the
 * workspace, grid[a] cells per position axis, clamped at the far faces,
 * row-major over (x, y, z); with sign bins, three bits (velocity >= 0) are
 * appended.  A coordinate within band of an interior face is ambiguous; there a
 * hinted index is adopted if it is one of the two adjacent indices. */
static int vel_index(int32_t dyn)
{
    return dyn == ORA_DI6 ? 3 : (dyn == ORA_QUAD12 ? 6 : -1);
}

int64_t ora_cell_of(const ora_problem* P, const double* x, const int64_t* hint, uint32_t* flags)
{
    int64_t hidx[3] = {-1, -1, -1};
    int64_t hbits = -1;
    if (hint && *hint >= 0) {
        int64_t c = *hint;
        if (P->vel_sign_bins) { hbits = c % 8; c /= 8; }
        hidx[2] = c % P->grid[2]; c /= P->grid[2];
        hidx[1] = c % P->grid[1]; c /= P->grid[1];
        hidx[0] = c;
    }
    int64_t idx[3];
    for (int a = 0; a < 3; ++a) {
        const double lo = P->ws_lo[a], hi = P->ws_hi[a];
        const int g = P->grid[a];
        double t = (double)g * (x[a] - lo) / (hi - lo);
        int64_t i = (int64_t)floor(t);
        if (i < 0) i = 0;
        if (i > g - 1) i = g - 1;
        double kf = nearbyint(t);
        if (kf >= 1.0 && kf <= (double)(g - 1)) {
            double face = lo + kf * (hi - lo) / (double)g;
            if (fabs(x[a] - face) <= P->band) {
                if (flags) *flags |= ORA_FLAG_CELL;
                int64_t k = (int64_t)kf;
                if (hidx[a] == k - 1 || hidx[a] == k) i = hidx[a];
            }
        }
        idx[a] = i;
    }
    int64_t cell = (idx[0] * P->grid[1] + idx[1]) * P->grid[2] + idx[2];
    if (P->vel_sign_bins) {
        int vi = vel_index(P->dynamics);
        int64_t bits = 0;
        for (int a = 0; a < 3; ++a) {
            int64_t b = x[vi + a] >= 0.0 ? 1 : 0;
            if (fabs(x[vi + a]) <= P->band) {
                if (flags) *flags |= ORA_FLAG_VSIGN;
                if (hbits >= 0) b = (hbits >> (2 - a)) & 1;
            }
            bits |= b << (2 - a);
        }
        cell = cell * 8 + bits;
    }
    return cell;
}

/* Goal set (Alg. 4).  Reading: a closed ball over the position
 * coordinates, tested at the end state of each edge. */
int ora_goal_test(const ora_problem* P, const double* x, double radius, const uint8_t* hint,
                  uint32_t* flags)
{
    double s = 0.0;
    for (int a = 0; a < 3; ++a) {
        double dlt = x[a] - (double)P->goal_center[a];
        s += dlt * dlt;
    }
    double dist = sqrt(s);
    int in = dist <= radius;
    if (fabs(dist - radius) <= P->band) {
        if (flags) *flags |= ORA_FLAG_GOAL;
        if (hint) in = *hint ? 1 : 0;
    }
    return in;
}

/* One expansion (Alg. 2): integrate n RK4 steps of size dt from x0
 * with the constant control u, testing validity after every step.
 * Reading: validity is checked at the substep end points x_1..x_n (x_0 is a
 * tree node and already valid) and integration stops at the first invalid
 * one.  hint_first_invalid < 0 means no hint. */
void ora_propagate_edge(const ora_problem* P, const double* x0, const float* u, int32_t n,
                        int32_t hint_first_invalid, ora_edge* out)
{
    const int d = ora_state_dim(P->dynamics);
    const int m = ora_control_dim(P->dynamics);
    double z[ORA_MAX_STATE + 1];
    double uu[ORA_MAX_CONTROL] = {0, 0, 0, 0};
    for (int i = 0; i < d; ++i) z[i] = x0[i];
    z[d] = 0.0;
    for (int i = 0; i < m; ++i) uu[i] = (double)u[i];
    const double h = (double)P->dt;
    out->first_invalid = 0;
    out->flags = 0;
    out->substeps = 0;
    for (int32_t k = 1; k <= n; ++k) {
        ora_rk4_step(P, z, uu, h);
        out->substeps = k;
        uint32_t fl = 0;
        int st = ora_point_status(P, z, (double)P->margin, P->band, &fl);
        int bad = st & 1;
        if (st & 2) {
            out->flags |= fl;
            if (hint_first_invalid >= 0) bad = (hint_first_invalid == k);
        }
        if (bad) {
            out->first_invalid = k;
            break;
        }
    }
    for (int i = 0; i < d; ++i) out->xn[i] = z[i];
    for (int i = d; i < ORA_MAX_STATE; ++i) out->xn[i] = 0.0;
    out->length = z[d];
}

/* ------------------------------------------------------------------------ */
/* App. A: exclusiveScan of a boolean mask and GraphSearch (Alg. 5),         */
/* I[S[tid]] = tid for every set tid.  The count of set entries is           */
/* S[n-1] + mask[n-1] (the last entry itself may be set).                    */
/* ------------------------------------------------------------------------ */
void ora_exclusive_scan(const uint8_t* mask, int64_t n, int64_t* S)
{
    int64_t acc = 0;
    for (int64_t i = 0; i < n; ++i) {
        S[i] = acc;
        acc += mask[i] ? 1 : 0;
    }
}

int64_t ora_graph_search(const uint8_t* mask, const int64_t* S, int64_t n, int64_t* I)
{
    for (int64_t tid = 0; tid < n; ++tid)
        if (mask[tid]) I[S[tid]] = tid;
    return n > 0 ? S[n - 1] + (mask[n - 1] ? 1 : 0) : 0;
}

/* ------------------------------------------------------------------------ */
/* Tree state                                                                */
/* ------------------------------------------------------------------------ */
static int64_t n_cells_of(const ora_problem* P)
{
    return (int64_t)P->grid[0] * P->grid[1] * P->grid[2] * (P->vel_sign_bins ? 8 : 1);
}

/* Candidate slots of one iteration at most: n_select * K, or, in the
 * uncapped form (samples_per_node = 0), the n_select slots that all active
 * nodes share (Sec. VI-A / App. A: lambda = floor(t_e / |V_A|), read with the
 * candidate buffer's size for t_e). */
static int64_t slots_max(const ora_problem* P)
{
    return (int64_t)P->n_select * (P->samples_per_node > 0 ? P->samples_per_node : 1);
}

/* Samples per node for a selection of n_sel nodes. */
static int64_t samples_for(const ora_problem* P, int64_t n_sel)
{
    if (P->samples_per_node > 0) return P->samples_per_node;
    if (n_sel <= 0) return 1;
    const int64_t k = P->n_select / n_sel;
    return k > 1 ? k : 1;
}

static int64_t survivors_bound(const ora_problem* P)
{
    int64_t slots = slots_max(P);
    int64_t cells = n_cells_of(P);
    return slots < cells ? slots : cells;
}

/* lexicographic (cost, id): equal costs are ordered by id (Reading: the
 * paper compares costs for equality; ties go to the lower id, so a tree node
 * beats this iteration's candidates and candidates are ordered by slot) */
static int key_less(double c1, int64_t i1, double c2, int64_t i2)
{
    if (c1 < c2) return 1;
    if (c1 > c2) return 0;
    return i1 < i2;
}

/* Initialisation of Alg. 1.  Reading: the root's region holds cost 0 and the root id,
 * so that the root counts as its region's best node. */
int ora_init(const ora_problem* P, ora_tree* T)
{
    const int d = ora_state_dim(P->dynamics);
    const int m = ora_control_dim(P->dynamics);
    if (d < 0 || m < 0) return ORA_ERR_ARG;
    if (P->cost != ORA_COST_TIME && P->cost != ORA_COST_PATH) return ORA_ERR_ARG;
    for (int a = 0; a < 3; ++a) {
        if (P->grid[a] < 1) return ORA_ERR_ARG;
        if (!(P->ws_lo[a] < P->ws_hi[a])) return ORA_ERR_ARG;
    }
    for (int i = 0; i < m; ++i)
        if (!(P->u_lo[i] <= P->u_hi[i])) return ORA_ERR_ARG;
    if (P->vel_sign_bins && vel_index(P->dynamics) < 0) return ORA_ERR_ARG;
    if (P->n_select < 1 || P->samples_per_node < 0) return ORA_ERR_ARG;
    if (P->steps_min < 1 || P->steps_max < P->steps_min) return ORA_ERR_ARG;
    if (!(P->dt > 0.0f) || !(P->margin >= 0.0f) || !(P->goal_radius > P->margin)) return ORA_ERR_ARG;
    if (P->n_boxes < 0 || (P->n_boxes > 0 && !P->boxes)) return ORA_ERR_ARG;
    if (T->cap < 1 + survivors_bound(P)) return ORA_ERR_ARG;
    if (T->n_cells != n_cells_of(P)) return ORA_ERR_ARG;

    double x0[ORA_MAX_STATE];
    for (int i = 0; i < ORA_MAX_STATE; ++i) x0[i] = i < d ? (double)P->x_init[i] : 0.0;
    if (ora_point_status(P, x0, (double)P->margin, 0.0, NULL) & 1) return ORA_ERR_INVALID_START;

    for (int64_t c = 0; c < T->n_cells; ++c) {
        T->tbl_cost[c] = INFINITY;
        T->tbl_id[c] = -1;
    }
    for (int i = 0; i < ORA_MAX_STATE; ++i) T->x[i] = x0[i];
    for (int i = 0; i < ORA_MAX_CONTROL; ++i) T->u[i] = 0.0f;
    T->steps[0] = 0;
    T->parent[0] = -1;
    T->cost[0] = 0.0;
    T->cell[0] = ora_cell_of(P, x0, NULL, NULL);
    T->status[0] = ORA_ACTIVE;
    T->icount[0] = 0;
    T->tbl_cost[T->cell[0]] = 0.0;
    T->tbl_id[T->cell[0]] = 0;
    T->n_tree = 1;
    T->cursor = 0;
    T->iter = 0;
    T->sol_cost = INFINITY;
    T->sol_id = -1;
    T->first_sol_iter = -1;
    /* Reading: a root that already lies in the goal set is a solution of cost
     * 0 (the empty trajectory), found before the first iteration.  Alg. 4
     * otherwise tests only the nodes it inserts. */
    if (ora_goal_test(P, x0, (double)P->goal_radius - (double)P->margin, NULL, NULL)) {
        T->sol_cost = 0.0;
        T->sol_id = 0;
        T->first_sol_iter = 0;
    }
    T->full = 0;
    T->last_n_sel = T->last_n_valid = T->last_n_surv = 0;
    return ORA_OK;
}

/* Which nodes of V_A are expanded this iteration.  Reading: at most n_select
 * nodes are expanded; V_A is ordered by region index rotated to start at the
 * cursor region and the first n_select are taken; the cursor moves past the
 * last one taken.  Every active node is therefore expanded again within a
 * bounded number of iterations (Thm. 1 needs every region-best node to be
 * selected infinitely often). */
typedef struct {
    int64_t rot, idx;
} ora_rank;

static int cmp_rank(const void* a, const void* b)
{
    const ora_rank* x = (const ora_rank*)a;
    const ora_rank* y = (const ora_rank*)b;
    if (x->rot != y->rot) return x->rot < y->rot ? -1 : 1;
    if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
    return 0;
}

int64_t ora_select(const ora_problem* P, const ora_tree* T, int64_t* sel, int64_t* cursor_next)
{
    int64_t n_active = 0;
    for (int64_t i = 0; i < T->n_tree; ++i)
        if (T->status[i] == ORA_ACTIVE) ++n_active;
    ora_rank* r = (ora_rank*)malloc(sizeof(ora_rank) * (size_t)(n_active > 0 ? n_active : 1));
    int64_t k = 0;
    for (int64_t i = 0; i < T->n_tree; ++i) {
        if (T->status[i] != ORA_ACTIVE) continue;
        int64_t rot = T->cell[i] - T->cursor;
        if (rot < 0) rot += T->n_cells;
        r[k].rot = rot;
        r[k].idx = i;
        ++k;
    }
    qsort(r, (size_t)n_active, sizeof(ora_rank), cmp_rank);
    int64_t n_sel = n_active < P->n_select ? n_active : P->n_select;
    for (int64_t j = 0; j < n_sel; ++j) sel[j] = r[j].idx;
    *cursor_next = T->cursor;
    if (n_sel > 0) *cursor_next = (T->cell[sel[n_sel - 1]] + 1) % T->n_cells;
    free(r);
    return n_sel;
}

/* Whether node i holds its region's minimum: the region's (cost, id) entry
 * names i itself (ties by id, see key_less). */
static int region_best(const ora_tree* T, int64_t i)
{
    return T->tbl_id[T->cell[i]] == i;
}

/* Whether some proper ancestor of node i does not hold its region's minimum.
 * It depends on the table and the parent links only. */
static int ancestor_beaten(const ora_tree* T, int64_t i)
{
    for (int64_t p = T->parent[i]; p >= 0; p = T->parent[p])
        if (!region_best(T, p)) return 1;
    return 0;
}

/* PruneNodes (Alg. 3) over the node sets of Sec. IV-A, node by node.  With
 * best = region_best(i), the dormancy count c = icount(i) and I_max:
 *
 *   status    best  count                   ancestor beaten  ->  status, count
 *   any       no    -                       -                ->  TERMINAL
 *   INACTIVE  yes   c + 1 > I_max           -                ->  ACTIVE, c + 1
 *   INACTIVE  yes   c + 1 <= I_max          -                ->  INACTIVE, c + 1
 *   ACTIVE    yes   c > I_max (woken once)  -                ->  ACTIVE
 *   ACTIVE    yes   c <= I_max              yes              ->  INACTIVE
 *   ACTIVE    yes   c <= I_max              no               ->  ACTIVE
 *
 * A dormant node that holds its region counts iterations and wakes past
 * I_max; a woken node is never made dormant again; a node that lost its region
 * leaves the tree's live sets for good.  Terminal nodes fall in the first row,
 * since a key that was beaten never becomes a region's minimum again. */
void ora_prune(const ora_problem* P, ora_tree* T)
{
    for (int64_t i = 0; i < T->n_tree; ++i) {
        if (!region_best(T, i)) {
            T->status[i] = ORA_TERMINAL;
            continue;
        }
        switch (T->status[i]) {
        case ORA_INACTIVE:
            T->icount[i] += 1;
            if (T->icount[i] > P->i_max) T->status[i] = ORA_ACTIVE;
            break;
        case ORA_ACTIVE:
            if (T->icount[i] <= P->i_max && ancestor_beaten(T, i)) T->status[i] = ORA_INACTIVE;
            break;
        default:
            break;
        }
    }
}

static int near_tie(double a, double b, double rel)
{
    double s = fmax(fabs(a), fabs(b));
    return fabs(a - b) <= rel * s;
}

/* Edge polish of one inserted node i (an extension, not in the paper): the
 * node's control u takes `polish_steps` projected gradient steps
 *   u <- clamp(u - lr grad L(u, u, u, u), U)
 * on the tied loss of kpx_oracle_diff.h (complex-step gradient) over the
 * margin-grown boxes, towards the goal centre, with the path length weighted
 * by polish_w_len.  The polished edge replaces the node's edge when the
 * planner's own propagation finds it valid, it ends in the node's region, a
 * goal node stays in the goal, and, for the path-length cost, it is shorter;
 * a node that enters the goal competes for the solution.  For the TIME cost
 * the node's cost (the step count) does not change; for the path-length cost
 * the shorter edge's cost (parent cost + length, Assumption 1) replaces it,
 * and the region's cost with it (the node has no descendants yet and keeps its
 * region).  The other side's decisions of the polished edge are passed per
 * test: its first invalid step (negative: none given), the region and the goal
 * bit of its end state, and its accept bit for the length comparison; each is
 * adopted only where the oracle's own decision of that same test lies within
 * band, as for any propagated edge.  Returns 1 when the polished edge replaced
 * the node's edge. */
static int polish_node(const ora_problem* P, ora_tree* T, int64_t i, int was_goal, const float* grown,
                       int32_t hint_fi, const int64_t* hint_cell, const uint8_t* hint_goal,
                       const uint8_t* hint_acc)
{
    orad_problem D;
    memset(&D, 0, sizeof(D));
    D.mass = P->dyn_params[0];
    D.jx = P->dyn_params[1];
    D.jy = P->dyn_params[2];
    D.jz = P->dyn_params[3];
    D.grav = P->dyn_params[4];
    D.dt = P->dt;
    D.boxes = grown;
    D.n_boxes = P->n_boxes;
    for (int a = 0; a < 3; ++a) D.goal[a] = P->goal_center[a];
    D.w_ctrl = P->polish_w_ctrl;
    D.w_obst = P->polish_w_obst;
    D.k_obst = P->polish_k_obst;
    D.d_safe = P->polish_d_safe;
    D.w_goal = P->polish_w_goal;
    D.w_len = P->polish_w_len;
    const double* x0 = &T->x[T->parent[i] * ORA_MAX_STATE];
    const int32_t n = T->steps[i];
    double u[4];
    for (int c = 0; c < 4; ++c) u[c] = (double)T->u[i * ORA_MAX_CONTROL + c];
    for (int r = 0; r < P->polish_steps; ++r) {
        double u16[16], g[4];
        for (int j = 0; j < 4; ++j)
            for (int c = 0; c < 4; ++c) u16[4 * j + c] = u[c];
        orad_grad_tied(&D, x0, u16, n, 1e-20, g);
        for (int c = 0; c < 4; ++c) {
            const double v = u[c] - P->polish_lr * g[c];
            u[c] = v < (double)P->u_lo[c] ? (double)P->u_lo[c] : v > (double)P->u_hi[c] ? (double)P->u_hi[c] : v;
        }
    }
    float uf[ORA_MAX_CONTROL];
    for (int c = 0; c < 4; ++c) uf[c] = (float)u[c];
    ora_edge e;
    ora_propagate_edge(P, x0, uf, n, hint_fi, &e);
    if (e.first_invalid != 0) return 0;
    const int64_t cell = ora_cell_of(P, e.xn, hint_cell, NULL);
    const int goal_now = ora_goal_test(P, e.xn, (double)P->goal_radius - (double)P->margin, hint_goal, NULL);
    if (cell != T->cell[i] || (was_goal && !goal_now)) return 0;
    if (P->cost == ORA_COST_PATH) {
        const double c_new = T->cost[T->parent[i]] + e.length;
        int shorter = c_new < T->cost[i];
        if (hint_acc && near_tie(c_new, T->cost[i], P->band)) shorter = *hint_acc != 0;
        if (!shorter) return 0;
        T->cost[i] = c_new;
        T->tbl_cost[T->cell[i]] = c_new;
    }
    for (int k = 0; k < ORA_MAX_STATE; ++k) T->x[i * ORA_MAX_STATE + k] = e.xn[k];
    for (int c = 0; c < 4; ++c) T->u[i * ORA_MAX_CONTROL + c] = uf[c];
    if (goal_now && key_less(T->cost[i], i, T->sol_cost, T->sol_id)) {
        if (T->sol_id < 0) T->first_sol_iter = T->iter;
        T->sol_cost = T->cost[i];
        T->sol_id = i;
    }
    return 1;
}

/* One iteration of Alg. 1: Propagate, PruneNodes, UpdateTree.
 * Reading: before anything else, if n_tree plus the most survivors one
 * iteration can add exceeds the capacity, nothing is done and ORA_FULL is
 * returned (the paper only notes that overflowing t_e would fault). */
int ora_step(const ora_problem* P, ora_tree* T, ora_cands* C, const ora_hints* H)
{
    const int d = ora_state_dim(P->dynamics);
    const int m = ora_control_dim(P->dynamics);
    if (T->full || T->n_tree + survivors_bound(P) > T->cap) {
        T->full = 1;
        C->n_slots = 0;
        C->k = 0;
        return ORA_FULL;
    }
    if (C->cap_slots < slots_max(P)) return ORA_ERR_ARG;
    const int64_t n_tree = T->n_tree;

    /* which nodes of V_A are expanded */
    int64_t* sel = (int64_t*)malloc(sizeof(int64_t) * (size_t)P->n_select);
    int64_t cursor_next = T->cursor;
    const int64_t n_sel = ora_select(P, T, sel, &cursor_next);
    const int64_t K = samples_for(P, n_sel);
    const int64_t n_slots = n_sel * K;
    C->n_slots = n_slots;
    C->k = K;
    C->substeps_total = 0;

    /* Alg. 2: each of the K expansions of each selected node.  The
     * expansions are independent; a build with OpenMP (the CPU timing
     * baseline only) shares them among threads, with the same results. */
    int64_t n_valid = 0, substeps_total = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : n_valid, substeps_total)
    for (int64_t s = 0; s < n_slots; ++s) {
        const int64_t par = sel[s / K];
        float u[ORA_MAX_CONTROL];
        int32_t n;
        ora_sample(P, (uint32_t)T->iter, (uint32_t)s, u, &n);
        C->parent[s] = par;
        for (int i = 0; i < ORA_MAX_CONTROL; ++i) C->u[s * ORA_MAX_CONTROL + i] = u[i];
        C->n[s] = n;
        ora_edge e;
        const int32_t hint_fi = (H && H->first_invalid) ? H->first_invalid[s] : -1;
        ora_propagate_edge(P, &T->x[par * ORA_MAX_STATE], u, n, hint_fi, &e);
        C->substeps[s] = e.substeps;
        substeps_total += e.substeps;
        C->first_invalid[s] = e.first_invalid;
        C->flags[s] = e.flags;
        C->valid[s] = e.first_invalid == 0;
        for (int i = 0; i < ORA_MAX_STATE; ++i) C->xn[s * ORA_MAX_STATE + i] = e.xn[i];
        C->survivor[s] = 0;
        C->new_index[s] = -1;
        C->goal[s] = 0;
        C->cell[s] = -1;
        C->cost[s] = INFINITY;
        if (!C->valid[s]) continue;
        ++n_valid;
        uint32_t fl = 0;
        C->cell[s] = ora_cell_of(P, e.xn, (H && H->cell) ? &H->cell[s] : NULL, &fl);
        /* Alg. 2: additive cost; TIME counts steps, PATH adds length */
        const double edge_cost = P->cost == ORA_COST_TIME ? (double)n : e.length;
        C->cost[s] = T->cost[par] + edge_cost;
        C->goal[s] = (uint8_t)ora_goal_test(P, e.xn, (double)P->goal_radius - (double)P->margin,
                                            (H && H->goal) ? &H->goal[s] : NULL, &fl);
        C->flags[s] |= fl;
    }
    C->substeps_total = substeps_total;

    /* Alg. 2: region minimum over this iteration's arrivals; the
     * arrival id of slot s is n_tree + s */
    double* old_cost = (double*)malloc(sizeof(double) * (size_t)T->n_cells);
    int64_t* old_id = (int64_t*)malloc(sizeof(int64_t) * (size_t)T->n_cells);
    memcpy(old_cost, T->tbl_cost, sizeof(double) * (size_t)T->n_cells);
    memcpy(old_id, T->tbl_id, sizeof(int64_t) * (size_t)T->n_cells);
    for (int64_t s = 0; s < n_slots; ++s) {
        if (!C->valid[s]) continue;
        const int64_t c = C->cell[s];
        if (key_less(C->cost[s], n_tree + s, T->tbl_cost[c], T->tbl_id[c])) {
            T->tbl_cost[c] = C->cost[s];
            T->tbl_id[c] = n_tree + s;
        }
    }
    if (P->cost == ORA_COST_PATH) {
        /* path lengths are real numbers: a rival within the relative band of
         * the minimum makes the region's winner ambiguous */
        uint8_t* amb = (uint8_t*)calloc((size_t)T->n_cells, 1);
        for (int64_t s = 0; s < n_slots; ++s) {
            if (!C->valid[s]) continue;
            const int64_t c = C->cell[s];
            if (T->tbl_id[c] != n_tree + s && near_tie(C->cost[s], T->tbl_cost[c], P->band))
                amb[c] = 1;
        }
        for (int64_t c = 0; c < T->n_cells; ++c)
            if (old_id[c] >= 0 && old_id[c] != T->tbl_id[c] &&
                near_tie(old_cost[c], T->tbl_cost[c], P->band))
                amb[c] = 1;
        for (int64_t s = 0; s < n_slots; ++s)
            if (C->valid[s] && amb[C->cell[s]] && near_tie(C->cost[s], T->tbl_cost[C->cell[s]], P->band))
                C->flags[s] |= ORA_FLAG_TIE;
        if (H && H->survivor) {
            for (int64_t c = 0; c < T->n_cells; ++c) {
                if (!amb[c]) continue;
                int64_t pick = -1;
                for (int64_t s = 0; s < n_slots; ++s)
                    if (C->valid[s] && C->cell[s] == c && H->survivor[s]) pick = s;
                if (pick >= 0 && near_tie(C->cost[pick], T->tbl_cost[c], P->band)) {
                    T->tbl_cost[c] = C->cost[pick];
                    T->tbl_id[c] = n_tree + pick;
                } else if (pick < 0 && old_id[c] >= 0 && near_tie(old_cost[c], T->tbl_cost[c], P->band)) {
                    T->tbl_cost[c] = old_cost[c];
                    T->tbl_id[c] = old_id[c];
                }
            }
        }
        free(amb);
    }
    free(old_cost);
    free(old_id);

    /* Alg. 3 against the updated regions */
    ora_prune(P, T);

    /* Alg. 4 + App. A: V_U = arrivals still holding their region minimum;
     * exclusive scan + GraphSearch give each its place |T| + rank */
    uint8_t* mask = (uint8_t*)calloc((size_t)(n_slots > 0 ? n_slots : 1), 1);
    int64_t* S = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_slots > 0 ? n_slots : 1));
    int64_t* I = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_slots > 0 ? n_slots : 1));
    for (int64_t s = 0; s < n_slots; ++s)
        mask[s] = C->valid[s] && T->tbl_id[C->cell[s]] == n_tree + s;
    ora_exclusive_scan(mask, n_slots, S);
    const int64_t n_surv = ora_graph_search(mask, S, n_slots, I);
    for (int64_t t = 0; t < n_surv; ++t) {
        const int64_t s = I[t];
        const int64_t i = n_tree + t;
        for (int k = 0; k < ORA_MAX_STATE; ++k) T->x[i * ORA_MAX_STATE + k] = k < d ? C->xn[s * ORA_MAX_STATE + k] : 0.0;
        for (int k = 0; k < ORA_MAX_CONTROL; ++k) T->u[i * ORA_MAX_CONTROL + k] = k < m ? C->u[s * ORA_MAX_CONTROL + k] : 0.0f;
        T->steps[i] = C->n[s];
        T->parent[i] = C->parent[s];
        T->cost[i] = C->cost[s];
        T->cell[i] = C->cell[s];
        T->status[i] = ORA_ACTIVE;
        T->icount[i] = 0;
        T->tbl_id[C->cell[s]] = i;
        C->survivor[s] = 1;
        C->new_index[s] = i;
        /* Alg. 4: a goal node that beats the solution replaces it */
        if (C->goal[s] && key_less(C->cost[s], i, T->sol_cost, T->sol_id)) {
            if (T->sol_id < 0) T->first_sol_iter = T->iter;
            T->sol_cost = C->cost[s];
            T->sol_id = i;
        }
    }
    if (P->polish_steps > 0 && P->dynamics == ORA_QUAD12) {
        float* grown = (float*)malloc(sizeof(float) * 6 * (size_t)(P->n_boxes > 0 ? P->n_boxes : 1));
        for (int32_t b = 0; b < P->n_boxes; ++b)
            for (int a = 0; a < 3; ++a) {
                grown[6 * b + a] = P->boxes[6 * b + a] - P->margin;
                grown[6 * b + 3 + a] = P->boxes[6 * b + 3 + a] + P->margin;
            }
        for (int64_t t = 0; t < n_surv; ++t) {
            const int32_t hfi = (H && H->polish_first_invalid) ? H->polish_first_invalid[t] : -1;
            const int64_t* hc = (H && H->polish_cell) ? &H->polish_cell[t] : NULL;
            const uint8_t* hg = (H && H->polish_goal) ? &H->polish_goal[t] : NULL;
            const uint8_t* ha = (H && H->polish_accepted) ? &H->polish_accepted[t] : NULL;
            /* the goal-only form leaves every node outside the goal set as inserted */
            const int acc = (P->polish_goal_only && !C->goal[I[t]])
                                ? 0
                                : polish_node(P, T, n_tree + t, C->goal[I[t]], grown, hfi, hc, hg, ha);
            if (C->polished) C->polished[t] = (uint8_t)acc;
        }
        free(grown);
    }
    T->n_tree = n_tree + n_surv;
    T->cursor = cursor_next;
    T->last_n_sel = n_sel;
    T->last_n_valid = n_valid;
    T->last_n_surv = n_surv;
    T->iter += 1;
    free(mask);
    free(S);
    free(I);
    free(sel);
    return ORA_OK;
}

/* Adaptive decomposition (the remark on non-uniform and adaptive
 * decompositions, Sec. IV; their analysis is deferred there).  Reading: the
 * grid is divided by an integer factor per axis between iterations; live
 * nodes (not terminal) are unique per old region and so per new region, and
 * each owns its new region; terminal nodes stay terminal; the cursor moves
 * to the first new cell of its old one, and the next selection is made over
 * the refined regions from there. */
int ora_refine(const ora_problem* P, ora_tree* T, int32_t factor, const int64_t* hint_cell)
{
    if (factor < 2) return ORA_ERR_ARG;
    const int64_t nc = n_cells_of(P);
    T->n_cells = nc;
    for (int64_t c = 0; c < nc; ++c) {
        T->tbl_cost[c] = INFINITY;
        T->tbl_id[c] = -1;
    }
    for (int64_t i = 0; i < T->n_tree; ++i) {
        const int64_t c = ora_cell_of(P, &T->x[i * ORA_MAX_STATE], hint_cell ? &hint_cell[i] : NULL, NULL);
        T->cell[i] = c;
        if (T->status[i] != ORA_TERMINAL && key_less(T->cost[i], i, T->tbl_cost[c], T->tbl_id[c])) {
            T->tbl_cost[c] = T->cost[i];
            T->tbl_id[c] = i;
        }
    }
    /* cursor: old region -> its first cell in the refined grid */
    int64_t c = T->cursor, bits = 0;
    if (P->vel_sign_bins) {
        bits = c % 8;
        c /= 8;
    }
    const int64_t og1 = P->grid[1] / factor, og2 = P->grid[2] / factor;
    const int64_t iz = c % og2, iy = (c / og2) % og1, ix = c / (og2 * og1);
    const int64_t s2 = ((ix * factor) * P->grid[1] + iy * factor) * P->grid[2] + iz * factor;
    T->cursor = P->vel_sign_bins ? s2 * 8 + bits : s2;
    if (T->n_tree + survivors_bound(P) > T->cap) T->full = 1;
    return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* Trajectory check: re-integrate the controls open loop from x_init in      */
/* float64, test every substep against the exact valid set (no margin),      */
/* test the end state against the exact goal ball and recompute the cost     */
/* (additivity, Assumption 1).                                               */
/* ------------------------------------------------------------------------ */
int ora_verify(const ora_problem* P, int32_t n_edges, const float* controls, const int32_t* steps,
               const float* states, double reported_cost, ora_verify_report* rep)
{
    const int d = ora_state_dim(P->dynamics);
    const int m = ora_control_dim(P->dynamics);
    memset(rep, 0, sizeof(*rep));
    rep->first_bad_edge = -1;
    rep->first_bad_substep = -1;
    rep->min_clearance = INFINITY;
    rep->collision_free = 1;
    rep->within_bounds = 1;
    rep->starts_at_init = 1;
    if (states)
        for (int i = 0; i < d; ++i)
            if (states[i] != P->x_init[i]) rep->starts_at_init = 0;
    double z[ORA_MAX_STATE + 1];
    for (int i = 0; i < d; ++i) z[i] = (double)P->x_init[i];
    z[d] = 0.0;
    const double h = (double)P->dt;
    double total_steps = 0.0, length = 0.0;
    for (int32_t e = 0; e < n_edges; ++e) {
        double uu[ORA_MAX_CONTROL] = {0, 0, 0, 0};
        for (int i = 0; i < m; ++i) uu[i] = (double)controls[e * ORA_MAX_CONTROL + i];
        z[d] = 0.0;
        for (int32_t k = 1; k <= steps[e]; ++k) {
            ora_rk4_step(P, z, uu, h);
            for (int b = 0; b < P->n_boxes; ++b) {
                const float* bx = P->boxes + 6 * b;
                double dist = -INFINITY;
                for (int a = 0; a < 3; ++a)
                    dist = fmax(dist, fmax((double)bx[a] - z[a], z[a] - (double)bx[3 + a]));
                if (dist < rep->min_clearance) rep->min_clearance = dist;
                if (dist <= 0.0 && rep->collision_free) {
                    rep->collision_free = 0;
                    if (rep->first_bad_edge < 0) { rep->first_bad_edge = e; rep->first_bad_substep = k; }
                }
            }
            uint32_t fl = 0;
            /* bounds and workspace with margin 0: bit 0 covers them together
             * with the boxes, so test the non-box part on its own */
            ora_problem Q = *P;
            Q.n_boxes = 0;
            if (ora_point_status(&Q, z, 0.0, 0.0, &fl) & 1) {
                if (rep->within_bounds && rep->first_bad_edge < 0) {
                    rep->first_bad_edge = e;
                    rep->first_bad_substep = k;
                }
                rep->within_bounds = 0;
            }
        }
        total_steps += steps[e];
        length += z[d];
        if (states) {
            for (int i = 0; i < d; ++i) {
                double gap = fabs(z[i] - (double)states[(e + 1) * ORA_MAX_STATE + i]);
                if (gap > rep->max_gap) rep->max_gap = gap;
            }
        }
    }
    double s = 0.0;
    for (int a = 0; a < 3; ++a) {
        double dlt = z[a] - (double)P->goal_center[a];
        s += dlt * dlt;
    }
    rep->goal_distance = sqrt(s);
    /* an empty plan reaches the goal only when the start lies in it */
    rep->reaches_goal = rep->goal_distance <= (double)P->goal_radius;
    if (P->cost == ORA_COST_TIME) {
        rep->cost = total_steps;
        rep->cost_ok = reported_cost == total_steps;
    } else {
        rep->cost = length;
        rep->cost_ok = fabs(reported_cost - length) <= 1e-4 * fmax(1.0, fabs(length));
    }
    rep->ok = rep->starts_at_init && rep->collision_free && rep->within_bounds &&
              rep->reaches_goal && rep->cost_ok;
    return rep->ok ? ORA_OK : ORA_ERR_ARG;
}
