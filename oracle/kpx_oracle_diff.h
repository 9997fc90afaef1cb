/*
 * kpx_oracle_diff.h -- float64 reference of the differentiable edge rollout
 * (TEST INFRASTRUCTURE: loaded only by tests/ and bench.py's baseline leg).
 *
 * An edge of the 12D quadrotor (the dynamics of the planner, Sec. V) is n RK4
 * steps of size dt from x0 under 4 piecewise-constant control segments: step k
 * (0-based) uses segment j with floor(j n / 4) <= k < floor((j + 1) n / 4).
 * Its loss is
 *   n dt + w_ctrl * sum u^2
 *        + w_obst * sum_{k=1..n} softplus(k_obst * (d_safe - sd(p_k)))
 *        + w_goal * |p_n - goal|^2 + w_len * l,
 * sd = signed distance of the position to the nearest box (negative inside),
 * l = length of the position path, the speed |v| integrated as one more
 * component of the same RK4 steps (the planner's path-length cost).
 * The gradient with respect to the 16 controls is taken by the complex step,
 * Im L(u + i h e_j) / h, which has no cancellation error.
 */
#ifndef KPX_ORACLE_DIFF_H
#define KPX_ORACLE_DIFF_H

#include <stdint.h>

typedef struct {
    double mass, jx, jy, jz, grav;
    double dt;
    const float* boxes;  /* n_boxes x 6: lo x y z, hi x y z */
    int32_t n_boxes;
    double goal[3];
    double w_ctrl, w_obst, k_obst, d_safe, w_goal;
    double w_len;        /* weight of the path length */
} orad_problem;

/* Control segment of step k of an n-step edge. */
int32_t orad_segment(int32_t k, int32_t n);

/* Signed distance of p to the closed box b (lo, hi): |max(q, 0)| +
 * min(max_a q_a, 0) with q_a = max(lo_a - p_a, p_a - hi_a). */
double orad_box_sd(const float* b, const double* p);

/* Loss of one edge; states (optional, (n + 1) x 12) receives x_0 .. x_n. */
double orad_loss(const orad_problem* D, const double* x0, const double* u, int32_t n, double* states);

/* Complex-step gradient of orad_loss with respect to the 16 controls. */
void orad_grad(const orad_problem* D, const double* x0, const double* u, int32_t n, double h, double* grad);

/* Complex-step gradient of orad_loss with the 4 segments tied to one control
 * (u has 16 entries, all segments equal): perturbing control c of every
 * segment at once gives dL/du_c of the tied loss L(u, u, u, u) (4 values). */
void orad_grad_tied(const orad_problem* D, const double* x0, const double* u, int32_t n, double h,
                    double* grad);

/* First step (1..n) whose state leaves the valid set: a position inside a
 * closed box or outside the closed workspace, or a state outside the closed
 * bounds; 0 when every state x_1 .. x_n is valid. */
int32_t orad_first_invalid(const orad_problem* D, const double* x0, const double* u, int32_t n,
                           const double* x_lo, const double* x_hi, const double* ws_lo,
                           const double* ws_hi);

#endif
