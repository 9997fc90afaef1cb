/*
 * kpx_oracle_diff.c -- float64 reference of the differentiable edge rollout.
 * TEST INFRASTRUCTURE: loaded only by tests/ and bench.py's baseline leg.
 *
 * The forward model is written once over complex numbers: every branch (the
 * nearest box, the box's outside/inside form, the axis of a max, the stable
 * form of softplus) is decided on real parts, so that with a zero imaginary
 * part it is the plain float64 loss, and with an imaginary step h e_j it
 * carries dL/du_j * h in its imaginary part (the complex-step derivative).
 */
#include "kpx_oracle_diff.h"

#include <complex.h>
#include <math.h>
#include <string.h>

typedef double complex cplx;

int32_t orad_segment(int32_t k, int32_t n)
{
    int32_t j = 0;
    while (j < 3 && k >= ((j + 1) * n) / 4) ++j;
    return j;
}

/* 12D quadrotor: position, ZYX Euler angles, world-frame velocity, body rates;
 * control: thrust and body torques (the planner's model). */
static void deriv(const orad_problem* D, const cplx* z, const cplx* u, cplx* zd)
{
    const cplx sphi = csin(z[3]), cphi = ccos(z[3]);
    const cplx sth = csin(z[4]), cth = ccos(z[4]);
    const cplx spsi = csin(z[5]), cpsi = ccos(z[5]);
    const cplx wp = z[9], wq = z[10], wr = z[11];
    zd[0] = z[6];
    zd[1] = z[7];
    zd[2] = z[8];
    zd[3] = wp + (sphi * wq + cphi * wr) * (sth / cth);
    zd[4] = cphi * wq - sphi * wr;
    zd[5] = (sphi * wq + cphi * wr) / cth;
    const cplx acc = u[0] / D->mass;
    zd[6] = acc * (cpsi * sth * cphi + spsi * sphi);
    zd[7] = acc * (spsi * sth * cphi - cpsi * sphi);
    zd[8] = acc * (cth * cphi) - D->grav;
    zd[9] = (u[1] - (D->jz - D->jy) * wq * wr) / D->jx;
    zd[10] = (u[2] - (D->jx - D->jz) * wp * wr) / D->jy;
    zd[11] = (u[3] - (D->jy - D->jx) * wp * wq) / D->jz;
}

/* speed |v| of a state (the rate of the path length) */
static cplx speed(const cplx* z)
{
    return csqrt(z[6] * z[6] + z[7] * z[7] + z[8] * z[8]);
}

/* classical RK4 step of size h; the path length *ell (when not NULL) is one
 * more component of the step, with rate |v| */
static void rk4(const orad_problem* D, cplx* z, const cplx* u, double h, cplx* ell)
{
    cplx k1[12], k2[12], k3[12], k4[12], t[12], s1, s2, s3, s4;
    deriv(D, z, u, k1);
    s1 = speed(z);
    for (int i = 0; i < 12; ++i) t[i] = z[i] + 0.5 * h * k1[i];
    deriv(D, t, u, k2);
    s2 = speed(t);
    for (int i = 0; i < 12; ++i) t[i] = z[i] + 0.5 * h * k2[i];
    deriv(D, t, u, k3);
    s3 = speed(t);
    for (int i = 0; i < 12; ++i) t[i] = z[i] + h * k3[i];
    deriv(D, t, u, k4);
    s4 = speed(t);
    for (int i = 0; i < 12; ++i) z[i] += h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    if (ell) *ell += h / 6.0 * (s1 + 2.0 * s2 + 2.0 * s3 + s4);
}

static cplx box_sd(const float* b, const cplx* p)
{
    cplx q[3];
    for (int a = 0; a < 3; ++a) {
        const cplx below = (double)b[a] - p[a], above = p[a] - (double)b[3 + a];
        q[a] = creal(below) >= creal(above) ? below : above;
    }
    cplx out2 = 0.0;
    int outside = 0;
    for (int a = 0; a < 3; ++a)
        if (creal(q[a]) > 0.0) {
            out2 += q[a] * q[a];
            outside = 1;
        }
    if (outside) return csqrt(out2);
    cplx m = q[0];
    for (int a = 1; a < 3; ++a)
        if (creal(q[a]) > creal(m)) m = q[a];
    return m;
}

double orad_box_sd(const float* b, const double* p)
{
    const cplx pc[3] = {p[0], p[1], p[2]};
    return creal(box_sd(b, pc));
}

/* signed distance to the nearest box (by real part); +inf without boxes */
static cplx nearest_sd(const orad_problem* D, const cplx* p)
{
    cplx best = INFINITY;
    for (int b = 0; b < D->n_boxes; ++b) {
        const cplx s = box_sd(D->boxes + 6 * b, p);
        if (creal(s) < creal(best)) best = s;
    }
    return best;
}

static cplx softplus(cplx z)
{
    return creal(z) > 0.0 ? z + clog(1.0 + cexp(-z)) : clog(1.0 + cexp(z));
}

static cplx loss_c(const orad_problem* D, const double* x0, const cplx* u, int32_t n, double* states)
{
    cplx z[12];
    for (int i = 0; i < 12; ++i) z[i] = x0[i];
    if (states)
        for (int i = 0; i < 12; ++i) states[i] = x0[i];
    cplx L = n * D->dt, ell = 0.0;
    for (int i = 0; i < 16; ++i) L += D->w_ctrl * u[i] * u[i];
    for (int32_t k = 0; k < n; ++k) {
        rk4(D, z, u + 4 * orad_segment(k, n), D->dt, &ell);
        if (states)
            for (int i = 0; i < 12; ++i) states[(k + 1) * 12 + i] = creal(z[i]);
        if (D->n_boxes > 0 && D->w_obst != 0.0)
            L += D->w_obst * softplus(D->k_obst * (D->d_safe - nearest_sd(D, z)));
    }
    for (int a = 0; a < 3; ++a) {
        const cplx e = z[a] - D->goal[a];
        L += D->w_goal * e * e;
    }
    return L + D->w_len * ell;
}

double orad_loss(const orad_problem* D, const double* x0, const double* u, int32_t n, double* states)
{
    cplx uc[16];
    for (int i = 0; i < 16; ++i) uc[i] = u[i];
    return creal(loss_c(D, x0, uc, n, states));
}

void orad_grad(const orad_problem* D, const double* x0, const double* u, int32_t n, double h, double* grad)
{
    for (int j = 0; j < 16; ++j) {
        cplx uc[16];
        for (int i = 0; i < 16; ++i) uc[i] = u[i];
        uc[j] += I * h;
        grad[j] = cimag(loss_c(D, x0, uc, n, NULL)) / h;
    }
}

void orad_grad_tied(const orad_problem* D, const double* x0, const double* u, int32_t n, double h,
                    double* grad)
{
    for (int c = 0; c < 4; ++c) {
        cplx uc[16];
        for (int i = 0; i < 16; ++i) uc[i] = u[i];
        for (int j = 0; j < 4; ++j) uc[4 * j + c] += I * h;
        grad[c] = cimag(loss_c(D, x0, uc, n, NULL)) / h;
    }
}

int32_t orad_first_invalid(const orad_problem* D, const double* x0, const double* u, int32_t n,
                           const double* x_lo, const double* x_hi, const double* ws_lo,
                           const double* ws_hi)
{
    cplx z[12], uc[16];
    for (int i = 0; i < 12; ++i) z[i] = x0[i];
    for (int i = 0; i < 16; ++i) uc[i] = u[i];
    for (int32_t k = 0; k < n; ++k) {
        rk4(D, z, uc + 4 * orad_segment(k, n), D->dt, NULL);
        double x[12];
        for (int i = 0; i < 12; ++i) x[i] = creal(z[i]);
        for (int i = 0; i < 12; ++i)
            if (!(x[i] >= x_lo[i] && x[i] <= x_hi[i])) return k + 1;
        for (int a = 0; a < 3; ++a)
            if (!(x[a] >= ws_lo[a] && x[a] <= ws_hi[a])) return k + 1;
        for (int b = 0; b < D->n_boxes; ++b) {
            const float* bx = D->boxes + 6 * b;
            int in = 1;
            for (int a = 0; a < 3; ++a) in &= x[a] >= bx[a] && x[a] <= bx[3 + a];
            if (in) return k + 1;
        }
    }
    return 0;
}
