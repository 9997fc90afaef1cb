// kpx_diff_device.hpp -- device half of the differentiable quadrotor edge
// rollout, shared by the batch call (kpx_diff.hip) and the planner's edge
// polish (kpx.hip): the 12D quadrotor of Sec. V in radians, its RK4 step and
// the adjoint of that step, the nearest-box signed distance, the smooth
// obstacle penalty, and one forward (+ adjoint) pass over an edge.
//
// An edge is n RK4 steps of size dt from x0 under 4 piecewise-constant
// control segments; step k uses segment j with floor(j n / 4) <= k <
// floor((j + 1) n / 4).  Its loss
//   n dt + w_ctrl |u|^2 + w_obst sum_{k=1..n} softplus(k_obst (d_safe - sd(p_k)))
//        + w_goal |p_n - goal|^2 + w_len l
// adds to the edge's duration a control effort, a smooth obstacle penalty on
// the signed distance sd of each substep position to the nearest box, a goal
// distance, and the length l of the position path (the speed |v| integrated
// by the same RK4 steps, as the planner's path-length cost is).  The forward pass keeps the state every 8 steps; the adjoint
// recomputes each 8-step block from its checkpoint and runs the adjoint of the
// RK4 steps through it, with the vector-Jacobian product of the dynamics
// written out by hand.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace kpxd {

constexpr int kCkpt = 8;  // steps per checkpoint block

struct DiffConst {
    float inv_m, inv_j[3], gyro[3], grav, dt;
    float goal[3];
    float w_ctrl, w_obst, k_obst, d_safe, w_goal, w_len;
    float u_lo[4], u_hi[4];
    float x_lo[12], x_hi[12], ws_lo[3], ws_hi[3];
    int n_boxes;
};

// dynamics: state (position, ZYX Euler angles phi theta psi, world-frame
// velocity, body rates p q r), control (thrust, body torques)
__device__ __forceinline__ void f_quad(const DiffConst& C, const float* x, const float* u, float* xd)
{
    float sph, cph, sth, cth, sps, cps;
    __sincosf(x[3], &sph, &cph);
    __sincosf(x[4], &sth, &cth);
    __sincosf(x[5], &sps, &cps);
    const float sec = 1.0f / cth, tth = sth * sec;
    const float a = sph * x[10] + cph * x[11];
    xd[0] = x[6];
    xd[1] = x[7];
    xd[2] = x[8];
    xd[3] = x[9] + a * tth;
    xd[4] = cph * x[10] - sph * x[11];
    xd[5] = a * sec;
    const float acc = u[0] * C.inv_m;
    xd[6] = acc * (cps * sth * cph + sps * sph);
    xd[7] = acc * (sps * sth * cph - cps * sph);
    xd[8] = acc * (cth * cph) - C.grav;
    xd[9] = (u[1] - C.gyro[0] * x[10] * x[11]) * C.inv_j[0];
    xd[10] = (u[2] - C.gyro[1] * x[9] * x[11]) * C.inv_j[1];
    xd[11] = (u[3] - C.gyro[2] * x[9] * x[10]) * C.inv_j[2];
}

// vector-Jacobian product of f_quad: gx += (df/dx)^T w, gu += (df/du)^T w
__device__ __forceinline__ void vjp_quad(const DiffConst& C, const float* x, const float* u, const float* w,
                                         float* gx, float* gu)
{
    float sph, cph, sth, cth, sps, cps;
    __sincosf(x[3], &sph, &cph);
    __sincosf(x[4], &sth, &cth);
    __sincosf(x[5], &sps, &cps);
    const float sec = 1.0f / cth, tth = sth * sec;
    const float wp = x[9], wq = x[10], wr = x[11];
    const float a = sph * wq + cph * wr;  // d a / d phi = b
    const float b = cph * wq - sph * wr;
    // position rates = velocity
    gx[6] += w[0];
    gx[7] += w[1];
    gx[8] += w[2];
    // Euler-angle rates
    gx[3] += w[3] * b * tth - w[4] * a + w[5] * b * sec;
    gx[4] += w[3] * a * sec * sec + w[5] * a * sec * tth;
    gx[9] += w[3];
    gx[10] += w[3] * sph * tth + w[4] * cph + w[5] * sph * sec;
    gx[11] += w[3] * cph * tth - w[4] * sph + w[5] * cph * sec;
    // thrust along the rotated body axis
    const float acc = u[0] * C.inv_m;
    const float r0 = cps * sth * cph + sps * sph, r1 = sps * sth * cph - cps * sph, r2 = cth * cph;
    gu[0] += (w[6] * r0 + w[7] * r1 + w[8] * r2) * C.inv_m;
    gx[3] += acc * (w[6] * (sps * cph - cps * sth * sph) - w[7] * (sps * sth * sph + cps * cph) -
                    w[8] * cth * sph);
    gx[4] += acc * cph * (w[6] * cps * cth + w[7] * sps * cth - w[8] * sth);
    gx[5] += acc * (w[6] * (cps * sph - sps * sth * cph) + w[7] * (cps * sth * cph + sps * sph));
    // Euler's equations
    const float w9 = w[9] * C.inv_j[0], w10 = w[10] * C.inv_j[1], w11 = w[11] * C.inv_j[2];
    gu[1] += w9;
    gu[2] += w10;
    gu[3] += w11;
    gx[9] -= w10 * C.gyro[1] * wr + w11 * C.gyro[2] * wq;
    gx[10] -= w9 * C.gyro[0] * wr + w11 * C.gyro[2] * wp;
    gx[11] -= w9 * C.gyro[0] * wq + w10 * C.gyro[1] * wp;
}

__device__ __forceinline__ float speed(const float* x)
{
    return sqrtf(fmaf(x[6], x[6], fmaf(x[7], x[7], x[8] * x[8])));
}

// g[6..8] += c v / |v| (the gradient of c |v|; zero at rest)
__device__ __forceinline__ void add_speed_grad(const float* x, float c, float* g)
{
    const float s = speed(x);
    if (!(s > 0.f)) return;
    const float q = c / s;
#pragma unroll
    for (int i = 6; i < 9; ++i) g[i] = fmaf(q, x[i], g[i]);
}

// One RK4 step; when ell is not null it also advances the path length by the
// RK4 combination of the speeds at the four stage states.
__device__ __forceinline__ void rk4_step(const DiffConst& C, float* x, const float* u, float* ell = nullptr)
{
    const float h = C.dt, h2 = 0.5f * C.dt, h6 = C.dt / 6.0f;
    float k[12], acc[12], t[12];
    float sacc = 0.f;
    if (ell) sacc = speed(x);
    f_quad(C, x, u, k);
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        acc[i] = k[i];
        t[i] = fmaf(h2, k[i], x[i]);
    }
    if (ell) sacc = fmaf(2.f, speed(t), sacc);
    f_quad(C, t, u, k);
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        acc[i] = fmaf(2.f, k[i], acc[i]);
        t[i] = fmaf(h2, k[i], x[i]);
    }
    if (ell) sacc = fmaf(2.f, speed(t), sacc);
    f_quad(C, t, u, k);
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        acc[i] = fmaf(2.f, k[i], acc[i]);
        t[i] = fmaf(h, k[i], x[i]);
    }
    if (ell) *ell = fmaf(h6, sacc + speed(t), *ell);
    f_quad(C, t, u, k);
#pragma unroll
    for (int i = 0; i < 12; ++i) x[i] = fmaf(h6, acc[i] + k[i], x[i]);
}

// Adjoint of one RK4 step from x: lam (dL/dx_{k+1}) becomes dL/dx_k, and
// gu accumulates dL/du through this step.  The stages are recomputed.  With
// wl != 0 the step's path-length increment, weighted by wl, is part of the
// loss: each stage state's speed adds its RK4 weight times wl v / |v|.
__device__ __forceinline__ void rk4_vjp(const DiffConst& C, const float* x, const float* u, float* lam, float* gu,
                                        float wl = 0.f)
{
    const float h = C.dt, h2 = 0.5f * C.dt, h6 = C.dt / 6.0f, h3 = C.dt / 3.0f;
    float k1[12], k2[12], k3[12], x2[12], x3[12], x4[12];
    f_quad(C, x, u, k1);
#pragma unroll
    for (int i = 0; i < 12; ++i) x2[i] = fmaf(h2, k1[i], x[i]);
    f_quad(C, x2, u, k2);
#pragma unroll
    for (int i = 0; i < 12; ++i) x3[i] = fmaf(h2, k2[i], x[i]);
    f_quad(C, x3, u, k3);
#pragma unroll
    for (int i = 0; i < 12; ++i) x4[i] = fmaf(h, k3[i], x[i]);
    float a[12], g[12], out[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        out[i] = lam[i];
        a[i] = h6 * lam[i];  // adjoint of k4
        g[i] = 0.f;
    }
    vjp_quad(C, x4, u, a, g, gu);  // g = dL/dx4
    if (wl != 0.f) add_speed_grad(x4, wl * h6, g);
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        out[i] += g[i];
        a[i] = fmaf(h3, lam[i], h * g[i]);  // adjoint of k3
        g[i] = 0.f;
    }
    vjp_quad(C, x3, u, a, g, gu);
    if (wl != 0.f) add_speed_grad(x3, wl * h3, g);
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        out[i] += g[i];
        a[i] = fmaf(h3, lam[i], h2 * g[i]);  // adjoint of k2
        g[i] = 0.f;
    }
    vjp_quad(C, x2, u, a, g, gu);
    if (wl != 0.f) add_speed_grad(x2, wl * h3, g);
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        out[i] += g[i];
        a[i] = fmaf(h6, lam[i], h2 * g[i]);  // adjoint of k1
        g[i] = 0.f;
    }
    vjp_quad(C, x, u, a, g, gu);
    if (wl != 0.f) add_speed_grad(x, wl * h6, g);
#pragma unroll
    for (int i = 0; i < 12; ++i) lam[i] = out[i] + g[i];
}

// Index of the box nearest to p (-1 without boxes or for a NaN position).
// The scan reads each box as centre and half extent (cx cy cz pad ex ey ez
// pad, LDS) at a wave-uniform index, so every read is a broadcast, and
// q = |p - c| - e per axis.  The key orders by signed distance without a
// square root: |max(q, 0)|^2 + min(max q, 0) is the squared distance of a box
// that does not hold p (positive) and the signed distance max q <= 0 of one
// that does, so holding boxes come first.  Ties go to the first box.
__device__ __forceinline__ int nearest_box(const float4* ce, int nb, const float* p)
{
    float best = INFINITY;
    int bi = -1;
#pragma unroll 8
    for (int b = 0; b < nb; ++b) {
        const float4 c = ce[2 * b], e = ce[2 * b + 1];
        const float qx = fabsf(p[0] - c.x) - e.x;
        const float qy = fabsf(p[1] - c.y) - e.y;
        const float qz = fabsf(p[2] - c.z) - e.z;
        const float m = fmaxf(qx, fmaxf(qy, qz));
        const float ox = fmaxf(qx, 0.f), oy = fmaxf(qy, 0.f), oz = fmaxf(qz, 0.f);
        const float key = fmaf(ox, ox, fmaf(oy, oy, fmaf(oz, oz, fminf(m, 0.f))));
        if (key < best) {
            best = key;
            bi = b;
        }
    }
    return bi;
}

// Signed distance of p to box b (LDS, two float4 per box) and its gradient:
// q = max(lo - p, p - hi) per axis; outside (max q > 0) sd = |max(q, 0)|,
// inside sd = max q (the first axis on ties).
__device__ __forceinline__ float box_sd(const float4* box, int b, const float* p, float* grad)
{
    const float4 lo = box[2 * b], hi = box[2 * b + 1];
    const float lov[3] = {lo.x, lo.y, lo.z}, hiv[3] = {hi.x, hi.y, hi.z};
    float q[3], s[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float below = lov[i] - p[i], above = p[i] - hiv[i];
        q[i] = fmaxf(below, above);
        s[i] = below >= above ? -1.f : 1.f;  // dq / dp
    }
    const float m = fmaxf(q[0], fmaxf(q[1], q[2]));
    if (!(m > 0.f)) {
        int ai = 0;
        if (q[1] > q[ai]) ai = 1;
        if (q[2] > q[ai]) ai = 2;
#pragma unroll
        for (int i = 0; i < 3; ++i) grad[i] = i == ai ? s[i] : 0.f;
        return m;
    }
    float o[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) o[i] = fmaxf(q[i], 0.f);
    const float d = sqrtf(fmaf(o[0], o[0], fmaf(o[1], o[1], o[2] * o[2])));
#pragma unroll
    for (int i = 0; i < 3; ++i) grad[i] = s[i] * o[i] / d;
    return d;
}

__device__ __forceinline__ float softplus(float z)
{
    return z > 0.f ? z + log1pf(expf(-z)) : log1pf(expf(z));
}

__device__ __forceinline__ float sigmoid(float z)
{
    return 1.f / (1.f + expf(-z));
}

// obstacle penalty of position p with nearest box b (< 0: none), with
// dP/dp added to g when g is not null
__device__ __forceinline__ float penalty(const DiffConst& C, const float4* box, int b, const float* p, float* g)
{
    if (b < 0 || C.w_obst == 0.f) return 0.f;
    float gs[3];
    const float sd = box_sd(box, b, p, gs);
    const float z = C.k_obst * (C.d_safe - sd);
    if (g) {
        const float c = -C.w_obst * C.k_obst * sigmoid(z);
#pragma unroll
        for (int i = 0; i < 3; ++i) g[i] += c * gs[i];
    }
    return C.w_obst * softplus(z);
}

__device__ __forceinline__ void segment_controls(const float* u, int seg, float* us)
{
#pragma unroll
    for (int c = 0; c < 4; ++c) us[c] = seg == 0 ? u[c] : seg == 1 ? u[4 + c] : seg == 2 ? u[8 + c] : u[12 + c];
}

// One pass over an edge: the loss (returned) and, when need_grad, its
// gradient with respect to the 16 controls in gu.  ck / nbx are this thread's
// checkpoint slots and nearest-box records in LDS (entry j at [j * stride]):
// 12 floats per started block of 8 steps and one short per step.  sbox holds each box as lo, hi
// and sce as centre, half extent (2 float4 each); nb = 0 skips the penalty.
// With check_valid, first_bad receives the first step whose state leaves C's
// valid set (state bounds, closed workspace, closed boxes), 0 if none.
__device__ __forceinline__ float edge_pass(const DiffConst& C, const float4* sbox, const float4* sce, int nb,
                                           const float* x0, const float* u, int n, float* ck,
                                           unsigned short* nbx, int stride, bool need_grad, float* gu,
                                           bool check_valid, int& first_bad)
{
    const int b1 = n / 4, b2 = n / 2, b3 = (3 * n) / 4;  // segment boundaries
    const int n_blk = (n + kCkpt - 1) / kCkpt;
    // forward, keeping x_k at slot k / 8 for k = 0, 8, ..
    float x[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) x[i] = x0[i];
    float pen = 0.f, ell = 0.f;
    const bool with_len = C.w_len != 0.f;  // uniform
    first_bad = 0;
    for (int k = 0; k < n; ++k) {
        if (k % kCkpt == 0 && need_grad)
#pragma unroll
            for (int i = 0; i < 12; ++i) ck[((k / kCkpt) * 12 + i) * stride] = x[i];
        float us[4];
        segment_controls(u, (k >= b1) + (k >= b2) + (k >= b3), us);
        rk4_step(C, x, us, with_len ? &ell : nullptr);
        const int bi = nearest_box(sce, nb, x);
        if (need_grad) nbx[k * stride] = (unsigned short)bi;
        pen += penalty(C, sbox, bi, x, nullptr);
        if (check_valid && first_bad == 0) {  // validity of x_{k+1}
            bool ok = true;
#pragma unroll
            for (int i = 0; i < 12; ++i) ok = ok && x[i] >= C.x_lo[i] && x[i] <= C.x_hi[i];
#pragma unroll
            for (int a = 0; a < 3; ++a) ok = ok && x[a] >= C.ws_lo[a] && x[a] <= C.ws_hi[a];
            if (bi >= 0) {  // a box holding x holds it nearest
                const float4 lo = sbox[2 * bi], hi = sbox[2 * bi + 1];
                ok = ok && !(x[0] >= lo.x && x[0] <= hi.x && x[1] >= lo.y && x[1] <= hi.y &&
                             x[2] >= lo.z && x[2] <= hi.z);
            }
            if (!ok) first_bad = k + 1;
        }
    }
    float u2 = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) u2 = fmaf(u[i], u[i], u2);
    float gd2 = 0.f, lam[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) lam[i] = 0.f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float d = x[a] - C.goal[a];
        gd2 = fmaf(d, d, gd2);
        lam[a] = 2.f * C.w_goal * d;
    }
    const float L = n * C.dt + C.w_ctrl * u2 + pen + C.w_goal * gd2 + C.w_len * ell;
    if (!need_grad) return L;
    // backward, block by block from the last: recompute the block's states
    // from its checkpoint, then the adjoint of its steps in reverse; x still
    // holds x_n
#pragma unroll
    for (int i = 0; i < 16; ++i) gu[i] = 2.f * C.w_ctrl * u[i];
    for (int blk = n_blk - 1; blk >= 0; --blk) {
        const int k0 = blk * kCkpt;
        float xb[kCkpt + 1][12];  // x_{k0} .. x_{k0 + 8} (entries past x_n unused)
#pragma unroll
        for (int i = 0; i < 12; ++i) xb[0][i] = ck[(blk * 12 + i) * stride];
#pragma unroll
        for (int t = 0; t < kCkpt; ++t) {
            const int k = k0 + t;
#pragma unroll
            for (int i = 0; i < 12; ++i) xb[t + 1][i] = xb[t][i];
            if (k + 1 < n) {
                float us[4];
                segment_controls(u, (k >= b1) + (k >= b2) + (k >= b3), us);
                rk4_step(C, xb[t + 1], us);
            } else if (k + 1 == n) {
#pragma unroll
                for (int i = 0; i < 12; ++i) xb[t + 1][i] = x[i];
            }
        }
#pragma unroll
        for (int t = kCkpt - 1; t >= 0; --t) {
            const int k = k0 + t;  // step k: x_k -> x_{k+1}
            if (k >= n) continue;
            const int seg = (k >= b1) + (k >= b2) + (k >= b3);
            float us[4], gs[4] = {0.f, 0.f, 0.f, 0.f};
            segment_controls(u, seg, us);
            const int bi = nb > 0 ? (int)(short)nbx[k * stride] : -1;
            penalty(C, sbox, bi, xb[t + 1], lam);  // the penalty term of x_{k+1}
            rk4_vjp(C, xb[t], us, lam, gs, C.w_len);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                gu[c] += seg == 0 ? gs[c] : 0.f;
                gu[4 + c] += seg == 1 ? gs[c] : 0.f;
                gu[8 + c] += seg == 2 ? gs[c] : 0.f;
                gu[12 + c] += seg == 3 ? gs[c] : 0.f;
            }
        }
    }
    return L;
}

}  // namespace kpxd
