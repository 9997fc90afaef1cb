// kpx_device.hpp -- float32 device math of one Kino-PAX+ expansion on gfx950:
// the Philox4x32-10 sample map, the three robot models, the RK4 step, the
// valid-set test and the region map.  Header-only; included by kpx.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kpx {

constexpr int kDI6 = 0;
constexpr int kQUAD12 = 1;
constexpr int kDUBINS6 = 2;
constexpr int kTIME = 0;
constexpr int kPATH = 1;

constexpr uint8_t kActive = 0;
constexpr uint8_t kInactive = 1;
constexpr uint8_t kTerminal = 2;

constexpr uint64_t kEmpty = ~0ull;

template <int DYN>
struct Dims;
template <>
struct Dims<kDI6> {
    static constexpr int D = 6, M = 3;
};
template <>
struct Dims<kQUAD12> {
    static constexpr int D = 12, M = 4;
};
template <>
struct Dims<kDUBINS6> {
    static constexpr int D = 6, M = 3;
};

// The integration loop keeps angles and angular rates in revolutions
// (radians / 2 pi): the hardware sine and cosine take revolutions, so no
// per-evaluation rescaling is needed, and the kinematic equations are
// homogeneous in (angle, rate) so they keep their form.  Components so scaled,
// and the controls that are angular rates or feed one:
//   QUAD12  angles 3-5, body rates 9-11; torques 1-3 (the gyroscopic
//           coefficients are multiplied by 2 pi to compensate)
//   DUBINS6 heading 3, flight-path angle 4; their rates, controls 0-1
constexpr float kInv2Pi = 0.15915494309189535f;
constexpr float k2Pi = 6.283185307179586f;

__host__ __device__ constexpr bool rev_state(int dyn, int i)
{
    return dyn == kQUAD12 ? ((i >= 3 && i <= 5) || i >= 9) : dyn == kDUBINS6 ? (i == 3 || i == 4) : false;
}
__host__ __device__ constexpr bool rev_control(int dyn, int i)
{
    return dyn == kQUAD12 ? (i >= 1) : dyn == kDUBINS6 ? (i <= 1) : false;
}

// Problem constants in the form the kernels use them (prepared on the host in
// float32): planning bounds already shrunk by the clearance margin, boxes grown
// by it, region scales and reciprocal inertias precomputed.
struct DevProblem {
    int dyn, cost, d, m;
    float dt, h2, h6;
    int steps_min, steps_range;
    float u_lo[4], u_span[4];
    float x_lo[12], x_hi[12];      // planning state bounds (+-inf when unbounded)
    float ws_lo[3], ws_hi[3];      // planning workspace
    float cell_lo[3], cell_scale[3];
    int grid[3];
    int vel_sign_bins, vel_idx;
    float goal_c[3], goal_r2;      // (goal radius - margin)^2
    float inv_mass, inv_j[3], gyro[3], grav;
    uint32_t bound_mask;           // bit i: component i has a finite bound
    // the bound test in integration units (angles and angular rates in
    // revolutions): component i is in bounds iff |fma(x_i, bnd_s[i], bnd_o[i])| <= 1;
    // (0, 0) for unbounded components and for those with one finite bound,
    // which are listed in os_mask and tested against os_lo / os_hi directly
    float bnd_s[12], bnd_o[12];
    uint32_t os_mask;
    float os_lo[12], os_hi[12];
    int n_boxes;
    // uniform grid over the workspace listing, per grid cell, the (grown)
    // boxes that overlap it: a point is only tested against its cell's list
    float gb_lo[3], gb_scale[3];
    int gb_n[3];
    int gb_cells, gb_entries;
    int n_cu;                      // compute units: propagate runs one block per CU
    int n_cells;
    int K, n_select, s_max;
    int i_max;
    int surv_max;
    long long cap;
    uint32_t seed_lo, seed_hi, query;
    int n_tiles;                   // survivor-count tiles covering s_max slots
    int n_bgroups, n_tgroups;      // group sums per parity: region blocks, tiles (two-level scans)
    int sort_shift;                // step-count sort: bin = (n - steps_min) >> sort_shift
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products
// with the published multipliers, the key advancing by the published Weyl
// increments between rounds.  Each product is formed whole, as one 64-bit
// multiply-add (v_mad_u64_u32), instead of its high and low words apart.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = (uint32_t)p1;
        c[2] = n2;
        c[3] = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Control and step count of expansion `slot` in iteration `it`: counter
// (it, slot, query, block), word i -> control i, word m -> step count.
template <int DYN>
__device__ __forceinline__ void sample(const DevProblem& P, uint32_t it, uint32_t slot,
                                       float* u, int& n)
{
    constexpr int M = Dims<DYN>::M;
    uint32_t w[8];
    uint32_t c0[4] = {it, slot, P.query, 0u};
    philox10(c0, P.seed_lo, P.seed_hi);
    w[0] = c0[0]; w[1] = c0[1]; w[2] = c0[2]; w[3] = c0[3];
    if (M >= 4) {
        uint32_t c1[4] = {it, slot, P.query, 1u};
        philox10(c1, P.seed_lo, P.seed_hi);
        w[4] = c1[0]; w[5] = c1[1]; w[6] = c1[2]; w[7] = c1[3];
    }
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const float unit = (float)(w[i] >> 8) * 0x1p-24f;
        u[i] = __builtin_fmaf(unit, P.u_span[i], P.u_lo[i]);
    }
    n = P.steps_min + (int)__umulhi(w[M], (uint32_t)P.steps_range);
}

// Constants the integration loop reads every substep, gathered into one small
// struct: state bounds (the workspace folded into the position bounds; +-inf
// where unbounded), step sizes and model constants.
template <int DYN>
struct Hot {
    static constexpr int D = Dims<DYN>::D;
    float dt, h2, h6, hh6;          // hh6 = dt^2 / 6
    float bs[D], bo[D];            // scaled bound test (see DevProblem)
    uint32_t os_mask;
    float inv_mass, inv_j[3], gyro_j[3], grav;  // gyro_j: gyroscopic coefficient times 1/J, revolution units
    float gb_lo[3], gb_scale[3];
    int gb_n[3];
};

template <int DYN>
__device__ __forceinline__ Hot<DYN> make_hot(const DevProblem& P)
{
    constexpr int D = Dims<DYN>::D;
    Hot<DYN> H;
    H.dt = P.dt;
    H.h2 = P.h2;
    H.h6 = P.h6;
    H.hh6 = P.dt * P.h6;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        H.bs[i] = P.bnd_s[i];
        H.bo[i] = P.bnd_o[i];
        // keep the bound coefficients in vector registers: the loop uses them
        // every substep and scalar registers are short
        asm volatile("" : "+v"(H.bs[i]));
        asm volatile("" : "+v"(H.bo[i]));
    }
    H.os_mask = P.os_mask;
    H.inv_mass = P.inv_mass;
    H.grav = P.grav;
    asm volatile("" : "+v"(H.dt), "+v"(H.h2), "+v"(H.h6), "+v"(H.hh6), "+v"(H.inv_mass), "+v"(H.grav));
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        H.inv_j[a] = P.inv_j[a];
        H.gyro_j[a] = P.gyro[a] * k2Pi * P.inv_j[a];
        H.gb_lo[a] = P.gb_lo[a];
        H.gb_scale[a] = P.gb_scale[a];
        H.gb_n[a] = P.gb_n[a];
        asm volatile("" : "+v"(H.inv_j[a]), "+v"(H.gyro_j[a]), "+v"(H.gb_lo[a]), "+v"(H.gb_scale[a]),
                     "+v"(H.gb_n[a]));
    }
    return H;
}

// ---------------------------------------------------------------------------
// A control in the form the derivative takes it, fixed for the whole edge:
// angular-rate controls in revolutions, and for the quadrotor the thrust
// divided by the mass and each torque divided by its moment of inertia, so
// that no substep repeats those products.
// ---------------------------------------------------------------------------
template <int DYN>
__device__ __forceinline__ void edge_controls(const Hot<DYN>& H, const float* u_in, float* u)
{
    constexpr int M = Dims<DYN>::M;
#pragma unroll
    for (int c = 0; c < M; ++c) u[c] = u_in[c] * (rev_control(DYN, c) ? kInv2Pi : 1.f);
    if constexpr (DYN == kQUAD12) {
        u[0] *= H.inv_mass;
#pragma unroll
        for (int a = 0; a < 3; ++a) u[1 + a] *= H.inv_j[a];
    }
}

// ---------------------------------------------------------------------------
// Dynamics f(x, u) (u as edge_controls leaves it) and, for the path-length
// cost, the speed |p'|.
// ---------------------------------------------------------------------------
template <int DYN, int COST>
__device__ __forceinline__ void deriv(const Hot<DYN>& P, const float* x, const float* u,
                                      float* xd, float& ld)
{
    if constexpr (DYN == kDI6) {
        xd[0] = x[3]; xd[1] = x[4]; xd[2] = x[5];
        xd[3] = u[0]; xd[4] = u[1]; xd[5] = u[2];
        if constexpr (COST == kPATH) ld = __builtin_sqrtf(x[3] * x[3] + x[4] * x[4] + x[5] * x[5]);
    } else if constexpr (DYN == kQUAD12) {
        // x[3..5] in revolutions
        const float sph = __builtin_amdgcn_sinf(x[3]), cph = __builtin_amdgcn_cosf(x[3]);
        const float sth = __builtin_amdgcn_sinf(x[4]), cth = __builtin_amdgcn_cosf(x[4]);
        const float sps = __builtin_amdgcn_sinf(x[5]), cps = __builtin_amdgcn_cosf(x[5]);
        const float rc = __builtin_amdgcn_rcpf(cth);
        const float wp = x[9], wq = x[10], wr = x[11];
        // Euler-angle rates W(roll, pitch) w
        const float b = __builtin_fmaf(sph, wq, cph * wr) * rc;
        xd[0] = x[6]; xd[1] = x[7]; xd[2] = x[8];
        xd[3] = __builtin_fmaf(b, sth, wp);
        xd[4] = __builtin_fmaf(cph, wq, -(sph * wr));
        xd[5] = b;
        // thrust along the body z axis, R_z(yaw) R_y(pitch) R_x(roll) e_3, minus gravity
        const float t1 = u[0] * sph, t2 = u[0] * cph, t3 = t2 * sth;
        xd[6] = __builtin_fmaf(cps, t3, sps * t1);
        xd[7] = __builtin_fmaf(sps, t3, -(cps * t1));
        xd[8] = __builtin_fmaf(t2, cth, -P.grav);
        // J^-1 (tau - w x J w) with diagonal J
        xd[9] = __builtin_fmaf(-(P.gyro_j[0] * wq), wr, u[1]);
        xd[10] = __builtin_fmaf(-(P.gyro_j[1] * wp), wr, u[2]);
        xd[11] = __builtin_fmaf(-(P.gyro_j[2] * wp), wq, u[3]);
        if constexpr (COST == kPATH) ld = __builtin_sqrtf(x[6] * x[6] + x[7] * x[7] + x[8] * x[8]);
    } else {
        // x[3], x[4] in revolutions
        const float cg = __builtin_amdgcn_cosf(x[4]), sg = __builtin_amdgcn_sinf(x[4]);
        const float v = x[5];
        const float vc = v * cg;
        xd[0] = vc * __builtin_amdgcn_cosf(x[3]);
        xd[1] = vc * __builtin_amdgcn_sinf(x[3]);
        xd[2] = v * sg;
        xd[3] = u[0]; xd[4] = u[1]; xd[5] = u[2];
        if constexpr (COST == kPATH) ld = v;
    }
}

// Classical RK4 step of size dt on the state (and the path length).
//
// Quadrotor under the time cost: the position rates are the velocities, and
// the velocity rates depend on neither positions nor velocities, so the four
// stage velocities v, v + h/2 a1, v + h/2 a2 and v + h a3 (a_i the velocity
// rates of stage i) weigh in as 6 v + h (a1 + a2 + a3): the position advances
// by h v + h^2/6 (a1 + a2 + a3).  That is the same step, rounded differently,
// and the stage velocities are never formed (the path-length cost needs them
// for the speed).
template <int DYN, int COST>
__device__ __forceinline__ void rk4(const Hot<DYN>& P, float* x, const float* u, float& len)
{
    constexpr int D = Dims<DYN>::D;
    float k[D], acc[D], t[D];
    float lk = 0.f, lacc = 0.f;
    if constexpr (DYN == kQUAD12 && COST != kPATH) {
        float a[3];
        deriv<DYN, COST>(P, x, u, k, lk);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            a[i] = k[6 + i];
            t[i] = x[i];
        }
#pragma unroll
        for (int i = 3; i < D; ++i) {
            acc[i] = k[i];
            t[i] = __builtin_fmaf(P.h2, k[i], x[i]);
        }
        deriv<DYN, COST>(P, t, u, k, lk);
#pragma unroll
        for (int i = 0; i < 3; ++i) a[i] += k[6 + i];
#pragma unroll
        for (int i = 3; i < D; ++i) {
            acc[i] = __builtin_fmaf(2.f, k[i], acc[i]);
            t[i] = __builtin_fmaf(P.h2, k[i], x[i]);
        }
        deriv<DYN, COST>(P, t, u, k, lk);
#pragma unroll
        for (int i = 0; i < 3; ++i) a[i] += k[6 + i];
#pragma unroll
        for (int i = 3; i < D; ++i) {
            acc[i] = __builtin_fmaf(2.f, k[i], acc[i]);
            t[i] = __builtin_fmaf(P.dt, k[i], x[i]);
        }
        deriv<DYN, COST>(P, t, u, k, lk);
#pragma unroll
        for (int i = 0; i < 3; ++i) x[i] = __builtin_fmaf(P.hh6, a[i], __builtin_fmaf(P.dt, x[6 + i], x[i]));
#pragma unroll
        for (int i = 3; i < D; ++i) x[i] = __builtin_fmaf(P.h6, acc[i] + k[i], x[i]);
        return;
    }
    deriv<DYN, COST>(P, x, u, k, lk);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        acc[i] = k[i];
        t[i] = __builtin_fmaf(P.h2, k[i], x[i]);
    }
    lacc = lk;
    deriv<DYN, COST>(P, t, u, k, lk);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        acc[i] = __builtin_fmaf(2.f, k[i], acc[i]);
        t[i] = __builtin_fmaf(P.h2, k[i], x[i]);
    }
    lacc = __builtin_fmaf(2.f, lk, lacc);
    deriv<DYN, COST>(P, t, u, k, lk);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        acc[i] = __builtin_fmaf(2.f, k[i], acc[i]);
        t[i] = __builtin_fmaf(P.dt, k[i], x[i]);
    }
    lacc = __builtin_fmaf(2.f, lk, lacc);
    deriv<DYN, COST>(P, t, u, k, lk);
#pragma unroll
    for (int i = 0; i < D; ++i) x[i] = __builtin_fmaf(P.h6, acc[i] + k[i], x[i]);
    if constexpr (COST == kPATH) len = __builtin_fmaf(P.h6, lacc + lk, len);
}

// Workspace and state bounds (closed).  Each two-sided bound is an affine map
// onto [-1, 1], and the largest magnitude of the mapped values must not
// exceed 1.  The IEEE maximum propagates a NaN (which then fails the test),
// and gfx950 folds three magnitudes into one instruction (absolute values are
// operand modifiers).  Components with one finite bound (rare) are compared
// directly.
template <int DYN>
__device__ __forceinline__ bool in_bounds(const Hot<DYN>& H, const float* x, const float* os_lo,
                                          const float* os_hi)
{
    constexpr int D = Dims<DYN>::D;
    float m = __builtin_fabsf(__builtin_fmaf(x[0], H.bs[0], H.bo[0]));
#pragma unroll
    for (int i = 1; i < D; ++i)
        m = __builtin_elementwise_maximum(m, __builtin_fabsf(__builtin_fmaf(x[i], H.bs[i], H.bo[i])));
    bool ok = m <= 1.f;
    if (H.os_mask) {  // uniform
#pragma unroll
        for (int i = 0; i < D; ++i)
            if (H.os_mask & (1u << i)) ok &= (x[i] >= os_lo[i]) & (x[i] <= os_hi[i]);
    }
    return ok;
}

// Index of the box-grid cell holding position p (clamped).
template <typename C>
__device__ __forceinline__ int box_grid_cell(const C& P, const float* x)
{
    int idx[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int i = (int)__builtin_floorf((x[a] - P.gb_lo[a]) * P.gb_scale[a]);
        i = i < 0 ? 0 : i;
        i = i > P.gb_n[a] - 1 ? P.gb_n[a] - 1 : i;
        idx[a] = i;
    }
    return (idx[0] * P.gb_n[1] + idx[1]) * P.gb_n[2] + idx[2];
}

// Point inside a closed box (grown by the margin): a collision.  The box is
// stored as two float4: (lo x, lo y, lo z, -), (hi x, hi y, hi z, -).
__device__ __forceinline__ bool in_box(const float4* b, float px, float py, float pz)
{
    const float4 lo = b[0], hi = b[1];
    return (px >= lo.x) & (px <= hi.x) & (py >= lo.y) & (py <= hi.y) & (pz >= lo.z) & (pz <= hi.z);
}

// Region index: grid over the workspace (clamped), row-major (x, y, z), then
// optionally three velocity-sign bits (velocity >= 0); p is the position and
// v the velocity.
__device__ __forceinline__ int cell_of(const DevProblem& P, const float* p, const float* v)
{
    int idx[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int i = (int)__builtin_floorf((p[a] - P.cell_lo[a]) * P.cell_scale[a]);
        i = i < 0 ? 0 : i;
        i = i > P.grid[a] - 1 ? P.grid[a] - 1 : i;
        idx[a] = i;
    }
    int c = (idx[0] * P.grid[1] + idx[1]) * P.grid[2] + idx[2];
    if (P.vel_sign_bins) c = c * 8 + ((v[0] >= 0.f) << 2) + ((v[1] >= 0.f) << 1) + (v[2] >= 0.f);
    return c;
}

__device__ __forceinline__ bool in_goal(const DevProblem& P, const float* x)
{
    const float dx = x[0] - P.goal_c[0], dy = x[1] - P.goal_c[1], dz = x[2] - P.goal_c[2];
    return __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz)) <= P.goal_r2;
}

}  // namespace kpx
