// kpx_diff.hip -- differentiable quadrotor edge rollout on MI355X (gfx950):
// loss and its gradient with respect to the edge's controls, for batches of
// independent edges, behind the kpx_diff_* calls of include/kpx.h.  One thread
// per edge; the rollout, its loss and adjoint are in kpx_diff_device.hpp.
#include "../../include/kpx.h"
#include "kpx_diff_device.hpp"

#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <string>

namespace {

using namespace kpxd;

constexpr int kDiffBlock = 256;
constexpr int kMaxBlocks = 5;                 // checkpoint blocks: n <= 40
constexpr int kDiffMaxSteps = kCkpt * kMaxBlocks;
constexpr int kDiffMaxBoxes = 1024;  // 64 KiB of LDS beside 80 KiB of per-edge records

// Loss of edge e and, when grad != nullptr, its gradient with respect to the
// 16 controls; `polish` > 0 instead takes that many projected gradient steps
// u <- clamp(u - lr * grad, u_lo, u_hi) in place and leaves the final loss.
// Dynamic LDS: the boxes (2 float4 each as lo, hi, then 2 each as centre,
// half extent), the checkpoints x_0, x_8, ... of every thread ([slot * 12 +
// component][thread]), and the nearest box of every x_{k+1} ([k][thread],
// 16 bits).
__global__ __launch_bounds__(kDiffBlock) void k_diff(DiffConst C, const float4* __restrict__ boxes,
                                                     const float* __restrict__ x0g, float* __restrict__ ug,
                                                     const int* __restrict__ ng, long long E,
                                                     float* __restrict__ loss, float* __restrict__ grad,
                                                     int polish, float lr, int* __restrict__ fbad)
{
    extern __shared__ float4 lds[];
    float4* sbox = lds;
    float* sck = reinterpret_cast<float*>(lds + 4 * C.n_boxes);
    unsigned short* sidx = reinterpret_cast<unsigned short*>(sck + kMaxBlocks * 12 * kDiffBlock);
    for (int i = threadIdx.x; i < 4 * C.n_boxes; i += blockDim.x) sbox[i] = boxes[i];
    __syncthreads();
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const int nb = C.w_obst != 0.f || fbad ? C.n_boxes : 0;
    const int n = ng[e];
    float u[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) u[i] = ug[(long long)i * E + e];
    if (n < 4 || n > kDiffMaxSteps) {  // outside the supported edge lengths
        loss[e] = NAN;
        if (grad)
#pragma unroll
            for (int i = 0; i < 16; ++i) grad[(long long)i * E + e] = 0.f;
        if (fbad) fbad[e] = -1;
        return;
    }
    float x0[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) x0[i] = x0g[(long long)i * E + e];
    const int rounds = polish > 0 ? polish + 1 : 1;
    float L = 0.f, gu[16];
    int first_bad = 0;
    for (int round = 0; round < rounds; ++round) {
        const bool last = round + 1 == rounds;
        L = edge_pass(C, sbox, sbox + 2 * C.n_boxes, nb, x0, u, n, sck + threadIdx.x, sidx + threadIdx.x,
                      kDiffBlock, grad != nullptr || !last, gu, last && fbad != nullptr, first_bad);
        if (!last) {  // a projected gradient step
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int c = i & 3;
                u[i] = fminf(fmaxf(u[i] - lr * gu[i], C.u_lo[c]), C.u_hi[c]);
            }
        } else if (grad) {
#pragma unroll
            for (int i = 0; i < 16; ++i) grad[(long long)i * E + e] = gu[i];
        }
    }
    loss[e] = L;
    if (fbad) fbad[e] = first_bad;
    if (polish > 0)
#pragma unroll
        for (int i = 0; i < 16; ++i) ug[(long long)i * E + e] = u[i];
}

}  // namespace

// dynamic LDS of k_diff: boxes, checkpoints, nearest-box indices
static size_t lds_bytes(int n_boxes)
{
    return sizeof(float4) * 4 * n_boxes + sizeof(float) * kMaxBlocks * 12 * kDiffBlock +
           sizeof(unsigned short) * kDiffMaxSteps * kDiffBlock;
}

struct kpx_diff {
    DiffConst C;
    float4* boxes = nullptr;
    hipStream_t stream = nullptr;
    std::string err;
};

extern "C" {

int kpx_diff_create(const kpx_diff_problem* p, void* hip_stream, kpx_diff** out)
{
    if (!p || !out) return KPX_ERR_ARG;
    *out = nullptr;
    if (p->n_boxes < 0 || p->n_boxes > kDiffMaxBoxes || (p->n_boxes > 0 && !p->boxes)) return KPX_ERR_ARG;
    const float m = p->dyn_params[0], jx = p->dyn_params[1], jy = p->dyn_params[2], jz = p->dyn_params[3];
    if (!(m > 0.f) || !(jx > 0.f) || !(jy > 0.f) || !(jz > 0.f) || !(p->dt > 0.f)) return KPX_ERR_ARG;
    if (!std::isfinite(p->w_len)) return KPX_ERR_ARG;
    for (int c = 0; c < 4; ++c)
        if (!(p->u_lo[c] <= p->u_hi[c])) return KPX_ERR_ARG;
    for (int b = 0; b < p->n_boxes; ++b)
        for (int a = 0; a < 3; ++a)
            if (!(p->boxes[6 * b + a] <= p->boxes[6 * b + 3 + a])) return KPX_ERR_ARG;
    // dynamic LDS beyond the default limit (many boxes beside the checkpoints)
    const size_t lds_max = lds_bytes(kDiffMaxBoxes);
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_diff), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds_max) != hipSuccess)
        return KPX_ERR_DEVICE;
    kpx_diff* d = new (std::nothrow) kpx_diff;
    if (!d) return KPX_ERR_OOM;
    DiffConst& C = d->C;
    C.inv_m = 1.0f / m;
    C.inv_j[0] = 1.0f / jx;
    C.inv_j[1] = 1.0f / jy;
    C.inv_j[2] = 1.0f / jz;
    C.gyro[0] = jz - jy;
    C.gyro[1] = jx - jz;
    C.gyro[2] = jy - jx;
    C.grav = p->dyn_params[4];
    C.dt = p->dt;
    for (int a = 0; a < 3; ++a) C.goal[a] = p->goal[a];
    C.w_ctrl = p->w_ctrl;
    C.w_obst = p->w_obst;
    C.k_obst = p->k_obst;
    C.d_safe = p->d_safe;
    C.w_goal = p->w_goal;
    C.w_len = p->w_len;
    for (int c = 0; c < 4; ++c) {
        C.u_lo[c] = p->u_lo[c];
        C.u_hi[c] = p->u_hi[c];
    }
    for (int i = 0; i < 12; ++i) {
        C.x_lo[i] = p->x_lo[i];
        C.x_hi[i] = p->x_hi[i];
    }
    for (int a = 0; a < 3; ++a) {
        C.ws_lo[a] = p->ws_lo[a];
        C.ws_hi[a] = p->ws_hi[a];
    }
    C.n_boxes = p->n_boxes;
    d->stream = (hipStream_t)hip_stream;
    const size_t nb = (size_t)(p->n_boxes > 0 ? p->n_boxes : 1);
    // lo, hi of every box, then centre, half extent of every box
    if (hipMalloc(&d->boxes, sizeof(float4) * 4 * nb) != hipSuccess) {
        delete d;
        return KPX_ERR_OOM;
    }
    float4* hb = new (std::nothrow) float4[4 * nb];
    if (!hb) {
        (void)hipFree(d->boxes);
        delete d;
        return KPX_ERR_OOM;
    }
    for (int b = 0; b < p->n_boxes; ++b) {
        const float* s = p->boxes + 6 * b;
        hb[2 * b] = make_float4(s[0], s[1], s[2], 0.f);
        hb[2 * b + 1] = make_float4(s[3], s[4], s[5], 0.f);
        float c[3], h[3];
        for (int a = 0; a < 3; ++a) {
            c[a] = (float)(0.5 * ((double)s[a] + (double)s[3 + a]));
            h[a] = (float)(0.5 * ((double)s[3 + a] - (double)s[a]));
        }
        hb[2 * p->n_boxes + 2 * b] = make_float4(c[0], c[1], c[2], 0.f);
        hb[2 * p->n_boxes + 2 * b + 1] = make_float4(h[0], h[1], h[2], 0.f);
    }
    const hipError_t e = p->n_boxes > 0 ? hipMemcpy(d->boxes, hb, sizeof(float4) * 4 * p->n_boxes,
                                                    hipMemcpyHostToDevice)
                                        : hipSuccess;
    delete[] hb;
    if (e != hipSuccess) {
        (void)hipFree(d->boxes);
        delete d;
        return KPX_ERR_DEVICE;
    }
    *out = d;
    return KPX_OK;
}

static int diff_launch(kpx_diff* d, const float* x0, float* u, const int32_t* n, int64_t E, float* loss,
                       float* grad, int polish, float lr, int32_t* first_invalid)
{
    if (!d || E < 0 || (E > 0 && (!x0 || !u || !n || !loss))) return KPX_ERR_ARG;
    if (E == 0) return KPX_OK;
    const long long blocks = (E + kDiffBlock - 1) / kDiffBlock;
    if (blocks > 0x7FFFFFFFll) return KPX_ERR_ARG;
    k_diff<<<(unsigned)blocks, kDiffBlock, lds_bytes(d->C.n_boxes), d->stream>>>(
        d->C, d->boxes, x0, u, n, E, loss, grad, polish, lr, first_invalid);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        d->err = hipGetErrorString(e);
        return KPX_ERR_DEVICE;
    }
    return KPX_OK;
}

int kpx_diff_loss_grad(kpx_diff* d, const float* x0, const float* u, const int32_t* n, int64_t E, float* loss,
                       float* grad)
{
    return diff_launch(d, x0, const_cast<float*>(u), n, E, loss, grad, 0, 0.f, nullptr);
}

int kpx_diff_polish(kpx_diff* d, const float* x0, float* u, const int32_t* n, int64_t E, int32_t steps, float lr,
                    float* loss, int32_t* first_invalid)
{
    if (steps < 0 || !(lr >= 0.f)) return KPX_ERR_ARG;
    return diff_launch(d, x0, u, n, E, loss, nullptr, steps, lr, first_invalid);
}

int kpx_diff_destroy(kpx_diff* d)
{
    if (!d) return KPX_OK;
    if (d->stream) (void)hipStreamSynchronize(d->stream);
    else (void)hipDeviceSynchronize();
    if (d->boxes) (void)hipFree(d->boxes);
    delete d;
    return KPX_OK;
}

const char* kpx_diff_last_error(const kpx_diff* d)
{
    return d ? d->err.c_str() : "";
}

}  // extern "C"
