// kpx.hip -- Kino-PAX+ hot path on AMD Instinct MI355X (gfx950): kernels and
// the C ABI declared in include/kpx.h.
//
// One iteration (Alg. 1 loop body) is four kernels on one stream, with every
// count kept in device memory so that nothing waits for the host:
//   1. propagate   one lane per expansion slot: Philox sample, RK4 substeps
//                  with the valid-set test after each, region map, additive
//                  cost, packed (cost | id) 64-bit atomicMin on the region
//                  table (Alg. 2, Alg. 6); the lane that takes a region from
//                  a tree node marks that node terminal (Alg. 3).
//   2. prune+flags one thread per region: Alg. 3 for the region's owner (the
//                  live nodes are exactly the region owners, so prune walks
//                  the region table instead of the whole tree); a region an
//                  arrival took marks that slot in the survivor mask V_U
//                  (the U-filter of App. A: valid and still the region
//                  minimum) and counts it in its tile.
//   3. insert      App. A UpdateTree: rank = exclusive scan of the mask, the
//                  survivor is appended at |T| + rank, its region is re-keyed
//                  to the new tree index, goal nodes atomicMin the solution.
//   4. finalize+select  one workgroup: counters, statistics, capacity check,
//                  then the next iteration's selection (active region owners
//                  in region order from a rotating cursor, at most n_select).
#include "../../include/kpx.h"
#include "kpx_device.hpp"
#include "kpx_diff_device.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace kpx;

namespace {

constexpr int kBlock = 256;
constexpr int kTile = kBlock;             // survivor slots per tile (one per thread)
constexpr int kSelectThreads = 1024;
constexpr int kSelWords = 8;            // activity words per select thread kept in registers
constexpr int kSelLds = 8192;            // selections ranked in LDS (more go through global memory)
constexpr int kGroup = 1024;             // tiles, or region blocks, per group of the two-level scans
constexpr int kDirect = 8 * kGroup;      // at most this many counts are summed in one level
constexpr int kGroupPad = 32;            // ints per group sum: one 128-byte line each
constexpr int kSortBins = 64;             // step-count bins of the in-block sort
static_assert(kSortBins == 64, "the sort bins' prefix is one wave's scan");
constexpr int kBoxGridMax = 16;           // box-grid cells per workspace axis (at most)
constexpr int kBoxGridBytes = 48 * 1024;  // LDS budget of the box grid, its clearances and lists
constexpr int kChunkMax = 1024;           // expansion slots per propagate chunk (at most)
constexpr int kChunkBig = 2048;           // ... for blocks whose share of the slots exceeds kChunkMax
constexpr int kChunkMin = 64;
constexpr int kParMax = 256;              // parent states staged per chunk (at most)
// from this many samples per node, propagate first keeps, per block and
// region, only the chunk's lowest key for the region table (few parents
// then send many edges to the same regions)
constexpr int kDedupK = 64;
constexpr int kInsertEarlyParents = 1 << 21;  // slot buffers up to this read every slot's parent in insert
// floats per candidate end-state row (slot-major: one row per slot, so that
// a lane writes its end state, and insert reads a survivor's, as whole
// 16-byte words)
__host__ __device__ constexpr int cx_row(int d) { return (d + 3) & ~3; }
// idle lanes of a propagate wave take new slots together, this many at a
// time; with two waves per SIMD the other wave hides part of a refill
constexpr int kRefillBatch = 16;
constexpr int kRefillBatchWide = 8;
static_assert(kChunkMax == 1024 && kChunkBig == 2048, "the dedupe table hashes regions to 10 or 11 bits");
constexpr int kPropBlock = 256;           // propagate: one wave per SIMD, one block per CU
constexpr int kPropBlockWide = 512;       // ... or two, for cheap models at large sizes
constexpr int kStatsCap = 1 << 16;
// regions per thread of prune and the close: one for a query of fewer than
// kRptRegions regions (short blocks, each a few dependent loads, all resident
// at once); four for larger ones and for batches, whose regions would
// otherwise need many successive generations of resident blocks
constexpr int kRptBatch = 4;
constexpr long long kRptRegions = 1LL << 20;
constexpr int kMaxPath = 1 << 16;

struct DevState {
    long long n_tree;
    long long it;
    long long first_sol_it;
    unsigned long long sol;
    unsigned long long substeps_acc;
    long long last_substeps;
    int n_valid_acc;
    int n_live_acc;      // regions a tree node still owns after propagate (prune's count)
    int last_n_valid;
    int n_sel;
    int last_n_sel;
    int last_n_surv;
    int cursor;
    int cursor_next;
    int full;
    int n_surv;          // survivors of this iteration (written by the insert kernel)
    int k;               // samples per selected node in this iteration
    int last_k;          // ... in the last completed one
};

struct DevPtrs {
    float* x;            // D x cap
    float* u;            // M x cap
    uint16_t* steps;
    int* parent;
    uint32_t* cost;
    int* cell;
    uint8_t* status;
    uint8_t* icount;
    uint8_t* dead;       // terminal, or some ancestor was beaten (monotone)
    int4* anc;           // 2 per node: the 8 nearest proper ancestors (-1 past the root)
    unsigned long long* tbl;
    int* sel;
    unsigned long long* ckey;
    int* ccell;
    float* cx;           // s_max rows of cx_row(D) floats: a slot's end state, padded to 16-byte words
    uint8_t* cflag;      // bit 0 valid, bit 1 goal
    uint8_t* csurv;
    int* tile_count;
    uint8_t* act;        // region will be expanded next (owner active after this iteration)
    float4* boxes;       // 2 per box: lo, hi (grown by the margin)
    int2* gcell;         // box grid, per grid cell: (first list entry | count << 20,
                         // bits of the clearance radius to the boxes not listed)
    uint16_t* glist;     // box grid: box indices
    DevState* st;        // two states, by iteration parity: the current one is read by every
                         // kernel of an iteration and the close of the iteration writes the other
    int2* bcount;        // per block of kBlock regions: active regions at / after the cursor, before it
    int2* bgroup;        // 2 x n_bgroups lines, by iteration parity: bcount summed over kGroup region blocks
    int* tgroup;         // 2 x n_tgroups lines, by iteration parity: tile_count summed over kGroup tiles
    kpx_iter_stats* stats;
    int* d_parent;       // dump (may be null)
    float* d_u;
    int* d_n;
    int* d_fi;
    int* d_pfi;          // dump of the edge polish, per node inserted: first invalid step,
    int* d_pcell;        //   region of the polished end state,
    uint8_t* d_pflag;    //   bit 0 accepted, bit 1 end state in the goal
    int* path;           // solution extraction
    float* path_x;
    float* path_u;
    int* path_n;
    int* path_len;
    float* x_init;
};

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int wave_sum(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// The same sum for a wave whose 64 lanes are all active, without LDS: DPP row
// shifts by 1, 2, 4 and 8 leave each row of 16 lanes its running sum, whose
// last lanes (15, 31, 47, 63) hold the row totals.
__device__ __forceinline__ int wave_sum_rows(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    return __builtin_amdgcn_readlane(v, 15) + __builtin_amdgcn_readlane(v, 31) +
           __builtin_amdgcn_readlane(v, 47) + __builtin_amdgcn_readlane(v, 63);
}

// Exclusive prefix sum over the 64 lanes of a fully active wave, without LDS:
// the DPP row shifts above give each lane the running sum of its row of 16,
// and the totals of the rows before its own come from lanes 15, 31 and 47.
__device__ __forceinline__ int wave_exclusive_scan(int v)
{
    int x = v;
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
    const int t0 = __builtin_amdgcn_readlane(x, 15), t1 = __builtin_amdgcn_readlane(x, 31),
              t2 = __builtin_amdgcn_readlane(x, 47);
    const int row = (int)(threadIdx.x & 63) >> 4;
    return x - v + (row > 0 ? t0 : 0) + (row > 1 ? t1 : 0) + (row > 2 ? t2 : 0);
}

__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Two-level scans.  Per-tile survivor counts and per-region-block activity
// counts are prefix-summed by each consumer block over the counts before it.
// Up to kDirect counts that is done in one level.  Beyond, the counts form
// groups of kGroup: the producer blocks add their count to their group's sum
// (one atomic per block, each group on a line of its own) and a consumer sums
// the counts of its group before it plus the earlier groups' sums.  The sums
// are kept per iteration parity; each close clears the other parity's.
__host__ __device__ constexpr bool grouped(int n_groups) { return n_groups > kDirect / kGroup; }

__device__ __forceinline__ int* tgroup_at(const DevPtrs& T, const DevProblem& P, int par, int g)
{
    return T.tgroup + ((size_t)par * P.n_tgroups + g) * kGroupPad;
}

__device__ __forceinline__ int2* bgroup_at(const DevPtrs& T, const DevProblem& P, int par, int g)
{
    return T.bgroup + ((size_t)par * P.n_bgroups + g) * (kGroupPad / 2);
}

// ------------------------------------------------------------------ init

__global__ void k_fill_table(unsigned long long* tbl, uint8_t* act, int n, int n_act)
{
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x)
        tbl[c] = kEmpty;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n_act; c += gridDim.x * blockDim.x)
        act[c] = 0;
}

// ------------------------------------------------------------ refinement

// Region of every node under the refined grid; the nodes that are not
// terminal claim their new regions (one per old region, so one per new one),
// and the active ones mark their regions for the selection.
__global__ void k_refine_nodes(DevProblem P, DevPtrs T, const DevState* st)
{
    const long long n_tree = st->n_tree;
    const int vi = P.dyn == kQUAD12 ? 6 : 3;  // first velocity component (unused without sign bins)
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n_tree;
         i += (long long)gridDim.x * blockDim.x) {
        float p[3], v[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            p[a] = T.x[(long long)a * P.cap + i];
            v[a] = P.vel_sign_bins ? T.x[(long long)(vi + a) * P.cap + i] : 0.f;
        }
        const int c = cell_of(P, p, v);
        T.cell[i] = c;
        const uint8_t s = T.status[i];
        if (s != kTerminal) {
            atomicMin(&T.tbl[c], ((unsigned long long)T.cost[i] << 32) | (unsigned long long)(uint32_t)i);
            if (s == kActive) T.act[c] = 1;  // the region's owner is active: it may be selected
        }
    }
}

// A region index of the old grid (og, f times coarser per axis) -> the first
// of its cells in the refined grid (velocity-sign bits kept).
__device__ __forceinline__ int refine_index(const DevProblem& P, int c, int og1, int og2, int f)
{
    const int bits = P.vel_sign_bins ? (c & 7) : 0;
    const int sp = P.vel_sign_bins ? (c >> 3) : c;
    const int iz = sp % og2, iy = (sp / og2) % og1, ix = sp / (og2 * og1);
    const int s2 = ((ix * f) * P.grid[1] + iy * f) * P.grid[2] + iz * f;
    return P.vel_sign_bins ? s2 * 8 + bits : s2;
}

__global__ void k_refine_state(DevProblem P, DevState* st, int og1, int og2, int f)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    st->cursor = refine_index(P, st->cursor, og1, og2, f);
    st->cursor_next = refine_index(P, st->cursor_next, og1, og2, f);
    if (st->n_tree + P.surv_max > P.cap) st->full = 1;
}

// Initialisation of Alg. 1: the root is x_init, active; its region holds (0, root).
template <int DYN>
__global__ void k_init_root(DevProblem P, DevPtrs T, DevState* st, const float* x_init)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    constexpr int D = Dims<DYN>::D, M = Dims<DYN>::M;
    float x[D];
    for (int k = 0; k < D; ++k) {
        x[k] = x_init[k];
        T.x[(long long)k * P.cap] = x[k];
    }
    for (int k = 0; k < M; ++k) T.u[(long long)k * P.cap] = 0.f;
    T.steps[0] = 0;
    T.parent[0] = -1;
    T.cost[0] = 0u;
    const int c = cell_of(P, x, x + (DYN == kQUAD12 ? 6 : 3));
    T.cell[0] = c;
    T.status[0] = kActive;
    T.icount[0] = 0;
    T.dead[0] = 0;
    T.anc[0] = make_int4(-1, -1, -1, -1);
    T.anc[1] = make_int4(-1, -1, -1, -1);
    T.tbl[c] = 0ull;  // cost 0, id 0
    T.act[c] = 1;
    st->n_tree = 1;
    st->it = 0;
    // a root in the goal set is already a solution: the empty trajectory, cost 0
    const bool root_goal = in_goal(P, x);
    st->first_sol_it = root_goal ? 0 : -1;
    st->sol = root_goal ? 0ull : kEmpty;
    st->substeps_acc = 0;
    st->last_substeps = 0;
    st->n_valid_acc = 0;
    st->n_live_acc = 0;
    st->last_n_valid = 0;
    st->n_sel = 0;
    st->last_n_sel = 0;
    st->last_n_surv = 0;
    st->cursor = 0;
    st->cursor_next = 0;
    st->full = 0;
    st->n_surv = 0;
    st->k = 0;
    st->last_k = 0;
}

// Samples per selected node for a selection of nsel nodes: K when fixed;
// otherwise (samples_per_node = 0, the uncapped form of Sec. VI-A / App. A)
// every active node is selected, up to the candidate buffer's n_select slots,
// and the buffer is shared out evenly: lambda = max(1, floor(n_select / nsel)).
__device__ __forceinline__ int samples_for(const DevProblem& P, int nsel)
{
    return P.K > 0 ? P.K : (nsel > 0 ? max(1, P.n_select / nsel) : 1);
}

// ------------------------------------------------------------------ propagate

// Copies three arrays of 16-byte words from global memory into LDS, at word
// offsets o0, o1 and o2 of `lds`, each thread issuing all of its loads (from
// clamped, always valid addresses) before its first store, so that one memory
// round trip covers the copy.  Past the end a thread stores the last word
// again (the same value to the same place), and the destinations are integer
// offsets: no store sits in a branch, where the compiler would move each load
// down to its store and wait for the loads one by one.
__device__ __forceinline__ void stage_lds(int4* lds, const int4* s0, int o0, int n0, const int4* s1, int o1,
                                          int n1, const int4* s2, int o2, int n2)
{
    constexpr int U = 8;
    const int e0 = n0, e1 = e0 + n1, e2 = e1 + n2;
    if (e2 == 0) return;
    // word i of the concatenation: source address base_k + 16 i, LDS word c_k + i
    const uintptr_t a0 = (uintptr_t)s0, a1 = (uintptr_t)s1 - 16u * (uintptr_t)e0,
                    a2 = (uintptr_t)s2 - 16u * (uintptr_t)e1;
    const int c0 = o0, c1 = o1 - e0, c2 = o2 - e1;
    for (int b = 0; b < e2; b += U * (int)blockDim.x) {
        int4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = min(b + (int)threadIdx.x + u * (int)blockDim.x, e2 - 1);
            const uintptr_t a = (i >= e1 ? a2 : i >= e0 ? a1 : a0) + 16u * (uintptr_t)i;
            v[u] = *(const int4*)(const __attribute__((address_space(1))) int4*)a;  // a global load
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = min(b + (int)threadIdx.x + u * (int)blockDim.x, e2 - 1);
            lds[(i >= e1 ? c2 : i >= e0 ? c1 : c0) + i] = v[u];
        }
    }
}

// One block's share of propagate: block `blk` of `nblk` working for the
// problem P (state `st`).
//
// CF selects the cost-first form of the App. A remark, which is exact: an
// edge is first integrated with the state and workspace bounds only; its
// region and key then follow from the end state, and when the region table
// already holds a smaller key the edge cannot be the region's minimum (the
// table only decreases during propagate, and a skipped edge that is valid
// still lies above the final minimum), so its obstacle test is skipped
// (first_invalid -1).  Otherwise the lane integrates the edge again from the
// parent with the obstacle test, bit for bit as the plain form does.  The
// table value is loaded when the first pass ends and compared after the next
// trip, so that its latency hides under one RK4 step.
constexpr short kSkipped = -1;
template <int DYN, int COST, bool CF = false, int NT = kPropBlock, int CH = kChunkMax>
__device__ __forceinline__ void propagate_body(const DevProblem& P, const DevPtrs& T, DevState* st, int blk,
                                               int nblk)
{
    constexpr int D = Dims<DYN>::D, M = Dims<DYN>::M;
    constexpr int PT = CH / NT;          // slot rounds per thread in a full chunk
    extern __shared__ float4 dyn_lds[];  // boxes | parent states | grid cells | grid lists
    constexpr int SD = (D + 3) & ~3;     // a staged parent state: whole 16-byte words
    __shared__ float4 s_u[CH];           // a slot's control (one 16-byte read per refill)
    __shared__ unsigned short s_n[CH];
    __shared__ uint32_t s_order[CH];     // slot in chunk | parent row << 16
    __shared__ short s_fi[CH];
    __shared__ float s_len[COST == kPATH ? CH : 1];
    __shared__ float s_pe[3][CH];        // end position of valid slots
    __shared__ uint8_t s_vs[CH];         // ... and the signs of their velocity (bit a: v_a >= 0)
    __shared__ int s_pid[kParMax];        // the chunk's parents: tree index
    __shared__ uint32_t s_pcost[kParMax]; //                     cost field
    constexpr int VI = DYN == kQUAD12 ? 6 : 3;  // first velocity component
    __shared__ int s_bin[kSortBins];
    __shared__ float s_os[2][D];
    const int gbp = (P.gb_cells + 1) & ~1;  // grid cells, padded to whole 16-byte words
    float4* sbox = dyn_lds;
    // parent states, one row of SD floats per parent, already in integration units
    float* spx = reinterpret_cast<float*>(dyn_lds + 2 * P.n_boxes);
    int2* sgc = reinterpret_cast<int2*>(spx + SD * kParMax);
    uint16_t* sgl = reinterpret_cast<uint16_t*>(sgc + gbp);

    // the obstacle data does not depend on the device state: its loads go
    // out together with the state's
    stage_lds(reinterpret_cast<int4*>(dyn_lds), reinterpret_cast<const int4*>(T.boxes), 0, 2 * P.n_boxes,
              reinterpret_cast<const int4*>(T.gcell), (int)(reinterpret_cast<float4*>(sgc) - dyn_lds), gbp / 2,
              reinterpret_cast<const int4*>(T.glist), (int)(reinterpret_cast<float4*>(sgl) - dyn_lds),
              (P.gb_entries + 7) / 8);
    const int K = st->k;
    const int S = st->n_sel * K;
    if (st->full || S == 0) return;  // kernel-uniform
    int chunk = max(kChunkMin, (S + nblk - 1) / nblk);
    // at most kParMax parents per chunk (K may be up to the buffer size: 64-bit)
    chunk = (int)min((long long)chunk, min((long long)CH, (long long)(kParMax - 1) * K));
    if (blk * chunk >= S) return;  // block-uniform
    if (blk == 0 && threadIdx.x == 0) T.stats[st->it & (kStatsCap - 1)].t_begin = wall_clock64();
    const long long n_tree = st->n_tree;
    const uint32_t it = (uint32_t)st->it;
    if (threadIdx.x < D) {
        s_os[0][threadIdx.x] = P.os_lo[threadIdx.x];
        s_os[1][threadIdx.x] = P.os_hi[threadIdx.x];
    }
    const Hot<DYN> H = make_hot<DYN>(P);
    const int lane = threadIdx.x & 63;
    int my_valid = 0;
    unsigned long long my_steps = 0;  // substeps of this lane's slots (64-bit: up to 2^28 slots of 32767 steps)

    for (int base = blk * chunk; base < S; base += nblk * chunk) {
        const int cnt = min(chunk, S - base);
        const int r0 = base / K;
        const int npar = (base + cnt - 1) / K - r0 + 1;
        // the sort bins are free once the previous chunk has left its
        // integration loop
        if (threadIdx.x < kSortBins) s_bin[threadIdx.x] = 0;
        __syncthreads();  // LDS of the previous chunk is free
        // 1. parents (tree index, cost, state) into LDS, samples, sort by step
        // count (longest first).  The parent loads are issued before the
        // sampling so that their latency overlaps it.
        // (Indexes past the end are clamped rather than branched on, so that
        // each group of loads leaves together.)
        constexpr int kStage = 4;
        const int nstage = npar * D;
        int prow[kStage];
        float pv[kStage];
#pragma unroll
        for (int r = 0; r < kStage; ++r) {
            const int idx = min((int)threadIdx.x + r * NT, nstage - 1);
            prow[r] = T.sel[r0 + idx % npar];
        }
        const int my_pid = T.sel[r0 + min((int)threadIdx.x, npar - 1)];
#pragma unroll
        for (int r = 0; r < kStage; ++r) {
            const int idx = min((int)threadIdx.x + r * NT, nstage - 1);
            pv[r] = T.x[(long long)(idx / npar) * P.cap + prow[r]];
        }
        const uint32_t my_pcost = T.cost[my_pid];
        const bool one_each = cnt <= NT;  // one slot per thread: no sort needed
        const int nr = (cnt + NT - 1) / NT;  // slot rounds of this chunk
        int bins[PT];
#pragma unroll
        for (int r = 0; r < PT; ++r) {
            if (r >= nr) break;  // block-uniform
            const int li = threadIdx.x + r * NT;
            bins[r] = -1;
            if (li < cnt) {
                float u[M];
                int n;
                sample<DYN>(P, it, (uint32_t)(base + li), u, n);
                float u3 = 0.f;
                if constexpr (M > 3) u3 = u[3];
                s_u[li] = make_float4(u[0], u[1], u[2], u3);
                s_n[li] = (unsigned short)n;
                bins[r] = (kSortBins - 1) - min(kSortBins - 1, (n - P.steps_min) >> P.sort_shift);
                if (one_each) s_order[li] = (uint32_t)li | (uint32_t)((base + li) / K - r0) << 16;
                else atomicAdd(&s_bin[bins[r]], 1);
            }
        }
        // staged parent component c of row j: x_c in integration units
        auto stage_x = [&](int idx, float v) {
            const int c = idx / npar, j = idx % npar;
            spx[j * SD + c] = v * (rev_state(DYN, c) ? kInv2Pi : 1.f);
        };
#pragma unroll
        for (int r = 0; r < kStage; ++r) {
            const int idx = threadIdx.x + r * NT;
            if (idx < nstage) stage_x(idx, pv[r]);
        }
        for (int idx = threadIdx.x + kStage * NT; idx < nstage; idx += NT)
            stage_x(idx, T.x[(long long)(idx / npar) * P.cap + T.sel[r0 + idx % npar]]);
        if ((int)threadIdx.x < npar) {
            s_pid[threadIdx.x] = my_pid;
            s_pcost[threadIdx.x] = my_pcost;
        }
        __syncthreads();
        if (!one_each) {  // block-uniform: counting sort of the queue, longest first
            if (threadIdx.x < 64)  // exclusive prefix over the 64 bins in one wave
                s_bin[threadIdx.x] = wave_exclusive_scan(s_bin[threadIdx.x]);
            __syncthreads();
#pragma unroll
            for (int r = 0; r < PT; ++r) {
                if (r >= nr) break;
                if (bins[r] >= 0)
                    s_order[atomicAdd(&s_bin[bins[r]], 1)] =
                        (uint32_t)(threadIdx.x + r * NT) |
                        (uint32_t)((base + (int)threadIdx.x + r * NT) / K - r0) << 16;
            }
            __syncthreads();
        }

        // 2. integrate, each lane refilling from the queue.  Wave w of the
        // block owns queue places w, w + NW, w + 2 NW, ... (the sorted order
        // dealt out round-robin, so every wave gets long and short edges
        // alike) and counts its own places, so a refill needs no atomic.
        constexpr int NW = NT / 64;
        const int wid = (int)threadIdx.x >> 6;
        float x[D], u[M];
        // a parent's staged state into x: 16-byte LDS reads
        auto load_parent = [&](int j) {
            const float4* r = reinterpret_cast<const float4*>(spx + j * SD);
#pragma unroll
            for (int w = 0; w < SD / 4; ++w) {
                const float4 v = r[w];
                const float a[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (4 * w + e < D) x[4 * w + e] = a[e];
            }
        };
        float len = 0.f;
        int li = -1, n = 0, k = 0;
        int pjl = 0;                        // the lane's parent row
        bool chk = !CF, pend = false;       // obstacle test on; table value in flight
        unsigned long long ckey = 0, ctv = 0;
        int gcur = -1, gstart = 0, gcount = 0;
        float gclr = 0.f;
        // safe ball: no box is within sqrt(r2) of (rx, ry, rz), the last
        // position whose grid cell was looked up
        float rx = 0.f, ry = 0.f, rz = 0.f, r2 = -1.f;
        int wtaken = 0;  // wave-uniform: queue places of this wave taken so far
        bool exhausted = wid >= cnt;  // wave-uniform: no place left for this wave
        while (true) {
            // idle lanes refill together, once a quarter of the wave waits
            // (an eighth in 512-thread blocks) or no lane integrates: a
            // refill's LDS round trips then cost the wave a few trips instead
            // of one per finished edge, and the longest edges, which set the
            // block's time, do not wait for them
            constexpr int kBatch = NT == kPropBlock ? kRefillBatch : kRefillBatchWide;
            const bool want = li < 0 && !exhausted;
            const unsigned long long m = __ballot(want);
            if (m && (__popcll(m) >= kBatch || !__any(li >= 0))) {
                const int qi = wtaken + __popcll(m & __lanemask_lt());
                wtaken += __popcll(m);
                if (wtaken * NW + wid >= cnt) exhausted = true;
                if (want) {
                    const int q = qi * NW + wid;
                    if (q < cnt) {
                        const uint32_t o = s_order[q];
                        li = (int)(o & 0xFFFFu);
                        const int pj = (int)(o >> 16);
                        n = s_n[li];
                        const float4 uv = s_u[li];
                        const float ua[4] = {uv.x, uv.y, uv.z, uv.w};
                        edge_controls<DYN>(H, ua, u);
                        load_parent(pj);
                        k = 0;
                        len = 0.f;
                        gcur = -1;
                        r2 = -1.f;
                        pjl = pj;
                        chk = !CF;
                        pend = false;
                    }
                }
            }
            if (!__any(li >= 0)) break;
            if (li >= 0) {
                rk4<DYN, COST>(H, x, u, len);
                ++k;
                if constexpr (CF) ++my_steps;  // substeps actually integrated, both passes
                bool ok = in_bounds<DYN>(H, x, s_os[0], s_os[1]);
                const float dx = x[0] - rx, dy = x[1] - ry, dz = x[2] - rz;
                if (ok && chk && __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz)) >= r2) {
                    const int g = box_grid_cell(H, x);
                    if (g != gcur) {
                        const int2 e = sgc[g];
                        gstart = e.x & 0xFFFFF;
                        gcount = e.x >> 20;
                        gclr = __int_as_float(e.y);
                        gcur = g;
                    }
                    // L-infinity distance to each listed box: at most 0 exactly
                    // when the closed box holds the point (the sign of a float
                    // difference is exact); four boxes per round of LDS reads
                    float dmin = __builtin_inff();
                    for (int j = 0; j < gcount; j += 4) {
                        int bi[4];
#pragma unroll
                        for (int t = 0; t < 4; ++t) bi[t] = sgl[gstart + min(j + t, gcount - 1)];
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            const float4 lo = sbox[2 * bi[t]], hi = sbox[2 * bi[t] + 1];
                            const float d = __builtin_fmaxf(
                                __builtin_fmaxf(__builtin_fmaxf(lo.x - x[0], lo.y - x[1]), lo.z - x[2]),
                                __builtin_fmaxf(__builtin_fmaxf(x[0] - hi.x, x[1] - hi.y), x[2] - hi.z));
                            dmin = __builtin_fminf(dmin, d);
                        }
                    }
                    ok = dmin > 0.f;
                    // the ball: the distance to the nearest box, shrunk for the
                    // float rounding of the distances compared against it
                    const float r = __builtin_fminf(gclr, dmin);
                    rx = x[0];
                    ry = x[1];
                    rz = x[2];
                    r2 = r * r * 0.99998f;
                }
                if constexpr (CF) {
                    if (pend) {  // the region's key, loaded one trip ago
                        pend = false;
                        if (ckey > ctv) {
                            s_fi[li] = kSkipped;
                            li = -1;
                        }
                    }
                    if (li >= 0 && !chk && ok && k == n) {
                        // first pass within bounds: the edge's region and key
                        const float pe[3] = {x[0], x[1], x[2]};
                        const float ve[3] = {x[VI], x[VI + 1], x[VI + 2]};
                        const int c = cell_of(P, pe, ve);
                        uint32_t cf;
                        if constexpr (COST == kTIME) cf = s_pcost[pjl] + (uint32_t)n;
                        else cf = __float_as_uint(__uint_as_float(s_pcost[pjl]) + len);
                        ckey = ((unsigned long long)cf << 32) | (unsigned long long)(uint32_t)(n_tree + base + li);
                        ctv = __hip_atomic_load(&T.tbl[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        pend = true;
                        chk = true;
                        load_parent(pjl);
                        k = 0;
                        len = 0.f;
                        gcur = -1;
                        r2 = -1.f;
                    }
                }
                if (li >= 0 && (!ok || k == n)) {
                    s_fi[li] = (short)(ok ? 0 : k);
                    if (ok) {
                        if constexpr (COST == kPATH) s_len[li] = len;
#pragma unroll
                        for (int a = 0; a < 3; ++a) s_pe[a][li] = x[a];
                        s_vs[li] = (uint8_t)((x[VI] >= 0.f) | (x[VI + 1] >= 0.f) << 1 | (x[VI + 2] >= 0.f) << 2);
                        float4* cr = reinterpret_cast<float4*>(T.cx) + (long long)(base + li) * (SD / 4);
#pragma unroll
                        for (int w = 0; w < SD / 4; ++w) {
                            float v[4];
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const int c = 4 * w + e;
                                v[e] = c < D ? x[c] * (rev_state(DYN, c) ? k2Pi : 1.f) : 0.f;
                            }
                            cr[w] = make_float4(v[0], v[1], v[2], v[3]);
                        }
                    }
                    li = -1;
                }
            }
        }
        __syncthreads();

        // 3. region map, cost, region minimum, candidate records.  A valid
        // slot first reads its region's entry and takes the atomic minimum
        // only when its key is below the value read: the entry only falls
        // while propagate runs, so a key at or above it can neither become
        // the minimum nor beat the region's node.  Regions that many edges
        // reach at once (the root's neighbours when the root alone shares a
        // large buffer) then see few atomics instead of one per edge.  A
        // thread issues all its loads, then all its atomics, before it looks
        // at their results, so that the round trips overlap.
        unsigned long long keys[PT], olds[PT];
        int cells[PT];
        bool beaten[PT];  // a lower key of this chunk reaches the same region
#pragma unroll
        for (int r = 0; r < PT; ++r) {
            if (r >= nr) break;  // block-uniform
            const int lj = threadIdx.x + r * NT;
            keys[r] = kEmpty;
            olds[r] = kEmpty;
            cells[r] = 0;
            beaten[r] = false;
            if (lj >= cnt) continue;
            const int s = base + lj;
            const int fi = s_fi[lj];
            const int nn = s_n[lj];
            // the survivor byte and the chunk's tile counts start the
            // iteration at zero (prune marks the survivors)
            T.csurv[s] = 0;
            if ((s & (kTile - 1)) == 0) T.tile_count[s / kTile] = 0;
            const int pj = s / K - r0;
            if constexpr (!CF) my_steps += fi ? fi : nn;
            if (fi == 0) {
                ++my_valid;
                const float pe[3] = {s_pe[0][lj], s_pe[1][lj], s_pe[2][lj]};
                // the velocity enters the region only through its signs
                const int vs = s_vs[lj];
                const float ve[3] = {vs & 1 ? 1.f : -1.f, vs & 2 ? 1.f : -1.f, vs & 4 ? 1.f : -1.f};
                const int c = cell_of(P, pe, ve);
                uint32_t cf;
                if constexpr (COST == kTIME) {
                    cf = s_pcost[pj] + (uint32_t)nn;
                } else {
                    cf = __float_as_uint(__uint_as_float(s_pcost[pj]) + s_len[lj]);
                }
                const unsigned long long key =
                    ((unsigned long long)cf << 32) | (unsigned long long)(uint32_t)(n_tree + s);
                keys[r] = key;
                cells[r] = c;
                T.ckey[s] = key;
                T.ccell[s] = c;
                T.cflag[s] = (uint8_t)(1 | (in_goal(P, pe) ? 2 : 0));
            } else {
                T.ckey[s] = kEmpty;
                T.ccell[s] = -1;
                T.cflag[s] = 0;
            }
            if (T.d_parent) {
                T.d_parent[s] = s_pid[pj];
#pragma unroll
                for (int q = 0; q < M; ++q) {
                    const float4 uv = s_u[lj];
                    T.d_u[(long long)q * P.s_max + s] = q == 0 ? uv.x : q == 1 ? uv.y : q == 2 ? uv.z : uv.w;
                }
                T.d_n[s] = nn;
                T.d_fi[s] = fi;
            }
        }
        if (K >= kDedupK) {  // block-uniform
            // The chunk's lowest key per region, in an LDS table of CH
            // buckets (region in the freed sort order, key in the freed
            // controls).  A slot whose region lost its bucket to another
            // region goes to the region table as it is.  A slot beaten by a
            // lower key of the chunk in its region can neither be the
            // region's minimum nor the first to beat the region's node.
            uint32_t* s_hcell = s_order;
            unsigned long long* s_hkey = reinterpret_cast<unsigned long long*>(s_u);
            __syncthreads();  // every read of s_u above is done
            for (int i = threadIdx.x; i < CH; i += NT) {
                s_hcell[i] = 0xFFFFFFFFu;
                s_hkey[i] = kEmpty;
            }
            __syncthreads();
            int hb[PT];
#pragma unroll
            for (int r = 0; r < PT; ++r) {
                hb[r] = -1;
                if (r >= nr || keys[r] == kEmpty) continue;
                const uint32_t c = (uint32_t)cells[r];
                constexpr int kHashShift = CH == kChunkBig ? 21 : 22;  // 11 or 10 bits: CH buckets
                const int h = (int)((c * 2654435761u) >> kHashShift);
                const uint32_t prev = atomicCAS(&s_hcell[h], 0xFFFFFFFFu, c);
                if (prev == 0xFFFFFFFFu || prev == c) {
                    atomicMin(&s_hkey[h], keys[r]);
                    hb[r] = h;
                }
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < PT; ++r)
                if (hb[r] >= 0 && s_hkey[hb[r]] != keys[r]) beaten[r] = true;
        }
#pragma unroll
        for (int r = 0; r < PT; ++r) {
            if (r >= nr) break;
            if (keys[r] != kEmpty && !beaten[r])
                olds[r] = __hip_atomic_load(&T.tbl[cells[r]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
#pragma unroll
        for (int r = 0; r < PT; ++r) {
            if (r >= nr) break;
            if (!beaten[r] && keys[r] < olds[r]) olds[r] = atomicMin(&T.tbl[cells[r]], keys[r]);
        }
#pragma unroll
        for (int r = 0; r < PT; ++r) {
            if (r >= nr) break;
            const unsigned long long key = keys[r], old = olds[r];
            if (!beaten[r] && key < old && old != kEmpty && (long long)(uint32_t)old < n_tree) {
                // this lane took the region from a tree node: it is beaten (V_T)
                const uint32_t o = (uint32_t)old;
                T.status[o] = kTerminal;
                T.dead[o] = 1;
            }
        }
    }
    const int wv = wave_sum(my_valid);
    const unsigned long long ws = wave_sum64(my_steps);
    if (lane == 0) {
        if (wv) atomicAdd(&st->n_valid_acc, wv);
        if (ws) atomicAdd(&st->substeps_acc, (unsigned long long)ws);
    }
}

template <int DYN, int COST, bool CF, int NT, int CH = kChunkMax>
__global__ __launch_bounds__(NT) void k_propagate(DevProblem P, DevPtrs T, DevState* st)
{
    propagate_body<DYN, COST, CF, NT, CH>(P, T, st, blockIdx.x, gridDim.x);
}

// ------------------------------------------------------------------ prune + survivor flags

// One block per region block of RPT x kBlock regions: thread t of block b
// holds regions c = b RPT kBlock + j kBlock + t (j < RPT), so that each slice
// j is read coalesced and the block's regions keep their order slice by slice.
template <int RPT>
__device__ __forceinline__ void prune_flags_body(const DevProblem& P, const DevPtrs& T, DevState* st,
                                                 int blk, int n_prune_blocks)
{
    __shared__ int s_w[kBlock / 64], s_w2[kBlock / 64], s_w3[kBlock / 64];
    if (blk >= n_prune_blocks) return;
    // Alg. 3 for the owner of each region (every live node owns its region);
    // also records whether the region's node is active after this iteration,
    // and per block the active regions on either side of the selection
    // cursor.  A region an arrival took marks that slot the survivor (its key
    // is the region's minimum) and counts it in its 256-slot tile, for the
    // ranks insert gives the survivors.
    const int base = blk * kBlock * RPT + (int)threadIdx.x;
    unsigned long long key[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) key[j] = T.tbl[min(base + j * kBlock, P.n_cells - 1)];
    const int full = st->full, cur = st->cursor_next;
    const long long n_tree = st->n_tree;
    if (full) return;  // kernel-uniform
    uint8_t a[RPT], s[RPT];
    bool owned[RPT];  // a tree node owns the region
    int ic0[RPT];
    uint32_t o[RPT];
    int4 A[RPT], B[RPT];
    // every owner's status, count and first ancestor list in one round trip;
    // lanes without an owner read node 0's (one line for the wave) rather than
    // branch, so that no load waits for another
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int c = base + j * kBlock;
        a[j] = 0;
        o[j] = (uint32_t)key[j];
        const bool taken = c < P.n_cells && key[j] != kEmpty;
        owned[j] = taken && (long long)o[j] < n_tree;
        const uint32_t on = owned[j] ? o[j] : 0u;
        s[j] = T.status[on];
        ic0[j] = T.icount[on];
        A[j] = T.anc[2 * (size_t)on];
        B[j] = T.anc[2 * (size_t)on + 1];
        if (taken && !owned[j]) {
            // an arrival of this iteration owns it: that slot is the region's
            // survivor (V_U, the App. A U-filter), inserted active
            a[j] = 1;
            const int sv = (int)((long long)o[j] - n_tree);
            T.csurv[sv] = 1;
            atomicAdd(&T.tile_count[sv / kTile], 1);
            if (grouped(P.n_tgroups)) atomicAdd(tgroup_at(T, P, (int)(st - T.st), sv / kTile / kGroup), 1);
        }
    }
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        if (!owned[j]) continue;
        uint8_t sj = s[j];
        if (sj == kInactive) {  // Alg. 3: a dormant node counts up and wakes past I_max
            const int ic = ic0[j] + 1;
            T.icount[o[j]] = (uint8_t)ic;
            if (ic > P.i_max) {
                sj = kActive;
                T.status[o[j]] = kActive;
            }
        } else if (sj == kActive && ic0[j] <= P.i_max) {
            // Alg. 3: any ancestor beaten in its region (or below one); eight
            // ancestors per step from the stored lists, the next list fetched
            // together with this step's flags (a missing ancestor, -1, reads
            // node 0's and is masked, so the step's loads share one round trip)
            int4 Aj = A[j], Bj = B[j];
            bool beaten = false;
            while (true) {
                const int ids[8] = {Aj.x, Aj.y, Aj.z, Aj.w, Bj.x, Bj.y, Bj.z, Bj.w};
                uint8_t d[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) d[q] = T.dead[max(ids[q], 0)];
                const int nq = ids[7];
                const size_t nqc = (size_t)max(nq, 0);
                const int4 NA = T.anc[2 * nqc], NB = T.anc[2 * nqc + 1];
#pragma unroll
                for (int q = 0; q < 8; ++q) beaten |= ids[q] >= 0 && d[q] != 0;
                if (beaten || nq < 0) break;
                Aj = NA;
                Bj = NB;
            }
            if (beaten) {
                sj = kInactive;
                T.status[o[j]] = kInactive;
                T.dead[o[j]] = 1;
            }
        }  // Alg. 3: a woken region-best node is left alone
        a[j] = sj == kActive;
    }
    int hi = 0, lo = 0, ow = 0;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int c = base + j * kBlock;
        if (c < P.n_cells) T.act[c] = a[j];
        hi += __popcll(__ballot(a[j] && c >= cur));
        lo += __popcll(__ballot(a[j] && c < cur));
        ow += __popcll(__ballot(owned[j]));
    }
    if ((threadIdx.x & 63) == 0) {
        s_w[threadIdx.x >> 6] = hi;
        s_w2[threadIdx.x >> 6] = lo;
        s_w3[threadIdx.x >> 6] = ow;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int th = 0, tl = 0, to = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) {
            th += s_w[w];
            tl += s_w2[w];
            to += s_w3[w];
        }
        T.bcount[blk] = make_int2(th, tl);
        if (to) atomicAdd(&st->n_live_acc, to);
        if (grouped(P.n_bgroups)) {
            int2* g = bgroup_at(T, P, (int)(st - T.st), blk / kGroup);
            if (th) atomicAdd(&g->x, th);
            if (tl) atomicAdd(&g->y, tl);
        }
    }
}

template <int RPT>
__global__ __launch_bounds__(kBlock) void k_prune_flags(DevProblem P, DevPtrs T, DevState* st,
                                                        int n_prune_blocks)
{
    prune_flags_body<RPT>(P, T, st, blockIdx.x, n_prune_blocks);
}

// Exclusive scan of two ints per thread over the block, with the totals.
// One barrier: each thread then sums the wave totals below its own wave.
// `s_w` holds 2 x 16 ints (at most 1024 threads).
__device__ __forceinline__ void block_scan2(int (&v)[2], int (&ex)[2], int (&tot)[2], int (*s_w)[16])
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int inc[2] = {v[0], v[1]};
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int y = __shfl_up(inc[k], o);
            if (lane >= o) inc[k] += y;
        }
    }
    if (lane == 63) {
#pragma unroll
        for (int k = 0; k < 2; ++k) s_w[k][wid] = inc[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        int below = 0, all = 0;
        for (int w = 0; w < nw; ++w) {
            const int t = s_w[k][w];
            below += w < wid ? t : 0;
            all += t;
        }
        ex[k] = below + inc[k] - v[k];
        tot[k] = all;
    }
}

// Selects the nodes of the pending iteration (after create, and again after
// a refinement): regions whose owner is active, in region order rotated to
// start at the cursor, at most n_select.  One block; each thread owns a run of
// whole 4-region words of the activity bytes (0/1, zero-padded past the last
// region).  The two cursor-split counts of active regions share one block scan.
__device__ void select_one_block(const DevProblem& P, const DevPtrs& T, DevState* st, DevState& q,
                                 int (*s_w)[16], int* s_sel)
{
    // every load of the block is in flight before the first barrier
    const int nwords = (P.n_cells + 3) >> 2;
    const int per = (nwords + (int)blockDim.x - 1) / (int)blockDim.x;
    const int w0 = min((int)threadIdx.x * per, nwords);
    const int w1 = min(w0 + per, nwords);
    const uint32_t* act = reinterpret_cast<const uint32_t*>(T.act);
    uint32_t wd[kSelWords];
#pragma unroll
    for (int i = 0; i < kSelWords; ++i) wd[i] = act[min(w0 + i, nwords - 1)];
    if (threadIdx.x == 0) q = *st;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kSelWords; ++i) wd[i] = w0 + i < w1 ? wd[i] & 0x01010101u : 0u;
    const bool in_regs = per <= kSelWords;
    const bool full = q.full != 0;
    const int cur = q.cursor;
    int v[2] = {0, 0};  // active regions at / after the cursor; before it
    auto count = [&](uint32_t w, int c0) {
        const int k = min(max(cur - c0, 0), 4);  // bytes of this word before the cursor
        const uint32_t below = k == 4 ? ~0u : (1u << (8 * k)) - 1u;
        v[1] += __popc(w & below);
        v[0] += __popc(w & ~below);
    };
    if (in_regs) {
#pragma unroll
        for (int i = 0; i < kSelWords; ++i) count(wd[i], 4 * (w0 + i));
    } else {
        for (int w = w0; w < w1; ++w) count(act[w] & 0x01010101u, 4 * w);
    }
    int ex[2], tot[2];
    block_scan2(v, ex, tot, s_w);
    const int nsel = full ? 0 : min(tot[0] + tot[1], P.n_select);
    // ranks: regions at or after the cursor first, then those before it
    int r_hi = ex[0], r_lo = tot[0] + ex[1];
    auto rank = [&](uint32_t w, int c0) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int a = (int)((w >> (8 * b)) & 1u);
            const int c = c0 + b;
            const bool h = c >= cur;
            const int rk = h ? r_hi : r_lo;
            if (a && rk < nsel) {
                if (nsel <= kSelLds) s_sel[rk] = c;
                else T.sel[rk] = c;
                if (rk == nsel - 1) q.cursor_next = (c + 1 == P.n_cells) ? 0 : c + 1;
            }
            r_hi += a & (int)h;
            r_lo += a & (int)!h;
        }
    };
    if (nsel > 0) {
        if (in_regs) {
#pragma unroll
            for (int i = 0; i < kSelWords; ++i) rank(wd[i], 4 * (w0 + i));
        } else {
            for (int w = w0; w < w1; ++w) rank(act[w] & 0x01010101u, 4 * w);
        }
    }
    __syncthreads();
    // owners: the low word of each selected region's key; four loads in flight per thread
    const uint32_t* tbl_lo = reinterpret_cast<const uint32_t*>(T.tbl);
    const int bd = blockDim.x;
    for (int r0 = threadIdx.x; r0 < nsel; r0 += 4 * bd) {
        int cc[4];
        uint32_t o[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int r = r0 + k * bd;
            cc[k] = r < nsel ? (nsel <= kSelLds ? s_sel[r] : T.sel[r]) : -1;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) o[k] = cc[k] >= 0 ? tbl_lo[2 * (size_t)cc[k]] : 0u;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (cc[k] >= 0) T.sel[r0 + k * bd] = (int)o[k];
    }
    if (threadIdx.x == 0) {
        q.n_sel = nsel;
        q.k = samples_for(P, nsel);
        if (nsel == 0 && !full) q.cursor_next = cur;
        q.n_surv = 0;
        *st = q;
    }
}

__global__ __launch_bounds__(kSelectThreads) void k_select(DevProblem P, DevPtrs T, DevState* st)
{
    __shared__ int s_w[2][16];
    __shared__ int s_sel[kSelLds];
    __shared__ DevState s_st;
    select_one_block(P, T, st, s_st, s_w, s_sel);
}

// ------------------------------------------------------------------ insert

// App. A UpdateTree: survivors appended at |T| + rank (exclusive scan of V_U).
// Every load that does not depend on another is issued first (the state, the
// counts of the earlier tiles, this slot's survivor mark and its parent), then
// a survivor's candidate record, end state and parent's ancestor lists; one
// barrier gives each survivor its rank while those are in flight.
template <int DYN>
__device__ __forceinline__ void insert_body(const DevProblem& P, const DevPtrs& T, DevState* st, int blk)
{
    constexpr int D = Dims<DYN>::D, M = Dims<DYN>::M;
    __shared__ int s_w[2][kBlock / 64];
    const int tile = blk;
    const int s = tile * kTile + threadIdx.x;
    const int sc = min(s, P.s_max - 1);
    // survivors before this tile: the earlier tiles (of its group, when the
    // counts are grouped), four per thread first
    const bool grp = grouped(P.n_tgroups);
    const int g0 = grp ? tile / kGroup * kGroup : 0;
    int pre = 0;
#pragma unroll
    for (int u = 0; u < kGroup / kBlock; ++u) {
        const int j = g0 + threadIdx.x + u * kBlock;
        const int v = T.tile_count[min(j, max(tile - 1, 0))];
        pre += j < tile ? v : 0;
    }
    const uint8_t f0 = T.csurv[sc];
    const int K = P.K > 0 ? P.K : st->k;
    // With a small slot buffer every slot's parent is read with its survivor
    // mark (a node's K slots share one entry), so that the parent's ancestor
    // lists need no third round trip; with a large one the per-slot division
    // and reads would cost more than that round trip, and only survivors read
    // theirs (uniform).
    const bool early = P.s_max <= kInsertEarlyParents;
    const int par0 = early ? T.sel[sc / max(K, 1)] : 0;
    const int full = st->full, n_sel = st->n_sel;
    const long long n_tree = st->n_tree;
    const uint32_t it = (uint32_t)st->it;
    if (full) return;  // kernel-uniform: nothing happens in a full tree
    const int S = n_sel * K;
    if (tile * kTile >= S) return;  // block-uniform
    for (int j = g0 + threadIdx.x + kGroup; j < tile; j += kBlock) pre += T.tile_count[j];
    if (grp)  // the earlier groups
        for (int j = threadIdx.x; j < tile / kGroup; j += kBlock) pre += *tgroup_at(T, P, (int)(st - T.st), j);
    const int f = s < S ? f0 : 0;
    const unsigned long long fm = __ballot(f);
    // a survivor's candidate cost, region and flags, end state and parent's
    // ancestor lists, in flight while the ranks are scanned.  In a wave that
    // holds a survivor the other lanes read slot 0 and node 0 (one line for
    // the wave) rather than branch, so that nothing waits for these loads
    // before the barrier; a wave without one (most of them, when survivors
    // are sparse) reads nothing (a wave-uniform branch).
    constexpr int SD = cx_row(D);
    uint32_t cf, flag;
    int c, par;
    float4 xr[SD / 4];
    int4 pa, pb;
    if (fm) {
        const int sl = f ? s : 0;
        par = f ? par0 : 0;
        if (!early && f) par = T.sel[s / K];
        cf = reinterpret_cast<const uint32_t*>(T.ckey)[2 * (size_t)sl + 1];
        c = T.ccell[sl];
        flag = T.cflag[sl];
        const float4* cr = reinterpret_cast<const float4*>(T.cx) + (long long)sl * (SD / 4);
#pragma unroll
        for (int w = 0; w < SD / 4; ++w) xr[w] = cr[w];
        pa = T.anc[2 * (size_t)par];
        pb = T.anc[2 * (size_t)par + 1];
    }
    // rank = survivors of the earlier tiles + those before this slot in its
    // tile (a ballot of the marks: the survivors before this lane in its wave)
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int wpre = wave_sum_rows(pre);
    if (lane == 0) {
        s_w[0][wid] = __popcll(fm);
        s_w[1][wid] = wpre;
    }
    __syncthreads();
    int rank = __popcll(fm & __lanemask_lt());
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) rank += (w < wid ? s_w[0][w] : 0) + s_w[1][w];
    if (threadIdx.x == 0 && (tile + 1) * kTile >= S) {  // the last tile: the survivor count
        int total = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) total += s_w[0][w] + s_w[1][w];
        st->n_surv = total;
    }
    if (f) {
        const long long i = n_tree + rank;
        float xv[SD];
#pragma unroll
        for (int w = 0; w < SD / 4; ++w) {
            xv[4 * w] = xr[w].x;
            xv[4 * w + 1] = xr[w].y;
            xv[4 * w + 2] = xr[w].z;
            xv[4 * w + 3] = xr[w].w;
        }
        float u[M];
        int n;
        sample<DYN>(P, it, (uint32_t)s, u, n);
#pragma unroll
        for (int q = 0; q < D; ++q) T.x[(long long)q * P.cap + i] = xv[q];
#pragma unroll
        for (int q = 0; q < M; ++q) T.u[(long long)q * P.cap + i] = u[q];
        T.anc[2 * i] = make_int4(par, pa.x, pa.y, pa.z);
        T.anc[2 * i + 1] = make_int4(pa.w, pb.x, pb.y, pb.z);
        T.steps[i] = (uint16_t)n;
        T.parent[i] = par;
        T.cost[i] = cf;
        T.cell[i] = c;
        T.status[i] = kActive;
        T.icount[i] = 0;
        T.dead[i] = 0;
        const unsigned long long nk = ((unsigned long long)cf << 32) | (unsigned long long)(uint32_t)i;
        T.tbl[c] = nk;
        // (an opaque copy, so that the compiler does not test the flag, and
        // wait for its load, before the barrier)
        asm volatile("" : "+v"(flag));
        if (flag & 2) atomicMin(&st->sol, nk);  // Alg. 4: a goal node competes for the solution
    }
}

template <int DYN>
__global__ __launch_bounds__(kBlock) void k_insert(DevProblem P, DevPtrs T, DevState* st)
{
    insert_body<DYN>(P, T, st, blockIdx.x);
}

// Edge polish of the nodes this iteration inserted (QUAD12, TIME cost), an
// extension past the paper: each node's control takes `steps` projected
// gradient steps u <- clamp(u - lr grad L(u, u, u, u), U) on the tied loss of
// kpx_diff_device.hpp (grown boxes, goal centre).  The polished edge is then
// integrated as propagate integrates an edge (integration units, closed state
// bounds and boxes after every step) and replaces the node's edge when it is
// valid, ends in the node's region and keeps a goal node in the goal; a node
// that enters the goal competes for the solution.  Region and cost (the step
// count) are unchanged, so no region minimum or status moves.  One thread per
// new node; dynamic LDS: boxes as lo, hi and as centre, half extent, then the
// adjoint's checkpoints and nearest-box records of every thread.
constexpr int kPolishBlock = 64;
constexpr int kPolishCkpt = 8;  // checkpoint blocks: edges of at most 64 steps

size_t polish_lds_bytes(int n_boxes)
{
    return sizeof(float4) * 4 * (size_t)n_boxes + sizeof(float) * kPolishCkpt * 12 * kPolishBlock +
           sizeof(unsigned short) * kPolishCkpt * kpxd::kCkpt * kPolishBlock;
}

template <int COST>
__global__ __launch_bounds__(kPolishBlock) void k_polish(DevProblem P, DevPtrs T, DevState* st, kpxd::DiffConst C,
                                                         int steps, float lr, int goal_only)
{
    extern __shared__ float4 plds[];
    const int nb = P.n_boxes;
    float4* sbox = plds;
    float4* sce = plds + 2 * nb;
    float* sck = reinterpret_cast<float*>(plds + 4 * nb);
    unsigned short* snb = reinterpret_cast<unsigned short*>(sck + kPolishCkpt * 12 * kPolishBlock);
    for (int i = threadIdx.x; i < 2 * nb; i += blockDim.x) sbox[i] = T.boxes[i];
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        const float4 lo = sbox[2 * b], hi = sbox[2 * b + 1];
        sce[2 * b] = make_float4(0.5f * (lo.x + hi.x), 0.5f * (lo.y + hi.y), 0.5f * (lo.z + hi.z), 0.f);
        sce[2 * b + 1] = make_float4(0.5f * (hi.x - lo.x), 0.5f * (hi.y - lo.y), 0.5f * (hi.z - lo.z), 0.f);
    }
    __syncthreads();
    const int K = P.K > 0 ? P.K : st->k;
    if (st->full || st->n_sel * K == 0) return;  // insert wrote no survivor count
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= st->n_surv) return;
    const long long i = st->n_tree + t;
    const int p = T.parent[i];
    const int n = T.steps[i];
    float x0[12], u[4], xo[3];
#pragma unroll
    for (int q = 0; q < 12; ++q) x0[q] = T.x[(long long)q * P.cap + p];
#pragma unroll
    for (int q = 0; q < 4; ++q) u[q] = T.u[(long long)q * P.cap + i];
#pragma unroll
    for (int a = 0; a < 3; ++a) xo[a] = T.x[(long long)a * P.cap + i];
    const bool was_goal = in_goal(P, xo);
    if (goal_only && !was_goal) {  // left as inserted
        if (T.d_pfi) {
            T.d_pfi[t] = 0;
            T.d_pcell[t] = -1;
            T.d_pflag[t] = 0;
        }
        return;
    }
    const int nb_pen = C.w_obst != 0.f ? nb : 0;
    for (int r = 0; r < steps; ++r) {
        float uu[16], gu[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) uu[q] = u[q & 3];
        int unused = 0;
        kpxd::edge_pass(C, sbox, sce, nb_pen, x0, uu, n, sck + threadIdx.x, snb + threadIdx.x, kPolishBlock,
                        true, gu, false, unused);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float g = (gu[c] + gu[4 + c]) + (gu[8 + c] + gu[12 + c]);
            u[c] = fminf(fmaxf(u[c] - lr * g, C.u_lo[c]), C.u_hi[c]);
        }
    }
    // the polished edge as propagate integrates and checks an edge
    const Hot<kQUAD12> H = make_hot<kQUAD12>(P);
    float x[12], ur[4], len = 0.f;
#pragma unroll
    for (int c = 0; c < 12; ++c) x[c] = x0[c] * (rev_state(kQUAD12, c) ? kInv2Pi : 1.f);
    edge_controls<kQUAD12>(H, u, ur);
    bool ok = true;
    int fi = 0;
    for (int k = 1; k <= n && ok; ++k) {
        rk4<kQUAD12, COST>(H, x, ur, len);
        ok = in_bounds<kQUAD12>(H, x, P.os_lo, P.os_hi);
        for (int b = 0; b < nb; ++b) ok = ok && !in_box(sbox + 2 * b, x[0], x[1], x[2]);
        if (!ok) fi = k;
    }
    float xe[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) xe[c] = x[c] * (rev_state(kQUAD12, c) ? k2Pi : 1.f);
    const bool goal_now = ok && in_goal(P, xe);
    const int cell = ok ? cell_of(P, xe, xe + 6) : -1;
    // the path-length cost: the polished edge must also be shorter (its cost
    // formed as propagate forms an arrival's)
    uint32_t cf = T.cost[i];
    bool shorter = true;
    if constexpr (COST == kPATH) {
        const float c_new = __uint_as_float(T.cost[p]) + len;
        shorter = c_new < __uint_as_float(cf);
        cf = __float_as_uint(c_new);
    }
    const bool accept = ok && cell == T.cell[i] && (!was_goal || goal_now) && shorter;
    if (T.d_pfi) {  // the decisions, for the oracle's replay
        T.d_pfi[t] = fi;
        T.d_pcell[t] = cell;
        T.d_pflag[t] = (uint8_t)((accept ? 1 : 0) | (goal_now ? 2 : 0));
    }
    if (!accept) return;
#pragma unroll
    for (int q = 0; q < 12; ++q) T.x[(long long)q * P.cap + i] = xe[q];
#pragma unroll
    for (int q = 0; q < 4; ++q) T.u[(long long)q * P.cap + i] = u[q];
    const unsigned long long key = ((unsigned long long)cf << 32) | (unsigned long long)(uint32_t)i;
    if constexpr (COST == kPATH) {
        // a node inserted this iteration has no descendants: its lower cost
        // re-keys only its own region, which it keeps
        T.cost[i] = cf;
        T.tbl[cell] = key;
    }
    if (goal_now && (!was_goal || COST == kPATH)) atomicMin(&st->sol, key);
}

// Closes the iteration and selects the next iteration's nodes with one block
// per region block of RPT x kBlock regions (the prune kernel's blocks, whose
// counts of active regions on either side of the cursor give each block the
// ranks of its own regions; ballots rank them within the block, slice by
// slice), the block offsets by the two-level scan.  It reads this iteration's state and writes the next one,
// so no block sees another's update; block 0 writes everything but the cursor
// past the last selected region, which the thread holding that rank writes.
// The group sums of the other parity, which the next iteration's prune adds
// to, are cleared here.
template <int RPT>
__device__ __forceinline__ void finalize_select_body(const DevProblem& P, const DevPtrs& T, const DevState* st,
                                                     DevState* st_next, int blk, int nb)
{
    constexpr int NW = kBlock / 64;
    __shared__ int s_r[4][NW];
    __shared__ int s_c[2][RPT][NW];  // per slice and wave: active regions at / after the cursor, before it
    const int b = blk, base = b * kBlock * RPT + (int)threadIdx.x;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    // every load first: this thread's regions and owners, the block counts, the state
    uint8_t act[RPT];
    uint32_t own[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int cc = min(base + j * kBlock, P.n_cells - 1);
        act[j] = T.act[cc];
        own[j] = reinterpret_cast<const uint32_t*>(T.tbl)[2 * (size_t)cc];
    }
    // the block counts summed here: every block's (for the totals too) in one
    // level, or those of this block's group before it when grouped
    const bool grp = grouped(P.n_bgroups);
    const int par = (int)(st - T.st);
    const int g0 = grp ? b / kGroup * kGroup : 0, jend = grp ? b : nb;
    int2 bc[kGroup / kBlock];
#pragma unroll
    for (int k = 0; k < kGroup / kBlock; ++k)
        bc[k] = T.bcount[min(g0 + (int)threadIdx.x + k * kBlock, max(jend - 1, 0))];
    // the whole state in one go (read before any store, which the compiler
    // could not otherwise move these loads across)
    const DevState q = *st;
    const int was_full = q.full, n_sel = q.n_sel, n_surv0 = q.n_surv, cur = q.cursor_next;
    const int k_cur = q.k;
    const long long n_tree = q.n_tree;
    // active regions at / after the cursor and before it: in the blocks before
    // this one, and in all
    int v[4] = {0, 0, 0, 0};
    auto add = [&](int j, int2 t) {
        // selects, not branches: a load whose value only a branch used would
        // be moved into it and waited for there
        const bool in = j < jend, before = in && j < b, all = in && !grp;
        v[0] += before ? t.x : 0;
        v[1] += before ? t.y : 0;
        v[2] += all ? t.x : 0;
        v[3] += all ? t.y : 0;
    };
#pragma unroll
    for (int k = 0; k < kGroup / kBlock; ++k) add(g0 + (int)threadIdx.x + k * kBlock, bc[k]);
    for (int j = g0 + (int)threadIdx.x + kGroup; j < jend; j += kBlock) add(j, T.bcount[j]);
    if (grp) {  // the group sums: all of them for the totals, the earlier ones for the offsets
        const int g = b / kGroup, ng = (nb + kGroup - 1) / kGroup;
        for (int j = threadIdx.x; j < ng; j += kBlock) {
            const int2 t = *bgroup_at(T, P, par, j);
            v[2] += t.x;
            v[3] += t.y;
            if (j < g) {
                v[0] += t.x;
                v[1] += t.y;
            }
        }
    }
    // the other parity's group sums start the next iteration at zero
    if (grouped(P.n_bgroups))
        for (int j = b * kBlock + (int)threadIdx.x; j < P.n_bgroups; j += nb * kBlock)
            *bgroup_at(T, P, par ^ 1, j) = make_int2(0, 0);
    if (grouped(P.n_tgroups))
        for (int j = b * kBlock + (int)threadIdx.x; j < P.n_tgroups; j += nb * kBlock)
            *tgroup_at(T, P, par ^ 1, j) = 0;
    bool a[RPT], h[RPT];
    unsigned long long mh[RPT], ml[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int c = base + j * kBlock;
        a[j] = c < P.n_cells && act[j] != 0;
        h[j] = c >= cur;
        mh[j] = __ballot(a[j] && h[j]);
        ml[j] = __ballot(a[j] && !h[j]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = wave_sum_rows(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) s_r[k][wid] = v[k];
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            s_c[0][j][wid] = __popcll(mh[j]);
            s_c[1][j][wid] = __popcll(ml[j]);
        }
    }
    __syncthreads();
    int HB = 0, LB = 0, HT = 0, LT = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        HB += s_r[0][w];
        LB += s_r[1][w];
        HT += s_r[2][w];
        LT += s_r[3][w];
    }
    const bool finalize = !was_full;
    const int n_surv = finalize && n_sel > 0 ? n_surv0 : 0;
    const bool full = was_full || n_tree + n_surv + P.surv_max > P.cap;
    const int nsel = full ? 0 : min(HT + LT, P.n_select);
    // ranks in region order: the block's earlier slices, then this slice's
    // earlier waves, then the lanes before this one
    int sh = 0, sl = 0;  // active regions of the block's slices before slice j
    const unsigned long long below = __lanemask_lt();
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        int wh = 0, wl = 0, th = 0, tl = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            wh += w < wid ? s_c[0][j][w] : 0;
            wl += w < wid ? s_c[1][j][w] : 0;
            th += s_c[0][j][w];
            tl += s_c[1][j][w];
        }
        if (a[j]) {
            const int c = base + j * kBlock;
            const int rank = h[j] ? HB + sh + wh + __popcll(mh[j] & below)
                                  : HT + LB + sl + wl + __popcll(ml[j] & below);
            if (rank < nsel) {
                T.sel[rank] = (int)own[j];
                if (rank == nsel - 1) st_next->cursor_next = (c + 1 == P.n_cells) ? 0 : c + 1;
            }
        }
        sh += th;
        sl += tl;
    }
    if (b == 0 && threadIdx.x == 0) {
        DevState* o = st_next;
        const long long it = q.it;
        o->sol = q.sol;
        o->full = full ? 1 : 0;
        o->n_sel = nsel;
        o->k = samples_for(P, nsel);
        o->n_surv = 0;
        if (finalize) {
            const long long nt = n_tree + n_surv;
            kpx_iter_stats* r = &T.stats[it & (kStatsCap - 1)];
            r->iteration = it;
            r->n_tree = nt;
            r->n_select = n_sel;
            r->n_valid = q.n_valid_acc;
            r->n_live = q.n_live_acc;
            r->n_survivors = n_surv;
            r->samples_per_node = k_cur;
            r->substeps = (long long)q.substeps_acc;
            r->solution_key = q.sol;
            r->t_end = wall_clock64();
            o->n_tree = nt;
            o->it = it + 1;
            o->first_sol_it = (q.sol != kEmpty && q.first_sol_it < 0) ? it : q.first_sol_it;
            o->last_n_sel = n_sel;
            o->last_k = k_cur;
            o->last_n_valid = q.n_valid_acc;
            o->last_n_surv = n_surv;
            o->last_substeps = (long long)q.substeps_acc;
            o->n_valid_acc = 0;
            o->n_live_acc = 0;
            o->substeps_acc = 0;
            o->cursor = cur;
        } else {
            o->n_tree = n_tree;
            o->it = it;
            o->first_sol_it = q.first_sol_it;
            o->last_n_sel = q.last_n_sel;
            o->last_k = q.last_k;
            o->last_n_valid = q.last_n_valid;
            o->last_n_surv = q.last_n_surv;
            o->last_substeps = q.last_substeps;
            o->n_valid_acc = q.n_valid_acc;
            o->n_live_acc = q.n_live_acc;
            o->substeps_acc = q.substeps_acc;
            o->cursor = q.cursor;
        }
        if (nsel == 0) o->cursor_next = cur;
    }
}

template <int RPT>
__global__ __launch_bounds__(kBlock) void k_finalize_select(DevProblem P, DevPtrs T, const DevState* st,
                                                            DevState* st_next, int nb)
{
    finalize_select_body<RPT>(P, T, st, st_next, blockIdx.x, nb);
}

// ------------------------------------------------------------------ batches of queries

// A batch runs the iterations of independent queries together.  Each launch
// covers the blocks of every query (of one robot model and cost, for the
// kernels that depend on them), and block b finds its query and its place
// among that query's blocks in a map: (query, block, blocks of the query,
// region blocks of the query).  The per-query problems and trees sit in
// device arrays; `par` is the state parity all the queries share.
// The batched kernels read each query's pointers from device memory, where
// the compiler cannot see that they address global memory, and would make
// every access through them a generic one.  Rebuilding each pointer from its
// integer value in the global address space makes them global accesses.
template <typename V>
__device__ __forceinline__ V* as_global(V* p)
{
    return (V*)(__attribute__((address_space(1))) V*)(uintptr_t)p;
}

__device__ __forceinline__ DevPtrs global_ptrs(const DevPtrs& src)
{
    DevPtrs T = src;
    T.x = as_global(T.x);
    T.u = as_global(T.u);
    T.steps = as_global(T.steps);
    T.parent = as_global(T.parent);
    T.cost = as_global(T.cost);
    T.cell = as_global(T.cell);
    T.status = as_global(T.status);
    T.icount = as_global(T.icount);
    T.dead = as_global(T.dead);
    T.anc = as_global(T.anc);
    T.tbl = as_global(T.tbl);
    T.sel = as_global(T.sel);
    T.ckey = as_global(T.ckey);
    T.ccell = as_global(T.ccell);
    T.cx = as_global(T.cx);
    T.cflag = as_global(T.cflag);
    T.csurv = as_global(T.csurv);
    T.tile_count = as_global(T.tile_count);
    T.act = as_global(T.act);
    T.boxes = as_global(T.boxes);
    T.gcell = as_global(T.gcell);
    T.glist = as_global(T.glist);
    T.st = as_global(T.st);
    T.bcount = as_global(T.bcount);
    T.bgroup = as_global(T.bgroup);
    T.tgroup = as_global(T.tgroup);
    T.stats = as_global(T.stats);
    T.d_parent = as_global(T.d_parent);
    T.d_u = as_global(T.d_u);
    T.d_n = as_global(T.d_n);
    T.d_fi = as_global(T.d_fi);
    T.d_pfi = as_global(T.d_pfi);
    T.d_pcell = as_global(T.d_pcell);
    T.d_pflag = as_global(T.d_pflag);
    T.path = as_global(T.path);
    T.path_x = as_global(T.path_x);
    T.path_u = as_global(T.path_u);
    T.path_n = as_global(T.path_n);
    T.path_len = as_global(T.path_len);
    T.x_init = as_global(T.x_init);
    return T;
}

template <int DYN, int COST, int NT>
__global__ __launch_bounds__(NT) void kb_propagate(const DevProblem* __restrict__ Ps,
                                                 const DevPtrs* __restrict__ Ts,
                                                 const int4* __restrict__ map, int par)
{
    const int4 m = map[blockIdx.x];
    const DevPtrs T = global_ptrs(Ts[m.x]);
    propagate_body<DYN, COST, false, NT>(Ps[m.x], T, T.st + par, m.y, m.z);
}

__global__ __launch_bounds__(kBlock) void kb_prune_flags(const DevProblem* __restrict__ Ps,
                                                         const DevPtrs* __restrict__ Ts,
                                                         const int4* __restrict__ map, int par)
{
    const int4 m = map[blockIdx.x];
    const DevPtrs T = global_ptrs(Ts[m.x]);
    prune_flags_body<kRptBatch>(Ps[m.x], T, T.st + par, m.y, m.w);
}

template <int DYN>
__global__ __launch_bounds__(kBlock) void kb_insert(const DevProblem* __restrict__ Ps, const DevPtrs* __restrict__ Ts,
                                                    const int4* __restrict__ map, int par)
{
    const int4 m = map[blockIdx.x];
    const DevPtrs T = global_ptrs(Ts[m.x]);
    insert_body<DYN>(Ps[m.x], T, T.st + par, m.y);
}

__global__ __launch_bounds__(kBlock) void kb_finalize_select(const DevProblem* __restrict__ Ps,
                                                             const DevPtrs* __restrict__ Ts,
                                                             const int4* __restrict__ map, int par)
{
    const int4 m = map[blockIdx.x];
    const DevPtrs T = global_ptrs(Ts[m.x]);
    finalize_select_body<kRptBatch>(Ps[m.x], T, T.st + par, T.st + (par ^ 1), m.y, m.w);
}

// ------------------------------------------------------------------ solution path

template <int DYN>
__global__ void k_extract_path(DevProblem P, DevPtrs T, const DevState* st, int max_nodes)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    constexpr int D = Dims<DYN>::D, M = Dims<DYN>::M;
    const unsigned long long sol = st->sol;
    if (sol == kEmpty) {
        *T.path_len = 0;
        return;
    }
    int len = 0;
    for (int q = (int)(uint32_t)sol; q >= 0; q = T.parent[q]) ++len;
    if (len > max_nodes) {
        *T.path_len = -len;
        return;
    }
    int q = (int)(uint32_t)sol;
    for (int j = len - 1; j >= 0; --j, q = T.parent[q]) T.path[j] = q;
    for (int j = 0; j < len; ++j) {
        const int i = T.path[j];
        for (int k = 0; k < KPX_MAX_STATE; ++k)
            T.path_x[j * KPX_MAX_STATE + k] = k < D ? T.x[(long long)k * P.cap + i] : 0.f;
        for (int k = 0; k < KPX_MAX_CONTROL; ++k)
            T.path_u[j * KPX_MAX_CONTROL + k] = k < M ? T.u[(long long)k * P.cap + i] : 0.f;
        T.path_n[j] = T.steps[i];
    }
    *T.path_len = len;
}

__global__ void k_philox_eval(const uint32_t* in, long long n, uint32_t* out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t c[4] = {in[6 * i], in[6 * i + 1], in[6 * i + 2], in[6 * i + 3]};
    philox10(c, in[6 * i + 4], in[6 * i + 5]);
    for (int k = 0; k < 4; ++k) out[4 * i + k] = c[k];
}

// ------------------------------------------------------------------ host side

int dims_of(int dyn, int* d, int* m)
{
    switch (dyn) {
    case KPX_DI6: *d = 6; *m = 3; return 0;
    case KPX_QUAD12: *d = 12; *m = 4; return 0;
    case KPX_DUBINS6: *d = 6; *m = 3; return 0;
    default: return -1;
    }
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// region blocks of rpt x kBlock regions covering n regions
int region_blocks(long long n, int rpt)
{
    return (int)((n + (long long)kBlock * rpt - 1) / ((long long)kBlock * rpt));
}

struct Sizes {
    int d, m;
    long long cap;
    int n_cells, s_max, n_tiles, n_boxes;
    int n_cells_cap;      // regions the arrays hold: n_cells * refine_max^3
    int n_bgroups;        // groups of kGroup region blocks (of the n_cells_cap regions)
    int n_tgroups;        // groups of kGroup tiles
    int n_act;            // activity bytes, padded to whole words
    int gb_n[3];          // box grid cells per axis
    int gb_entries;       // total list entries of the box grid
};

// all device arrays, in order; the same function sizes and carves them
template <typename F>
void for_each_array(const Sizes& z, F&& f)
{
    const size_t cap = (size_t)z.cap, S = (size_t)z.s_max;
    f("x", sizeof(float) * z.d * cap);
    f("u", sizeof(float) * z.m * cap);
    f("steps", sizeof(uint16_t) * cap);
    f("parent", sizeof(int) * cap);
    f("cost", sizeof(uint32_t) * cap);
    f("cell", sizeof(int) * cap);
    f("status", cap);
    f("icount", cap);
    f("dead", cap);
    f("anc", sizeof(int4) * 2 * cap);
    f("tbl", sizeof(unsigned long long) * (size_t)z.n_cells_cap);
    f("sel", sizeof(int) * S);
    f("ckey", sizeof(unsigned long long) * S);
    f("ccell", sizeof(int) * S);
    f("cx", sizeof(float) * cx_row(z.d) * S);
    f("cflag", S);
    f("csurv", S);
    f("tile_count", sizeof(int) * (size_t)z.n_tiles);
    f("act", (size_t)z.n_act);
    f("boxes", sizeof(float4) * 2 * (size_t)(z.n_boxes > 0 ? z.n_boxes : 1));
    f("gcell", sizeof(int2) * (size_t)z.gb_n[0] * z.gb_n[1] * z.gb_n[2]);
    f("glist", sizeof(uint16_t) * (size_t)(z.gb_entries > 0 ? z.gb_entries : 1));
    f("st", 2 * sizeof(DevState));  // double-buffered by iteration parity
    f("bcount", sizeof(int2) * (size_t)((z.n_cells_cap + kBlock - 1) / kBlock));
    f("bgroup", sizeof(int) * kGroupPad * 2 * (size_t)z.n_bgroups);
    f("tgroup", sizeof(int) * kGroupPad * 2 * (size_t)z.n_tgroups);
    f("stats", sizeof(kpx_iter_stats) * kStatsCap);
    f("d_parent", sizeof(int) * S);
    f("d_u", sizeof(float) * z.m * S);
    f("d_n", sizeof(int) * S);
    f("d_fi", sizeof(int) * S);
    // nodes inserted by one iteration: at most min(regions, slots)
    const size_t SU = std::min(S, (size_t)z.n_cells_cap);
    f("d_pfi", sizeof(int) * SU);
    f("d_pcell", sizeof(int) * SU);
    f("d_pflag", SU);
    f("path", sizeof(int) * kMaxPath);
    f("path_x", sizeof(float) * KPX_MAX_STATE * kMaxPath);
    f("path_u", sizeof(float) * KPX_MAX_CONTROL * kMaxPath);
    f("path_n", sizeof(int) * kMaxPath);
    f("path_len", sizeof(int));
    f("x_init", sizeof(float) * KPX_MAX_STATE);
}

bool finite(float v) { return std::isfinite(v); }

// Box grid: a uniform G^3 grid over the workspace; each grid cell lists the
// boxes (grown by the margin) that overlap it, grown by a small slack so that
// rounding in the device's float32 cell index can never miss a box.  Each cell
// also carries a clearance radius: a lower bound on the distance from any
// point of the (slack-grown) cell to any box that the cell does not list.  A
// point p whose cell was looked up is then at least min(clearance, distance
// to each listed box) from every box, and any later point closer than that
// to p needs no box test.  G is the finest resolution whose cells and lists
// fit the LDS budget.
struct BoxGrid {
    int n[3];
    std::vector<int> cells;     // first entry | count << 20
    std::vector<float> clear;   // clearance radius, rounded down
    std::vector<uint16_t> list;
};

void build_box_grid_at(const kpx_problem* p, int G, BoxGrid* g)
{
    for (int a = 0; a < 3; ++a) g->n[a] = G;
    const size_t nc = (size_t)G * G * G;
    std::vector<std::vector<uint16_t>> per(nc);
    for (int b = 0; b < p->n_boxes; ++b) {
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            const double w0 = p->ws_lo[a], w1 = p->ws_hi[a];
            const double slack = 1e-4 * (w1 - w0);
            const double scale = G / (w1 - w0);
            const double blo = (double)p->boxes[6 * b + a] - p->margin - slack;
            const double bhi = (double)p->boxes[6 * b + 3 + a] + p->margin + slack;
            lo[a] = std::max(0, std::min(G - 1, (int)std::floor((blo - w0) * scale)));
            hi[a] = std::max(0, std::min(G - 1, (int)std::floor((bhi - w0) * scale)));
        }
        for (int i = lo[0]; i <= hi[0]; ++i)
            for (int j = lo[1]; j <= hi[1]; ++j)
                for (int k = lo[2]; k <= hi[2]; ++k) per[((size_t)i * G + j) * G + k].push_back((uint16_t)b);
    }
    g->cells.resize(nc);
    g->list.clear();
    for (size_t c = 0; c < nc; ++c) {
        g->cells[c] = (int)g->list.size() | ((int)per[c].size() << 20);
        g->list.insert(g->list.end(), per[c].begin(), per[c].end());
    }
}

// Clearance of every cell: the distance (double) between the slack-grown cell
// and the nearest margin-grown box it does not list, shrunk by a relative
// 1e-5 and rounded down to float.  Without such a box, FLT_MAX.
void box_grid_clearance(const kpx_problem* p, BoxGrid* g)
{
    const int G0 = g->n[0], G1 = g->n[1], G2 = g->n[2];
    g->clear.assign((size_t)G0 * G1 * G2, 3.4028234663852886e38f);
    if (p->n_boxes == 0) return;
    double lo[3], step[3], slack[3];
    for (int a = 0; a < 3; ++a) {
        const double w = (double)p->ws_hi[a] - p->ws_lo[a];
        lo[a] = p->ws_lo[a];
        step[a] = w / g->n[a];
        slack[a] = 1e-4 * w;
    }
    std::vector<char> listed(p->n_boxes);
    for (int i = 0; i < G0; ++i)
        for (int j = 0; j < G1; ++j)
            for (int k = 0; k < G2; ++k) {
                const size_t c = ((size_t)i * G1 + j) * G2 + k;
                std::fill(listed.begin(), listed.end(), 0);
                const int first = g->cells[c] & 0xFFFFF, count = g->cells[c] >> 20;
                for (int e = 0; e < count; ++e) listed[g->list[first + e]] = 1;
                const int id[3] = {i, j, k};
                double best = INFINITY;
                for (int b = 0; b < p->n_boxes; ++b) {
                    if (listed[b]) continue;
                    double d2 = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        const double c0 = lo[a] + id[a] * step[a] - slack[a];
                        const double c1 = lo[a] + (id[a] + 1) * step[a] + slack[a];
                        const double b0 = (double)p->boxes[6 * b + a] - p->margin;
                        const double b1 = (double)p->boxes[6 * b + 3 + a] + p->margin;
                        const double gap = std::max(0.0, std::max(b0 - c1, c0 - b1));
                        d2 += gap * gap;
                    }
                    best = std::min(best, d2);
                }
                if (!std::isfinite(best)) continue;
                const double r = std::sqrt(best) * (1.0 - 1e-5);
                float rf = (float)r;
                if ((double)rf > r) rf = std::nextafter(rf, 0.f);
                g->clear[c] = rf;
            }
}

size_t box_grid_bytes(const BoxGrid& g)
{
    return sizeof(int2) * g.cells.size() + sizeof(uint16_t) * g.list.size();
}

void build_box_grid(const kpx_problem* p, BoxGrid* g)
{
    if (p->n_boxes == 0) {
        build_box_grid_at(p, 1, g);
    } else {
        for (int G = kBoxGridMax; G >= 1; --G) {
            build_box_grid_at(p, G, g);
            if (box_grid_bytes(*g) <= (size_t)kBoxGridBytes || G == 1) break;
        }
    }
    box_grid_clearance(p, g);
}

// Host-side validation of Problem 1 and the parameters; no GPU call.
int validate(const kpx_problem* p, const kpx_params* q, Sizes* z, std::string* why)
{
    auto bad = [&](const char* msg) {
        if (why) *why = msg;
        return KPX_ERR_ARG;
    };
    if (!p || !q) return bad("NULL problem or params");
    int d, m;
    if (dims_of(p->dynamics, &d, &m)) return bad("unknown dynamics");
    if (p->cost != KPX_COST_TIME && p->cost != KPX_COST_PATH_LENGTH) return bad("unknown cost");
    if (p->n_boxes < 0 || p->n_boxes > KPX_MAX_BOXES) return bad("n_boxes out of range");
    if (p->n_boxes > 0 && !p->boxes) return bad("boxes is NULL");
    for (int b = 0; b < p->n_boxes; ++b)
        for (int a = 0; a < 3; ++a) {
            const float lo = p->boxes[6 * b + a], hi = p->boxes[6 * b + 3 + a];
            if (!finite(lo) || !finite(hi) || lo > hi) return bad("box with lo > hi or non-finite");
        }
    for (int a = 0; a < 3; ++a)
        if (!finite(p->ws_lo[a]) || !finite(p->ws_hi[a]) || !(p->ws_lo[a] < p->ws_hi[a]))
            return bad("workspace bounds");
    for (int i = 0; i < m; ++i)
        if (!finite(p->u_lo[i]) || !finite(p->u_hi[i]) || p->u_lo[i] > p->u_hi[i])
            return bad("control bounds");
    for (int i = 0; i < d; ++i) {
        if (std::isnan(p->x_lo[i]) || std::isnan(p->x_hi[i]) || p->x_lo[i] > p->x_hi[i])
            return bad("state bounds");
        if (!finite(p->x_init[i])) return bad("x_init not finite");
    }
    if (!finite(p->margin) || p->margin < 0.f) return bad("margin");
    if (!finite(p->goal_radius) || !(p->goal_radius > p->margin)) return bad("goal radius must exceed margin");
    for (int a = 0; a < 3; ++a)
        if (!finite(p->goal_center[a])) return bad("goal center");
    if (p->dynamics == KPX_QUAD12)
        for (int k = 0; k < 5; ++k)
            if (!finite(p->dyn_params[k]) || !(p->dyn_params[k] > 0.f)) return bad("quadrotor parameters");
    if (!finite(q->dt) || !(q->dt > 0.f)) return bad("dt");
    // step counts and first invalid steps travel as 16-bit signed values
    if (q->steps_min < 1 || q->steps_max < q->steps_min || q->steps_max > 32767) return bad("steps range");
    long long nc = 1;
    for (int a = 0; a < 3; ++a) {
        if (q->grid[a] < 1 || q->grid[a] > (1 << 20)) return bad("grid");
        nc *= q->grid[a];
    }
    if (q->vel_sign_bins != 0 && q->vel_sign_bins != 1) return bad("vel_sign_bins");
    if (q->vel_sign_bins && p->dynamics == KPX_DUBINS6) return bad("sign bins need a velocity state");
    if (q->vel_sign_bins) nc *= 8;
    if (nc > (1ll << 30)) return bad("too many regions");
    if (q->refine_max > 8) return bad("refine_max out of 0..8");
    const long long rf = q->refine_max > 1 ? q->refine_max : 1;
    const long long nc_cap = nc * rf * rf * rf;
    if (nc_cap > (1ll << 30)) return bad("too many regions after refinement");
    if (q->n_select < 1 || q->samples_per_node < 0) return bad("n_select / samples_per_node");
    // candidate slots per iteration: n_select * K, or n_select (the buffer the
    // uncapped form shares out) when samples_per_node = 0
    const long long S = (long long)q->n_select * (q->samples_per_node > 0 ? q->samples_per_node : 1);
    if (S > (1ll << 28)) return bad("n_select * samples_per_node too large");
    if (q->i_max < 0 || q->i_max > 254) return bad("i_max out of 0..254");
    const long long surv = std::min(nc, S);
    if (q->tree_cap < 1 + surv) return bad("tree_cap < 1 + most survivors of one iteration");
    if (q->tree_cap + S > (1ll << 31) - 1) return bad("tree_cap too large");
    if (z) {
        z->d = d;
        z->m = m;
        z->cap = q->tree_cap;
        z->n_cells = (int)nc;
        z->n_cells_cap = (int)nc_cap;
        z->s_max = (int)S;
        z->n_tiles = (int)((S + kTile - 1) / kTile);
        z->n_bgroups = (int)(((nc_cap + kBlock - 1) / kBlock + kGroup - 1) / kGroup);
        z->n_tgroups = (z->n_tiles + kGroup - 1) / kGroup;
        z->n_boxes = p->n_boxes;
        z->n_act = (int)((nc_cap + 4095) & ~4095ll);
        BoxGrid g;
        build_box_grid(p, &g);
        for (int a = 0; a < 3; ++a) z->gb_n[a] = g.n[a];
        z->gb_entries = (int)g.list.size();
    }
    return KPX_OK;
}

DevProblem make_dev_problem(const kpx_problem* p, const kpx_params* q, const Sizes& z)
{
    DevProblem P;
    std::memset(&P, 0, sizeof(P));
    const float m = p->margin;
    P.dyn = p->dynamics;
    P.cost = p->cost;
    P.d = z.d;
    P.m = z.m;
    P.dt = q->dt;
    P.h2 = 0.5f * q->dt;
    P.h6 = q->dt / 6.0f;
    P.steps_min = q->steps_min;
    P.steps_range = q->steps_max - q->steps_min + 1;
    for (int i = 0; i < 4; ++i) {
        P.u_lo[i] = i < z.m ? p->u_lo[i] : 0.f;
        P.u_span[i] = i < z.m ? p->u_hi[i] - p->u_lo[i] : 0.f;
    }
    for (int i = 0; i < 12; ++i) {
        P.x_lo[i] = i < z.d ? p->x_lo[i] + m : -INFINITY;
        P.x_hi[i] = i < z.d ? p->x_hi[i] - m : INFINITY;
    }
    for (int a = 0; a < 3; ++a) {
        P.ws_lo[a] = p->ws_lo[a] + m;
        P.ws_hi[a] = p->ws_hi[a] - m;
        P.cell_lo[a] = p->ws_lo[a];
        P.cell_scale[a] = (float)q->grid[a] / (p->ws_hi[a] - p->ws_lo[a]);
        P.grid[a] = q->grid[a];
        P.goal_c[a] = p->goal_center[a];
    }
    P.vel_sign_bins = q->vel_sign_bins;
    P.vel_idx = p->dynamics == KPX_QUAD12 ? 6 : 3;
    const float r = p->goal_radius - m;
    P.goal_r2 = r * r;
    if (p->dynamics == KPX_QUAD12) {
        const float mass = p->dyn_params[0], jx = p->dyn_params[1], jy = p->dyn_params[2],
                    jz = p->dyn_params[3];
        P.inv_mass = 1.0f / mass;
        P.inv_j[0] = 1.0f / jx;
        P.inv_j[1] = 1.0f / jy;
        P.inv_j[2] = 1.0f / jz;
        P.gyro[0] = jz - jy;
        P.gyro[1] = jx - jz;
        P.gyro[2] = jy - jx;
        P.grav = p->dyn_params[4];
    }
    P.bound_mask = 0;
    for (int i = 0; i < z.d; ++i)
        if (std::isfinite(p->x_lo[i]) || std::isfinite(p->x_hi[i])) P.bound_mask |= 1u << i;
    // the bound test in integration units: planning bounds (the workspace
    // folded into the position bounds), angular components in revolutions
    P.os_mask = 0;
    for (int i = 0; i < KPX_MAX_STATE; ++i) {
        P.bnd_s[i] = 0.f;
        P.bnd_o[i] = 0.f;
        P.os_lo[i] = -INFINITY;
        P.os_hi[i] = INFINITY;
        if (i >= z.d) continue;
        double lo = P.x_lo[i], hi = P.x_hi[i];
        if (i < 3) {
            lo = std::max(lo, (double)P.ws_lo[i]);
            hi = std::min(hi, (double)P.ws_hi[i]);
        }
        if (rev_state(p->dynamics, i)) {
            lo *= 0.15915494309189535;
            hi *= 0.15915494309189535;
        }
        if (std::isfinite(lo) && std::isfinite(hi) && hi > lo) {
            P.bnd_s[i] = (float)(2.0 / (hi - lo));
            P.bnd_o[i] = (float)(-(hi + lo) / (hi - lo));
        } else if (std::isfinite(lo) || std::isfinite(hi)) {
            // one finite bound, or an interval of at most one point: direct test
            P.os_mask |= 1u << i;
            P.os_lo[i] = (float)lo;
            P.os_hi[i] = (float)hi;
        }
    }
    P.n_boxes = p->n_boxes;
    for (int a = 0; a < 3; ++a) {
        P.gb_lo[a] = p->ws_lo[a];
        P.gb_scale[a] = (float)z.gb_n[a] / (p->ws_hi[a] - p->ws_lo[a]);
        P.gb_n[a] = z.gb_n[a];
    }
    P.gb_cells = z.gb_n[0] * z.gb_n[1] * z.gb_n[2];
    P.gb_entries = z.gb_entries;
    P.n_cu = 1;
    P.sort_shift = 0;
    while (((q->steps_max - q->steps_min) >> P.sort_shift) >= kSortBins) ++P.sort_shift;
    P.n_cells = z.n_cells;
    P.K = q->samples_per_node;
    P.n_select = q->n_select;
    P.s_max = z.s_max;
    P.i_max = q->i_max;
    P.surv_max = (int)std::min<long long>(z.n_cells, z.s_max);
    P.cap = z.cap;
    P.seed_lo = (uint32_t)(q->seed & 0xFFFFFFFFull);
    P.seed_hi = (uint32_t)(q->seed >> 32);
    P.query = q->query_id;
    P.n_tiles = z.n_tiles;
    P.n_bgroups = z.n_bgroups;
    P.n_tgroups = z.n_tgroups;
    return P;
}

// planning valid set on the host (float32, same tests as the device)
bool start_is_valid(const kpx_problem* p, int d)
{
    const float m = p->margin;
    const float* x = p->x_init;
    for (int a = 0; a < 3; ++a)
        if (!(x[a] >= p->ws_lo[a] + m && x[a] <= p->ws_hi[a] - m)) return false;
    for (int i = 0; i < d; ++i)
        if (!(x[i] >= p->x_lo[i] + m && x[i] <= p->x_hi[i] - m)) return false;
    for (int b = 0; b < p->n_boxes; ++b) {
        const float* bx = p->boxes + 6 * b;
        bool in = true;
        for (int a = 0; a < 3; ++a) in = in && x[a] >= bx[a] - m && x[a] <= bx[3 + a] + m;
        if (in) return false;
    }
    return true;
}

}  // namespace

struct kpx_handle {
    kpx_problem prob;
    kpx_params prm;
    Sizes z;
    DevProblem P;
    DevPtrs T;
    hipStream_t stream = nullptr;
    void* base = nullptr;
    size_t bytes = 0;
    bool owns = false;
    bool dump_on = false;
    int timing_mask = 0;                      // bit k: kernel k is timed
    int timing_every = 1;                     // ... in every timing_every-th iteration
    long long timing_iter = 0;                // iterations since timing was set
    long long enq_iter = 0;                   // iterations enqueued since creation
    struct Timed {
        int kernel;
        long long iter;                       // the launch's iteration (enq_iter)
        hipEvent_t begin, end;
    };
    std::vector<Timed> timed;                 // one per timed launch
    std::vector<hipEvent_t> spare;
    int full_cached = 0;
    int n_prune_blocks = 0;                   // region blocks of rpt x kBlock regions
    int rpt = 1;                              // regions per thread of prune and the close
    int cur = 0;                              // which device state is current
    int refined = 1;                          // total refinement factor per axis so far
    int polish_steps = 0;                     // edge polish of inserted nodes (0: off)
    float polish_lr = 0.f;
    int polish_goal_only = 0;                 // 1: polish only nodes inserted in the goal set
    bool cost_first = false;                  // propagate in the cost-first form
    int prop_threads = kPropBlock;            // propagate block size (kPropBlock or kPropBlockWide)
    int prop_chunk = kChunkMax;               // propagate chunk (kChunkMax or kChunkBig slots)
    kpxd::DiffConst polish_c{};
    std::string err;
};

namespace {

int fail(kpx_handle* h, int code, const std::string& msg)
{
    if (h) h->err = msg;
    return code;
}

#define KPX_HIP(h, expr)                                                                    \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((h), KPX_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

void carve(kpx_handle* h)
{
    char* b = (char*)h->base;
    size_t o = 0;
    DevPtrs& T = h->T;
    std::memset(&T, 0, sizeof(T));
    void* ptrs[48];
    int k = 0;
    for_each_array(h->z, [&](const char*, size_t bytes) {
        ptrs[k++] = b + o;
        o = align_up(o + (bytes ? bytes : 1));
    });
    k = 0;
    T.x = (float*)ptrs[k++];
    T.u = (float*)ptrs[k++];
    T.steps = (uint16_t*)ptrs[k++];
    T.parent = (int*)ptrs[k++];
    T.cost = (uint32_t*)ptrs[k++];
    T.cell = (int*)ptrs[k++];
    T.status = (uint8_t*)ptrs[k++];
    T.icount = (uint8_t*)ptrs[k++];
    T.dead = (uint8_t*)ptrs[k++];
    T.anc = (int4*)ptrs[k++];
    T.tbl = (unsigned long long*)ptrs[k++];
    T.sel = (int*)ptrs[k++];
    T.ckey = (unsigned long long*)ptrs[k++];
    T.ccell = (int*)ptrs[k++];
    T.cx = (float*)ptrs[k++];
    T.cflag = (uint8_t*)ptrs[k++];
    T.csurv = (uint8_t*)ptrs[k++];
    T.tile_count = (int*)ptrs[k++];
    T.act = (uint8_t*)ptrs[k++];
    T.boxes = (float4*)ptrs[k++];
    T.gcell = (int2*)ptrs[k++];
    T.glist = (uint16_t*)ptrs[k++];
    T.st = (DevState*)ptrs[k++];
    T.bcount = (int2*)ptrs[k++];
    T.bgroup = (int2*)ptrs[k++];
    T.tgroup = (int*)ptrs[k++];
    T.stats = (kpx_iter_stats*)ptrs[k++];
    T.d_parent = (int*)ptrs[k++];
    T.d_u = (float*)ptrs[k++];
    T.d_n = (int*)ptrs[k++];
    T.d_fi = (int*)ptrs[k++];
    T.d_pfi = (int*)ptrs[k++];
    T.d_pcell = (int*)ptrs[k++];
    T.d_pflag = (uint8_t*)ptrs[k++];
    T.path = (int*)ptrs[k++];
    T.path_x = (float*)ptrs[k++];
    T.path_u = (float*)ptrs[k++];
    T.path_n = (int*)ptrs[k++];
    T.path_len = (int*)ptrs[k++];
    T.x_init = (float*)ptrs[k++];
}

size_t total_bytes(const Sizes& z)
{
    size_t o = 0;
    for_each_array(z, [&](const char*, size_t bytes) { o = align_up(o + (bytes ? bytes : 1)); });
    return o;
}

DevState* cur_state(const kpx_handle* h) { return h->T.st + h->cur; }
DevState* next_state(const kpx_handle* h) { return h->T.st + (h->cur ^ 1); }

DevPtrs kernel_ptrs(const kpx_handle* h)
{
    DevPtrs T = h->T;
    if (!h->dump_on) {
        T.d_parent = nullptr;
        T.d_u = nullptr;
        T.d_n = nullptr;
        T.d_fi = nullptr;
        T.d_pfi = nullptr;
        T.d_pcell = nullptr;
        T.d_pflag = nullptr;
    }
    return T;
}

size_t propagate_lds_bytes(const Sizes& z, int d)
{
    // every region padded to whole 16-byte words (the kernel stages them as such)
    const size_t gbp = ((size_t)z.gb_n[0] * z.gb_n[1] * z.gb_n[2] + 1) & ~(size_t)1;
    return sizeof(float4) * 2 * (size_t)z.n_boxes + sizeof(float) * (size_t)((d + 3) & ~3) * kParMax +
           sizeof(int2) * gbp + 16 * (((size_t)z.gb_entries + 7) / 8);
}

template <int DYN, int COST, int CH>
void launch_propagate_ch(kpx_handle* h, const DevPtrs& T, size_t lds)
{
    const bool wide = h->prop_threads == kPropBlockWide;
    if (h->cost_first && wide)
        k_propagate<DYN, COST, true, kPropBlockWide, CH><<<h->P.n_cu, kPropBlockWide, lds, h->stream>>>(h->P, T, cur_state(h));
    else if (h->cost_first)
        k_propagate<DYN, COST, true, kPropBlock, CH><<<h->P.n_cu, kPropBlock, lds, h->stream>>>(h->P, T, cur_state(h));
    else if (wide)
        k_propagate<DYN, COST, false, kPropBlockWide, CH><<<h->P.n_cu, kPropBlockWide, lds, h->stream>>>(h->P, T, cur_state(h));
    else
        k_propagate<DYN, COST, false, kPropBlock, CH><<<h->P.n_cu, kPropBlock, lds, h->stream>>>(h->P, T, cur_state(h));
}

template <int DYN, int COST>
void launch_propagate(kpx_handle* h, const DevPtrs& T)
{
    const size_t lds = propagate_lds_bytes(h->z, Dims<DYN>::D);
    if (h->prop_chunk == kChunkBig) launch_propagate_ch<DYN, COST, kChunkBig>(h, T, lds);
    else launch_propagate_ch<DYN, COST, kChunkMax>(h, T, lds);
}

// Allows `dynamic` bytes of dynamic LDS for a propagate kernel, after checking
// that they fit beside its static LDS: KPX_OK, KPX_ERR_ARG (too large) or
// KPX_ERR_DEVICE.
int allow_lds(const void* kernel, size_t dynamic, int lds_max)
{
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, kernel) != hipSuccess) return KPX_ERR_DEVICE;
    if (fa.sharedSizeBytes + dynamic > (size_t)lds_max) return KPX_ERR_ARG;
    if (hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dynamic) != hipSuccess)
        return KPX_ERR_DEVICE;
    return KPX_OK;
}

// The propagate kernel for a (model, cost) pair: batched, or single-query in
// the plain or the cost-first form.
template <int DYN, int COST, int CH>
const void* propagate_kernel_ch(bool cf, bool wide)
{
    if (wide)
        return cf ? (const void*)k_propagate<DYN, COST, true, kPropBlockWide, CH>
                  : (const void*)k_propagate<DYN, COST, false, kPropBlockWide, CH>;
    return cf ? (const void*)k_propagate<DYN, COST, true, kPropBlock, CH>
              : (const void*)k_propagate<DYN, COST, false, kPropBlock, CH>;
}
template <int DYN, int COST>
const void* propagate_kernel_t(bool batched, bool cf, bool wide, bool big)
{
    if (batched) return wide ? (const void*)kb_propagate<DYN, COST, kPropBlockWide> : (const void*)kb_propagate<DYN, COST, kPropBlock>;
    return big ? propagate_kernel_ch<DYN, COST, kChunkBig>(cf, wide) : propagate_kernel_ch<DYN, COST, kChunkMax>(cf, wide);
}
const void* propagate_kernel(int dyn, int cost, bool batched, bool cf = false, bool wide = false, bool big = false)
{
    switch (dyn * 2 + cost) {
    case 0: return propagate_kernel_t<kDI6, kTIME>(batched, cf, wide, big);
    case 1: return propagate_kernel_t<kDI6, kPATH>(batched, cf, wide, big);
    case 2: return propagate_kernel_t<kQUAD12, kTIME>(batched, cf, wide, big);
    case 3: return propagate_kernel_t<kQUAD12, kPATH>(batched, cf, wide, big);
    case 4: return propagate_kernel_t<kDUBINS6, kTIME>(batched, cf, wide, big);
    default: return propagate_kernel_t<kDUBINS6, kPATH>(batched, cf, wide, big);
    }
}

void propagate(kpx_handle* h, const DevPtrs& T)
{
    const int key = h->P.dyn * 2 + h->P.cost;
    switch (key) {
    case 0: launch_propagate<kDI6, kTIME>(h, T); break;
    case 1: launch_propagate<kDI6, kPATH>(h, T); break;
    case 2: launch_propagate<kQUAD12, kTIME>(h, T); break;
    case 3: launch_propagate<kQUAD12, kPATH>(h, T); break;
    case 4: launch_propagate<kDUBINS6, kTIME>(h, T); break;
    default: launch_propagate<kDUBINS6, kPATH>(h, T); break;
    }
}

void insert(kpx_handle* h, const DevPtrs& T)
{
    const int grid = h->z.n_tiles;
    switch (h->P.dyn) {
    case kDI6: k_insert<kDI6><<<grid, kBlock, 0, h->stream>>>(h->P, T, cur_state(h)); break;
    case kQUAD12: k_insert<kQUAD12><<<grid, kBlock, 0, h->stream>>>(h->P, T, cur_state(h)); break;
    default: k_insert<kDUBINS6><<<grid, kBlock, 0, h->stream>>>(h->P, T, cur_state(h)); break;
    }
}

hipEvent_t take_event(kpx_handle* h)
{
    if (!h->spare.empty()) {
        hipEvent_t e = h->spare.back();
        h->spare.pop_back();
        return e;
    }
    // Timing events only: recorded without the system-scope fence, which
    // would make each record write back and invalidate the caches between
    // two kernels of the iteration (nothing of the device memory need be
    // visible to the host when such an event completes).
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

// Launches kernel k of an iteration through `launch`, bracketed by events on
// the handle's stream when k is timed.
template <typename F>
int timed_launch(kpx_handle* h, int k, F&& launch)
{
    if (!(h->timing_mask & (1 << k)) || h->timing_iter % h->timing_every != 0) {
        launch();
        return KPX_OK;
    }
    hipEvent_t a = take_event(h), b = a ? take_event(h) : nullptr;
    if (!a || !b) return fail(h, KPX_ERR_DEVICE, "hipEventCreate failed");
    KPX_HIP(h, hipEventRecord(a, h->stream));
    launch();
    KPX_HIP(h, hipEventRecord(b, h->stream));
    h->timed.push_back({k, h->enq_iter, a, b});
    return KPX_OK;
}

int refresh_full(kpx_handle* h)
{
    int full = 0;
    KPX_HIP(h, hipMemcpyAsync(&full, &cur_state(h)->full, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    KPX_HIP(h, hipStreamSynchronize(h->stream));
    h->full_cached = full;
    return KPX_OK;
}

}  // namespace

// ============================================================== batches

// Independent queries iterated together (see the batched kernels).  The batch
// keeps only the per-query problem and pointer arrays, the block maps and,
// optionally, HIP graphs of two iterations; the queries stay in their handles.
struct kpx_batch {
    std::vector<kpx_handle*> hs;
    hipStream_t user = nullptr;     // the handles' stream
    hipStream_t stream = nullptr;   // the batch's own stream (capturable)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    void* mem = nullptr;            // problems | pointers | block maps
    DevProblem* d_P = nullptr;
    DevPtrs* d_T = nullptr;
    struct Group {
        int dyn = 0, cost = 0;
        int nt = kPropBlock;        // propagate threads per block (kpx_batch_set_threads)
        int4* prop = nullptr;
        int n_prop = 0;
        size_t lds = 0;
        int4* ins = nullptr;
        int n_ins = 0;
        int4* prune = nullptr;      // prune and the close, over the group's queries
        int n_prune = 0;
        int4* fin = nullptr;
        int n_fin = 0;
    };
    std::vector<Group> groups;
    int cur = 0;
    bool graph_on = false;
    hipGraphExec_t exec[2] = {nullptr, nullptr};  // two iterations from state parity 0 / 1
    std::vector<int> cells;         // each handle's region count when the batch was made
    std::vector<char> dump;         // ... and whether it recorded its expansions (fixed since)
    // groups after the first run their iterations on side streams forked from
    // and joined back to the batch stream, so that the models' kernels overlap
    // (each propagate is bound by its longest edge, not by the machine, and
    // one group's prune and close run while another still propagates)
    std::vector<hipStream_t> side;
    hipEvent_t ev_fork = nullptr;
    std::vector<hipEvent_t> ev_join;
    std::string err;
};

namespace {

int bfail(kpx_batch* b, int code, const std::string& msg)
{
    if (b) b->err = msg;
    return code;
}

template <int DYN, int COST>
void kb_propagate_launch(const kpx_batch* b, const kpx_batch::Group& g, int par, hipStream_t s)
{
    if (g.nt == kPropBlockWide)
        kb_propagate<DYN, COST, kPropBlockWide><<<g.n_prop, kPropBlockWide, g.lds, s>>>(b->d_P, b->d_T, g.prop, par);
    else
        kb_propagate<DYN, COST, kPropBlock><<<g.n_prop, kPropBlock, g.lds, s>>>(b->d_P, b->d_T, g.prop, par);
}

// Stream of group gi: the batch stream for the first, a side stream otherwise.
hipStream_t group_stream(const kpx_batch* b, size_t gi) { return gi == 0 ? b->stream : b->side[gi - 1]; }

// The side streams start after the work already on the batch stream ...
void batch_fork(const kpx_batch* b)
{
    if (b->side.empty()) return;
    (void)hipEventRecord(b->ev_fork, b->stream);
    for (hipStream_t s : b->side) (void)hipStreamWaitEvent(s, b->ev_fork, 0);
}

// ... and the batch stream continues after theirs.
void batch_join(const kpx_batch* b)
{
    for (size_t j = 0; j < b->side.size(); ++j) {
        (void)hipEventRecord(b->ev_join[j], b->side[j]);
        (void)hipStreamWaitEvent(b->stream, b->ev_join[j], 0);
    }
}

// Enqueues one iteration of every query, at state parity par: each group's
// four kernels in order on the group's stream (between a batch_fork and a
// batch_join); the groups' queries are independent, so nothing orders one
// group after another.
void batch_enqueue(const kpx_batch* b, int par)
{
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        const auto& g = b->groups[gi];
        const hipStream_t s = group_stream(b, gi);
        switch (g.dyn * 2 + g.cost) {
        case 0: kb_propagate_launch<kDI6, kTIME>(b, g, par, s); break;
        case 1: kb_propagate_launch<kDI6, kPATH>(b, g, par, s); break;
        case 2: kb_propagate_launch<kQUAD12, kTIME>(b, g, par, s); break;
        case 3: kb_propagate_launch<kQUAD12, kPATH>(b, g, par, s); break;
        case 4: kb_propagate_launch<kDUBINS6, kTIME>(b, g, par, s); break;
        default: kb_propagate_launch<kDUBINS6, kPATH>(b, g, par, s); break;
        }
        kb_prune_flags<<<g.n_prune, kBlock, 0, s>>>(b->d_P, b->d_T, g.prune, par);
        switch (g.dyn) {
        case kDI6: kb_insert<kDI6><<<g.n_ins, kBlock, 0, s>>>(b->d_P, b->d_T, g.ins, par); break;
        case kQUAD12: kb_insert<kQUAD12><<<g.n_ins, kBlock, 0, s>>>(b->d_P, b->d_T, g.ins, par); break;
        default: kb_insert<kDUBINS6><<<g.n_ins, kBlock, 0, s>>>(b->d_P, b->d_T, g.ins, par); break;
        }
        kb_finalize_select<<<g.n_fin, kBlock, 0, s>>>(b->d_P, b->d_T, g.fin, par);
    }
}

// Captures two iterations starting at parity p into b->exec[p].
int batch_capture(kpx_batch* b, int p)
{
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return bfail(b, KPX_ERR_DEVICE, "hipStreamBeginCapture failed");
    batch_fork(b);
    batch_enqueue(b, p);
    batch_enqueue(b, p ^ 1);
    batch_join(b);
    if (hipStreamEndCapture(b->stream, &g) != hipSuccess || !g)
        return bfail(b, KPX_ERR_DEVICE, "hipStreamEndCapture failed");
    const hipError_t e = hipGraphInstantiate(&b->exec[p], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b->exec[p] = nullptr;
        return bfail(b, KPX_ERR_DEVICE, "hipGraphInstantiate failed");
    }
    return KPX_OK;
}

void batch_free(kpx_batch* b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (auto& e : b->exec)
        if (e) (void)hipGraphExecDestroy(e);
    if (b->mem) (void)hipFree(b->mem);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    for (hipStream_t s : b->side) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    for (hipEvent_t e : b->ev_join) (void)hipEventDestroy(e);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

}  // namespace

// ============================================================== C ABI

extern "C" {

int kpx_workspace_bytes(const kpx_problem* prob, const kpx_params* prm, size_t* out_bytes)
{
    if (!out_bytes) return KPX_ERR_ARG;
    Sizes z;
    const int rc = validate(prob, prm, &z, nullptr);
    if (rc != KPX_OK) return rc;
    *out_bytes = total_bytes(z);
    return KPX_OK;
}

int kpx_create(const kpx_problem* prob, const kpx_params* prm, void* hip_stream, void* workspace,
               size_t workspace_bytes, kpx_handle** out)
{
    if (!out) return KPX_ERR_ARG;
    *out = nullptr;
    Sizes z;
    std::string why;
    int rc = validate(prob, prm, &z, &why);
    if (rc != KPX_OK) return rc;
    if (!start_is_valid(prob, z.d)) return KPX_ERR_INVALID_START;
    const size_t need = total_bytes(z);
    if (workspace && workspace_bytes < need) return KPX_ERR_OOM;

    kpx_handle* h = new (std::nothrow) kpx_handle();
    if (!h) return KPX_ERR_OOM;
    h->prob = *prob;
    h->prob.boxes = nullptr;
    h->prm = *prm;
    h->z = z;
    h->P = make_dev_problem(prob, prm, z);
    h->stream = (hipStream_t)hip_stream;
    h->bytes = need;
    {
        int dev = 0, n_cu = 0, lds_max = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
            delete h;
            return KPX_ERR_DEVICE;
        }
        h->P.n_cu = std::max(1, n_cu);
        // The cheap models' RK4 step is short beside the LDS latency of a
        // refill or a box lookup, so with two slots or more per lane they run
        // two waves per SIMD, which hide each other's waits.  The quadrotor
        // keeps one wave per SIMD: a lone wave issues a dependent VALU
        // instruction only every ~7.5 clocks, but a second wave on the SIMD
        // delays the wave holding the longest edge, which bounds the kernel,
        // whatever their priorities (25% slower measured).
        h->prop_threads = (h->P.dyn != kQUAD12 && (long long)z.s_max >= 2LL * kPropBlock * h->P.n_cu)
                              ? kPropBlockWide : kPropBlock;
        // Chunks of kChunkBig slots when a block's share of the slot buffer
        // exceeds kChunkMax: one chunk instead of two up to kChunkBig, half as
        // many beyond, each paying its parents, sort and longest edge once.
        // The larger LDS arrays must fit beside the scene's obstacle data,
        // else the block keeps kChunkMax.
        const bool wide = h->prop_threads == kPropBlockWide;
        const size_t dyn_lds = propagate_lds_bytes(z, z.d);
        int rc = KPX_OK;
        if ((long long)z.s_max > (long long)kChunkMax * h->P.n_cu) {
            bool fits = true;
            for (bool cf : {false, true})
                fits = fits && allow_lds(propagate_kernel(h->P.dyn, h->P.cost, false, cf, wide, true), dyn_lds,
                                         lds_max) == KPX_OK;
            if (fits) h->prop_chunk = kChunkBig;
        }
        for (bool cf : {false, true})  // both forms, so that kpx_set_cost_first needs no device call
            if (rc == KPX_OK)
                rc = allow_lds(propagate_kernel(h->P.dyn, h->P.cost, false, cf, wide, h->prop_chunk == kChunkBig),
                               dyn_lds, lds_max);
        if (rc != KPX_OK) {
            delete h;
            return rc;
        }
    }
    if (workspace) {
        h->base = workspace;
    } else {
        hipError_t e = hipMalloc(&h->base, need);
        if (e != hipSuccess) {
            delete h;
            return e == hipErrorOutOfMemory ? KPX_ERR_OOM : KPX_ERR_DEVICE;
        }
        h->owns = true;
    }
    carve(h);
    h->rpt = (long long)z.n_cells_cap >= kRptRegions ? kRptBatch : 1;
    h->n_prune_blocks = region_blocks(z.n_cells, h->rpt);

    // boxes grown by the margin (two float4 each), the box grid, x_init
    std::vector<float> boxes((size_t)8 * (z.n_boxes > 0 ? z.n_boxes : 1), 0.f);
    for (int b = 0; b < z.n_boxes; ++b)
        for (int a = 0; a < 3; ++a) {
            boxes[8 * b + a] = prob->boxes[6 * b + a] - prob->margin;
            boxes[8 * b + 4 + a] = prob->boxes[6 * b + 3 + a] + prob->margin;
        }
    BoxGrid grid;
    build_box_grid(prob, &grid);
    auto cleanup = [&](int code) {
        kpx_destroy(h);
        return code;
    };
    if (hipMemcpyAsync(h->T.boxes, boxes.data(), sizeof(float) * boxes.size(), hipMemcpyHostToDevice,
                       h->stream) != hipSuccess)
        return cleanup(KPX_ERR_DEVICE);
    std::vector<int2> gcell(grid.cells.size());
    for (size_t c = 0; c < gcell.size(); ++c) {
        int bits;
        std::memcpy(&bits, &grid.clear[c], sizeof(bits));
        gcell[c] = make_int2(grid.cells[c], bits);
    }
    if (hipMemcpyAsync(h->T.gcell, gcell.data(), sizeof(int2) * gcell.size(), hipMemcpyHostToDevice,
                       h->stream) != hipSuccess)
        return cleanup(KPX_ERR_DEVICE);
    if (!grid.list.empty() &&
        hipMemcpyAsync(h->T.glist, grid.list.data(), sizeof(uint16_t) * grid.list.size(),
                       hipMemcpyHostToDevice, h->stream) != hipSuccess)
        return cleanup(KPX_ERR_DEVICE);
    // the group sums of both parities start at zero (each close clears the
    // other parity's for the next iteration)
    if (hipMemsetAsync(h->T.bgroup, 0, sizeof(int) * kGroupPad * 2 * (size_t)z.n_bgroups, h->stream) != hipSuccess ||
        hipMemsetAsync(h->T.tgroup, 0, sizeof(int) * kGroupPad * 2 * (size_t)z.n_tgroups, h->stream) != hipSuccess)
        return cleanup(KPX_ERR_DEVICE);
    float* xi = h->T.x_init;
    if (hipMemcpyAsync(xi, prob->x_init, sizeof(float) * KPX_MAX_STATE, hipMemcpyHostToDevice,
                       h->stream) != hipSuccess)
        return cleanup(KPX_ERR_DEVICE);
    k_fill_table<<<std::min(1024, (z.n_act + kBlock - 1) / kBlock), kBlock, 0, h->stream>>>(
        h->T.tbl, h->T.act, z.n_cells, z.n_act);
    switch (h->P.dyn) {
    case kDI6: k_init_root<kDI6><<<1, 64, 0, h->stream>>>(h->P, h->T, h->T.st, xi); break;
    case kQUAD12: k_init_root<kQUAD12><<<1, 64, 0, h->stream>>>(h->P, h->T, h->T.st, xi); break;
    default: k_init_root<kDUBINS6><<<1, 64, 0, h->stream>>>(h->P, h->T, h->T.st, xi); break;
    }
    k_select<<<1, kSelectThreads, 0, h->stream>>>(h->P, h->T, h->T.st);
    if (hipGetLastError() != hipSuccess) return cleanup(KPX_ERR_DEVICE);
    if (hipStreamSynchronize(h->stream) != hipSuccess) return cleanup(KPX_ERR_DEVICE);
    *out = h;
    return KPX_OK;
}

int kpx_iterate(kpx_handle* h, int32_t n_iters)
{
    if (!h || n_iters < 0) return KPX_ERR_ARG;
    if (h->full_cached) return KPX_FULL;
    for (int i = 0; i < n_iters; ++i) {
        const DevPtrs T = kernel_ptrs(h);
        int rc;
        if ((rc = timed_launch(h, 0, [&] { propagate(h, T); })) != KPX_OK) return rc;
        if ((rc = timed_launch(h, 1, [&] {
                 if (h->rpt == 1)
                     k_prune_flags<1><<<h->n_prune_blocks, kBlock, 0, h->stream>>>(h->P, T, cur_state(h),
                                                                                   h->n_prune_blocks);
                 else
                     k_prune_flags<kRptBatch><<<h->n_prune_blocks, kBlock, 0, h->stream>>>(
                         h->P, T, cur_state(h), h->n_prune_blocks);
             })) != KPX_OK)
            return rc;
        if ((rc = timed_launch(h, 2, [&] { insert(h, T); })) != KPX_OK) return rc;
        if (h->polish_steps > 0) {
            const dim3 grid((h->P.surv_max + kPolishBlock - 1) / kPolishBlock);
            const size_t lds = polish_lds_bytes(h->P.n_boxes);
            if (h->P.cost == kPATH)
                k_polish<kPATH><<<grid, kPolishBlock, lds, h->stream>>>(h->P, T, cur_state(h), h->polish_c,
                                                                        h->polish_steps, h->polish_lr,
                                                                        h->polish_goal_only);
            else
                k_polish<kTIME><<<grid, kPolishBlock, lds, h->stream>>>(h->P, T, cur_state(h), h->polish_c,
                                                                        h->polish_steps, h->polish_lr,
                                                                        h->polish_goal_only);
        }
        if ((rc = timed_launch(h, 3, [&] {
                 if (h->rpt == 1)
                     k_finalize_select<1><<<h->n_prune_blocks, kBlock, 0, h->stream>>>(
                         h->P, T, cur_state(h), next_state(h), h->n_prune_blocks);
                 else
                     k_finalize_select<kRptBatch><<<h->n_prune_blocks, kBlock, 0, h->stream>>>(
                         h->P, T, cur_state(h), next_state(h), h->n_prune_blocks);
             })) != KPX_OK)
            return rc;
        h->cur ^= 1;  // the state the close of this iteration wrote is current
        ++h->timing_iter;
        ++h->enq_iter;
    }
    KPX_HIP(h, hipGetLastError());
    return KPX_OK;
}

int kpx_sync(kpx_handle* h)
{
    if (!h) return KPX_ERR_ARG;
    const int rc = refresh_full(h);
    if (rc != KPX_OK) return rc;
    return h->full_cached ? KPX_FULL : KPX_OK;
}

int kpx_counters_read(kpx_handle* h, kpx_counters* out)
{
    if (!h || !out) return KPX_ERR_ARG;
    DevState s;
    KPX_HIP(h, hipMemcpyAsync(&s, cur_state(h), sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
    KPX_HIP(h, hipStreamSynchronize(h->stream));
    h->full_cached = s.full;
    out->n_tree = s.n_tree;
    out->iteration = s.it;
    out->cursor = s.cursor;
    out->n_select = s.last_n_sel;
    out->n_valid = s.last_n_valid;
    out->n_survivors = s.last_n_surv;
    out->substeps = s.last_substeps;
    out->first_solution_iteration = s.first_sol_it;
    out->solution_key = s.sol;
    out->full = s.full;
    out->samples_per_node = s.last_k;
    return KPX_OK;
}

int kpx_solution(kpx_handle* h, kpx_solution_info* info, float* states, float* controls,
                 int32_t* steps, int32_t capacity_edges)
{
    if (!h || !info) return KPX_ERR_ARG;
    kpx_counters c;
    int rc = kpx_counters_read(h, &c);
    if (rc != KPX_OK) return rc;
    std::memset(info, 0, sizeof(*info));
    info->first_solution_iteration = c.first_solution_iteration;
    info->n_tree = c.n_tree;
    info->iteration = c.iteration;
    info->tree_index = -1;
    if (c.solution_key == kEmpty) return KPX_OK;
    switch (h->P.dyn) {
    case kDI6: k_extract_path<kDI6><<<1, 64, 0, h->stream>>>(h->P, kernel_ptrs(h), cur_state(h), kMaxPath); break;
    case kQUAD12: k_extract_path<kQUAD12><<<1, 64, 0, h->stream>>>(h->P, kernel_ptrs(h), cur_state(h), kMaxPath); break;
    default: k_extract_path<kDUBINS6><<<1, 64, 0, h->stream>>>(h->P, kernel_ptrs(h), cur_state(h), kMaxPath); break;
    }
    KPX_HIP(h, hipGetLastError());
    int len = 0;
    KPX_HIP(h, hipMemcpyAsync(&len, h->T.path_len, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    KPX_HIP(h, hipStreamSynchronize(h->stream));
    info->found = 1;
    info->tree_index = (int64_t)(uint32_t)c.solution_key;
    info->cost_field = (uint32_t)(c.solution_key >> 32);
    if (h->prob.cost == KPX_COST_TIME) {
        info->cost = (double)info->cost_field * (double)h->prm.dt;
    } else {
        float f;
        std::memcpy(&f, &info->cost_field, sizeof(f));
        info->cost = f;
    }
    if (len < 0) {
        info->n_edges = -len - 1;
        return fail(h, KPX_ERR_BUFFER, "solution path longer than the extraction buffer");
    }
    info->n_edges = len - 1;
    if (!states && !controls && !steps) return KPX_OK;
    if (capacity_edges < info->n_edges) return fail(h, KPX_ERR_BUFFER, "capacity_edges < n_edges");
    std::vector<float> px((size_t)len * KPX_MAX_STATE), pu((size_t)len * KPX_MAX_CONTROL);
    std::vector<int> pn((size_t)len);
    KPX_HIP(h, hipMemcpyAsync(px.data(), h->T.path_x, sizeof(float) * px.size(), hipMemcpyDeviceToHost, h->stream));
    KPX_HIP(h, hipMemcpyAsync(pu.data(), h->T.path_u, sizeof(float) * pu.size(), hipMemcpyDeviceToHost, h->stream));
    KPX_HIP(h, hipMemcpyAsync(pn.data(), h->T.path_n, sizeof(int) * pn.size(), hipMemcpyDeviceToHost, h->stream));
    KPX_HIP(h, hipStreamSynchronize(h->stream));
    if (states) std::memcpy(states, px.data(), sizeof(float) * px.size());
    for (int e = 0; e < info->n_edges; ++e) {
        if (controls)
            for (int k = 0; k < KPX_MAX_CONTROL; ++k)
                controls[e * KPX_MAX_CONTROL + k] = pu[(size_t)(e + 1) * KPX_MAX_CONTROL + k];
        if (steps) steps[e] = pn[e + 1];
    }
    return KPX_OK;
}

int kpx_snapshot(kpx_handle* h, kpx_tree_view* v, kpx_counters* counters)
{
    if (!h || !v) return KPX_ERR_ARG;
    kpx_counters c;
    int rc = kpx_counters_read(h, &c);
    if (rc != KPX_OK) return rc;
    if (counters) *counters = c;
    const size_t n = (size_t)c.n_tree;
    if (v->capacity < (int64_t)n) return fail(h, KPX_ERR_BUFFER, "view capacity < n_tree");
    const size_t cap = (size_t)h->z.cap, ld = (size_t)v->capacity;
    if (v->state)
        for (int k = 0; k < KPX_MAX_STATE; ++k) {
            if (k < h->z.d)
                KPX_HIP(h, hipMemcpyAsync(v->state + k * ld, h->T.x + k * cap, sizeof(float) * n,
                                          hipMemcpyDeviceToHost, h->stream));
            else
                std::memset(v->state + k * ld, 0, sizeof(float) * n);
        }
    if (v->control)
        for (int k = 0; k < KPX_MAX_CONTROL; ++k) {
            if (k < h->z.m)
                KPX_HIP(h, hipMemcpyAsync(v->control + k * ld, h->T.u + k * cap, sizeof(float) * n,
                                          hipMemcpyDeviceToHost, h->stream));
            else
                std::memset(v->control + k * ld, 0, sizeof(float) * n);
        }
    std::vector<uint16_t> st16;
    if (v->steps) {
        st16.resize(n ? n : 1);
        KPX_HIP(h, hipMemcpyAsync(st16.data(), h->T.steps, sizeof(uint16_t) * n, hipMemcpyDeviceToHost, h->stream));
    }
    if (v->parent) KPX_HIP(h, hipMemcpyAsync(v->parent, h->T.parent, sizeof(int) * n, hipMemcpyDeviceToHost, h->stream));
    if (v->cost) KPX_HIP(h, hipMemcpyAsync(v->cost, h->T.cost, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, h->stream));
    if (v->cell) KPX_HIP(h, hipMemcpyAsync(v->cell, h->T.cell, sizeof(int) * n, hipMemcpyDeviceToHost, h->stream));
    if (v->status) KPX_HIP(h, hipMemcpyAsync(v->status, h->T.status, n, hipMemcpyDeviceToHost, h->stream));
    if (v->icount) KPX_HIP(h, hipMemcpyAsync(v->icount, h->T.icount, n, hipMemcpyDeviceToHost, h->stream));
    if (v->cell_table) {
        if (v->cell_table_len < h->z.n_cells) return fail(h, KPX_ERR_BUFFER, "cell_table_len < n_cells");
        KPX_HIP(h, hipMemcpyAsync(v->cell_table, h->T.tbl, sizeof(unsigned long long) * h->z.n_cells,
                                  hipMemcpyDeviceToHost, h->stream));
    }
    KPX_HIP(h, hipStreamSynchronize(h->stream));
    if (v->steps)
        for (size_t i = 0; i < n; ++i) v->steps[i] = st16[i];
    return KPX_OK;
}

int kpx_set_dump(kpx_handle* h, int32_t enable)
{
    if (!h || (enable != 0 && enable != 1)) return KPX_ERR_ARG;
    h->dump_on = enable == 1;
    return KPX_OK;
}

int kpx_read_dump(kpx_handle* h, kpx_dump_view* v, int64_t* n_slots)
{
    if (!h || !v || !n_slots) return KPX_ERR_ARG;
    if (!h->dump_on) return fail(h, KPX_ERR_STATE, "dump recording is off");
    kpx_counters c;
    int rc = kpx_counters_read(h, &c);
    if (rc != KPX_OK) return rc;
    const size_t S = (size_t)c.n_select * (size_t)c.samples_per_node;
    *n_slots = (int64_t)S;
    if (v->capacity < (int64_t)S) return fail(h, KPX_ERR_BUFFER, "dump capacity < slots");
    if (S == 0) return KPX_OK;
    const size_t sm = (size_t)h->z.s_max, ld = (size_t)v->capacity;
    auto get = [&](void* dst, const void* src, size_t bytes) -> int {
        KPX_HIP(h, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, h->stream));
        return KPX_OK;
    };
    if (v->parent && (rc = get(v->parent, h->T.d_parent, sizeof(int) * S))) return rc;
    if (v->steps && (rc = get(v->steps, h->T.d_n, sizeof(int) * S))) return rc;
    if (v->first_invalid && (rc = get(v->first_invalid, h->T.d_fi, sizeof(int) * S))) return rc;
    if (v->cell && (rc = get(v->cell, h->T.ccell, sizeof(int) * S))) return rc;
    if (v->key && (rc = get(v->key, h->T.ckey, sizeof(unsigned long long) * S))) return rc;
    if (v->survivor && (rc = get(v->survivor, h->T.csurv, S))) return rc;
    if (v->control)
        for (int k = 0; k < KPX_MAX_CONTROL; ++k) {
            if (k < h->z.m) {
                if ((rc = get(v->control + k * ld, h->T.d_u + k * sm, sizeof(float) * S))) return rc;
            } else {
                std::memset(v->control + k * ld, 0, sizeof(float) * S);
            }
        }
    if (v->state) {
        // slot-major rows on the device, component-major in the view
        const int R = cx_row(h->z.d);
        std::vector<float> rows((size_t)R * S);
        if ((rc = get(rows.data(), h->T.cx, sizeof(float) * rows.size()))) return rc;
        for (int k = 0; k < KPX_MAX_STATE; ++k)
            for (size_t q = 0; q < (size_t)S; ++q) v->state[k * ld + q] = k < h->z.d ? rows[q * R + k] : 0.f;
    }
    std::vector<uint8_t> flag(S);
    if ((rc = get(flag.data(), h->T.cflag, S))) return rc;
    // edge polish decisions, one per inserted node
    const size_t NI = (size_t)std::max<int64_t>(0, c.n_survivors);
    const bool pol = h->polish_steps > 0 && NI > 0;
    std::vector<uint8_t> pflag(pol ? NI : 1, 0);
    if (pol) {
        if (v->polish_first_invalid && (rc = get(v->polish_first_invalid, h->T.d_pfi, sizeof(int) * NI))) return rc;
        if (v->polish_cell && (rc = get(v->polish_cell, h->T.d_pcell, sizeof(int) * NI))) return rc;
        if ((rc = get(pflag.data(), h->T.d_pflag, NI))) return rc;
    }
    KPX_HIP(h, hipStreamSynchronize(h->stream));
    if (v->goal)
        for (size_t s = 0; s < S; ++s) v->goal[s] = (flag[s] >> 1) & 1;
    if (!pol) {
        if (v->polish_first_invalid) std::memset(v->polish_first_invalid, 0, sizeof(int32_t) * NI);
        if (v->polish_cell) std::memset(v->polish_cell, 0, sizeof(int32_t) * NI);
    }
    for (size_t t = 0; t < NI; ++t) {
        if (v->polish_accepted) v->polish_accepted[t] = pol ? (pflag[t] & 1) : 0;
        if (v->polish_goal) v->polish_goal[t] = pol ? ((pflag[t] >> 1) & 1) : 0;
    }
    return KPX_OK;
}

int kpx_refine(kpx_handle* h, int32_t factor)
{
    if (!h || factor < 2) return KPX_ERR_ARG;
    const long long rf_max = h->prm.refine_max > 1 ? h->prm.refine_max : 1;
    if ((long long)h->refined * factor > rf_max) return fail(h, KPX_ERR_ARG, "refine: beyond refine_max");
    int og[3];
    long long nc = h->prm.vel_sign_bins ? 8 : 1;
    for (int a = 0; a < 3; ++a) {
        og[a] = h->prm.grid[a];
        nc *= (long long)og[a] * factor;
    }
    if (nc > h->z.n_cells_cap) return fail(h, KPX_ERR_ARG, "refine: more regions than allocated");
    h->refined *= factor;
    for (int a = 0; a < 3; ++a) {
        h->prm.grid[a] = og[a] * factor;
        h->P.grid[a] = h->prm.grid[a];
        h->P.cell_scale[a] = (float)h->prm.grid[a] / (h->prob.ws_hi[a] - h->prob.ws_lo[a]);
    }
    h->z.n_cells = (int)nc;
    h->P.n_cells = (int)nc;
    h->P.surv_max = (int)std::min<long long>(nc, h->z.s_max);
    h->n_prune_blocks = region_blocks(nc, h->rpt);
    const DevPtrs T = kernel_ptrs(h);
    k_fill_table<<<std::min(1024, (h->z.n_act + kBlock - 1) / kBlock), kBlock, 0, h->stream>>>(
        T.tbl, T.act, h->z.n_cells, h->z.n_act);
    k_refine_nodes<<<1024, kBlock, 0, h->stream>>>(h->P, T, cur_state(h));
    k_refine_state<<<1, 64, 0, h->stream>>>(h->P, cur_state(h), og[1], og[2], factor);
    // the pending selection again, over the refined regions from the moved cursor
    k_select<<<1, kSelectThreads, 0, h->stream>>>(h->P, T, cur_state(h));
    KPX_HIP(h, hipGetLastError());
    return KPX_OK;
}

int kpx_set_polish(kpx_handle* h, const kpx_polish* p)
{
    if (!h) return KPX_ERR_ARG;
    if (!p || p->steps == 0) {
        h->polish_steps = 0;
        return KPX_OK;
    }
    if (p->steps < 0 || p->steps > 16 || !(p->lr >= 0.f) || !std::isfinite(p->lr))
        return fail(h, KPX_ERR_ARG, "polish: steps in 0..16 and a finite lr >= 0");
    if (p->goal_only != 0 && p->goal_only != 1) return fail(h, KPX_ERR_ARG, "polish: goal_only is 0 or 1");
    const float w[6] = {p->w_ctrl, p->w_obst, p->k_obst, p->d_safe, p->w_goal, p->w_len};
    for (float v : w)
        if (!std::isfinite(v)) return fail(h, KPX_ERR_ARG, "polish: finite weights");
    if (h->P.dyn != kQUAD12)
        return fail(h, KPX_ERR_ARG, "polish: the quadrotor model only");
    if (h->prm.steps_max > kPolishCkpt * kpxd::kCkpt)
        return fail(h, KPX_ERR_ARG, "polish: edges of at most 64 steps");
    KPX_HIP(h, hipFuncSetAttribute(h->P.cost == kPATH ? reinterpret_cast<const void*>(&k_polish<kPATH>)
                                                      : reinterpret_cast<const void*>(&k_polish<kTIME>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)polish_lds_bytes(h->P.n_boxes)));
    kpxd::DiffConst& C = h->polish_c;
    C = kpxd::DiffConst{};
    const float* dp = h->prob.dyn_params;
    C.inv_m = 1.0f / dp[0];
    C.inv_j[0] = 1.0f / dp[1];
    C.inv_j[1] = 1.0f / dp[2];
    C.inv_j[2] = 1.0f / dp[3];
    C.gyro[0] = dp[3] - dp[2];
    C.gyro[1] = dp[1] - dp[3];
    C.gyro[2] = dp[2] - dp[1];
    C.grav = dp[4];
    C.dt = h->prm.dt;
    for (int a = 0; a < 3; ++a) C.goal[a] = h->prob.goal_center[a];
    C.w_ctrl = p->w_ctrl;
    C.w_obst = p->w_obst;
    C.k_obst = p->k_obst;
    C.d_safe = p->d_safe;
    C.w_goal = p->w_goal;
    C.w_len = p->w_len;
    for (int c = 0; c < 4; ++c) {
        C.u_lo[c] = h->prob.u_lo[c];
        C.u_hi[c] = h->prob.u_hi[c];
    }
    C.n_boxes = h->P.n_boxes;
    h->polish_steps = p->steps;
    h->polish_lr = p->lr;
    h->polish_goal_only = p->goal_only;
    return KPX_OK;
}

int kpx_set_timing(kpx_handle* h, int32_t kernel_mask)
{
    if (!h || kernel_mask < 0 || kernel_mask > 15) return KPX_ERR_ARG;
    KPX_HIP(h, hipStreamSynchronize(h->stream));
    for (const auto& t : h->timed) {
        h->spare.push_back(t.begin);
        h->spare.push_back(t.end);
    }
    h->timed.clear();
    h->timing_mask = kernel_mask;
    h->timing_iter = 0;
    return KPX_OK;
}

int kpx_set_cost_first(kpx_handle* h, int32_t enable)
{
    if (!h || (enable != 0 && enable != 1)) return KPX_ERR_ARG;
    h->cost_first = enable == 1;
    return KPX_OK;
}

int kpx_set_timing_every(kpx_handle* h, int32_t period)
{
    if (!h || period < 1) return KPX_ERR_ARG;
    h->timing_every = period;
    h->timing_iter = 0;
    return KPX_OK;
}

int kpx_read_timing(kpx_handle* h, double ms[4], int64_t launches[4])
{
    if (!h || !ms || !launches) return KPX_ERR_ARG;
    // waits; iterations enqueued after the tree filled did not run
    kpx_counters c;
    const int rc = kpx_counters_read(h, &c);
    if (rc != KPX_OK) return rc;
    for (int k = 0; k < 4; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    for (const auto& e : h->timed) {
        if (e.iter >= c.iteration) continue;
        float t = 0.f;
        KPX_HIP(h, hipEventElapsedTime(&t, e.begin, e.end));
        ms[e.kernel] += t;
        launches[e.kernel] += 1;
    }
    return KPX_OK;
}

int kpx_stats_capacity(const kpx_handle* h, int64_t* out)
{
    if (!h || !out) return KPX_ERR_ARG;
    *out = kStatsCap;
    return KPX_OK;
}

int kpx_read_stats(kpx_handle* h, int64_t first, int64_t count, kpx_iter_stats* out)
{
    if (!h || !out || first < 0 || count < 0 || count > kStatsCap) return KPX_ERR_ARG;
    kpx_counters c;
    int rc = kpx_counters_read(h, &c);
    if (rc != KPX_OK) return rc;
    if (first + count > c.iteration || first < c.iteration - kStatsCap)
        return fail(h, KPX_ERR_ARG, "iterations not in the statistics ring");
    for (int64_t i = 0; i < count; ++i) {
        const int64_t it = first + i;
        KPX_HIP(h, hipMemcpyAsync(out + i, h->T.stats + (it & (kStatsCap - 1)), sizeof(kpx_iter_stats),
                                  hipMemcpyDeviceToHost, h->stream));
    }
    KPX_HIP(h, hipStreamSynchronize(h->stream));
    return KPX_OK;
}

int kpx_clock_rate_khz(kpx_handle* h, int64_t* out)
{
    if (!h || !out) return KPX_ERR_ARG;
    int dev = 0, rate = 0;
    KPX_HIP(h, hipGetDevice(&dev));
    KPX_HIP(h, hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, dev));
    *out = rate;
    return KPX_OK;
}

int kpx_philox(const uint32_t* counter_key, int64_t n, uint32_t* out)
{
    if (n < 0 || (n > 0 && (!counter_key || !out))) return KPX_ERR_ARG;
    if (n == 0) return KPX_OK;
    uint32_t *din = nullptr, *dout = nullptr;
    int rc = KPX_OK;
    if (hipMalloc(&din, sizeof(uint32_t) * 6 * n) != hipSuccess) return KPX_ERR_OOM;
    if (hipMalloc(&dout, sizeof(uint32_t) * 4 * n) != hipSuccess) {
        (void)hipFree(din);
        return KPX_ERR_OOM;
    }
    if (hipMemcpy(din, counter_key, sizeof(uint32_t) * 6 * n, hipMemcpyHostToDevice) != hipSuccess) rc = KPX_ERR_DEVICE;
    if (rc == KPX_OK) {
        k_philox_eval<<<(unsigned)((n + 255) / 256), 256>>>(din, n, dout);
        if (hipGetLastError() != hipSuccess) rc = KPX_ERR_DEVICE;
    }
    if (rc == KPX_OK && hipMemcpy(out, dout, sizeof(uint32_t) * 4 * n, hipMemcpyDeviceToHost) != hipSuccess)
        rc = KPX_ERR_DEVICE;
    (void)hipFree(din);
    (void)hipFree(dout);
    return rc;
}

// Staging for kpx_philox_static: KPX_PHILOX_STATIC_MAX input records of 6
// words, then as many output records of 4.  Each device holds its own copy
// for the life of the process; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device.
constexpr long long kPhiloxStaticWords = 10LL * KPX_PHILOX_STATIC_MAX;
static __device__ __align__(256) uint32_t scratch[kPhiloxStaticWords];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static uint32_t* g_scratch_ptr[kMaxDevices];  // per device; null until looked up

// The device address of `scratch` on the current device (looked up once per
// device), or null on failure.
static uint32_t* scratch_on_current_device()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch_ptr[dev] = static_cast<uint32_t*>(p);
    }
    return g_scratch_ptr[dev];
}

int kpx_philox_static(const uint32_t* counter_key, int64_t n, uint32_t* out)
{
    if (n < 0 || n > KPX_PHILOX_STATIC_MAX || (n > 0 && (!counter_key || !out))) return KPX_ERR_ARG;
    if (n == 0) return KPX_OK;
    uint32_t* din = scratch_on_current_device();
    if (!din) return KPX_ERR_DEVICE;
    uint32_t* dout = din + 6LL * KPX_PHILOX_STATIC_MAX;
    if (hipMemcpy(din, counter_key, sizeof(uint32_t) * 6 * n, hipMemcpyHostToDevice) != hipSuccess)
        return KPX_ERR_DEVICE;
    k_philox_eval<<<(unsigned)((n + 255) / 256), 256>>>(din, n, dout);
    if (hipGetLastError() != hipSuccess) return KPX_ERR_DEVICE;
    if (hipMemcpy(out, dout, sizeof(uint32_t) * 4 * n, hipMemcpyDeviceToHost) != hipSuccess) return KPX_ERR_DEVICE;
    return KPX_OK;
}

int kpx_destroy(kpx_handle* h)
{
    if (!h) return KPX_OK;
    if (h->stream || h->base) (void)hipStreamSynchronize(h->stream);
    for (const auto& t : h->timed) {
        (void)hipEventDestroy(t.begin);
        (void)hipEventDestroy(t.end);
    }
    for (hipEvent_t e : h->spare) (void)hipEventDestroy(e);
    if (h->owns && h->base) (void)hipFree(h->base);
    delete h;
    return KPX_OK;
}

const char* kpx_status_string(int status)
{
    switch (status) {
    case KPX_OK: return "ok";
    case KPX_FULL: return "tree full (capacity pre-check failed)";
    case KPX_ERR_ARG: return "invalid argument";
    case KPX_ERR_INVALID_START: return "x_init is not in the valid set";
    case KPX_ERR_OOM: return "out of device memory or workspace too small";
    case KPX_ERR_DEVICE: return "HIP runtime error";
    case KPX_ERR_BUFFER: return "caller buffer too small";
    case KPX_ERR_STATE: return "call not valid in the current state";
    default: return "unknown status";
    }
}

const char* kpx_last_error(const kpx_handle* h)
{
    return h ? h->err.c_str() : "";
}

int kpx_batch_create(kpx_handle* const* handles, int32_t n, kpx_batch** out)
{
    if (!handles || n < 1 || !out) return KPX_ERR_ARG;
    *out = nullptr;
    for (int q = 0; q < n; ++q) {
        const kpx_handle* h = handles[q];
        if (!h || h->stream != handles[0]->stream || h->cur != handles[0]->cur || h->polish_steps > 0)
            return KPX_ERR_ARG;
        for (int r = 0; r < q; ++r)
            if (handles[r] == h) return KPX_ERR_ARG;
    }
    kpx_batch* b = new (std::nothrow) kpx_batch;
    if (!b) return KPX_ERR_OOM;
    b->hs.assign(handles, handles + n);
    for (int q = 0; q < n; ++q) {
        b->cells.push_back(handles[q]->z.n_cells);
        b->dump.push_back(handles[q]->dump_on ? 1 : 0);
    }
    b->user = handles[0]->stream;
    b->cur = handles[0]->cur;
    int dev = 0, lds_max = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess) {
        batch_free(b);
        return KPX_ERR_DEVICE;
    }
    // block maps: (query, block, blocks of the query, region blocks of the query)
    std::vector<std::vector<int4>> prop, ins, prune, fin;
    for (int q = 0; q < n; ++q) {
        const kpx_handle* h = handles[q];
        int gi = -1;
        for (size_t i = 0; i < b->groups.size(); ++i)
            if (b->groups[i].dyn == h->P.dyn && b->groups[i].cost == h->P.cost) gi = (int)i;
        if (gi < 0) {
            kpx_batch::Group g;
            g.dyn = h->P.dyn;
            g.cost = h->P.cost;
            b->groups.push_back(g);
            prop.emplace_back();
            ins.emplace_back();
            prune.emplace_back();
            fin.emplace_back();
            gi = (int)b->groups.size() - 1;
        }
        auto& g = b->groups[gi];
        g.lds = std::max(g.lds, propagate_lds_bytes(h->z, h->z.d));
        // propagate: about two slots per lane, at most one block per compute unit
        const int np = std::max(1, std::min(h->P.n_cu, (h->z.s_max + 2 * kPropBlock - 1) / (2 * kPropBlock)));
        for (int k = 0; k < np; ++k) prop[gi].push_back(make_int4(q, k, np, h->n_prune_blocks));
        for (int k = 0; k < h->z.n_tiles; ++k) ins[gi].push_back(make_int4(q, k, h->z.n_tiles, h->n_prune_blocks));
        const int nrb = region_blocks(h->z.n_cells, kRptBatch);  // the batch's region blocks of this query
        for (int k = 0; k < nrb; ++k) prune[gi].push_back(make_int4(q, k, nrb, nrb));
        for (int k = 0; k < nrb; ++k) fin[gi].push_back(make_int4(q, k, nrb, nrb));
    }
    for (auto& g : b->groups) {
        const int rc = allow_lds(propagate_kernel(g.dyn, g.cost, true), g.lds, lds_max);
        if (rc != KPX_OK) {
            batch_free(b);
            return rc;
        }
    }
    // one side stream (default priority) and join event per group after the first
    if (b->groups.size() > 1 && hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess) {
        b->ev_fork = nullptr;
        batch_free(b);
        return KPX_ERR_DEVICE;
    }
    for (size_t i = 1; i < b->groups.size(); ++i) {
        hipStream_t s = nullptr;
        hipEvent_t e = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            batch_free(b);
            return KPX_ERR_DEVICE;
        }
        b->side.push_back(s);
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            batch_free(b);
            return KPX_ERR_DEVICE;
        }
        b->ev_join.push_back(e);
    }
    size_t n4 = 0;
    for (size_t i = 0; i < b->groups.size(); ++i) n4 += prop[i].size() + ins[i].size() + prune[i].size() + fin[i].size();
    const size_t bytes = align_up(sizeof(DevProblem) * n) + align_up(sizeof(DevPtrs) * n) + sizeof(int4) * n4;
    if (hipMalloc(&b->mem, bytes) != hipSuccess) {
        b->mem = nullptr;
        batch_free(b);
        return KPX_ERR_OOM;
    }
    char* m = (char*)b->mem;
    b->d_P = (DevProblem*)m;
    b->d_T = (DevPtrs*)(m + align_up(sizeof(DevProblem) * n));
    int4* maps = (int4*)(m + align_up(sizeof(DevProblem) * n) + align_up(sizeof(DevPtrs) * n));
    std::vector<DevProblem> hp(n);
    std::vector<DevPtrs> ht(n);
    for (int q = 0; q < n; ++q) {
        hp[q] = handles[q]->P;
        ht[q] = kernel_ptrs(handles[q]);
    }
    std::vector<int4> all;
    all.reserve(n4);
    auto place = [&](std::vector<int4>& v, int4*& dst, int& count) {
        dst = maps + all.size();
        count = (int)v.size();
        all.insert(all.end(), v.begin(), v.end());
    };
    for (size_t i = 0; i < b->groups.size(); ++i) {
        place(prop[i], b->groups[i].prop, b->groups[i].n_prop);
        place(ins[i], b->groups[i].ins, b->groups[i].n_ins);
        place(prune[i], b->groups[i].prune, b->groups[i].n_prune);
        place(fin[i], b->groups[i].fin, b->groups[i].n_fin);
    }
    if (hipMemcpy(b->d_P, hp.data(), sizeof(DevProblem) * n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->d_T, ht.data(), sizeof(DevPtrs) * n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(maps, all.data(), sizeof(int4) * all.size(), hipMemcpyHostToDevice) != hipSuccess) {
        batch_free(b);
        return KPX_ERR_DEVICE;
    }
    *out = b;
    return KPX_OK;
}

int kpx_batch_set_threads(kpx_batch* b, int32_t dynamics, int32_t threads)
{
    if (!b || (threads != kPropBlock && threads != kPropBlockWide)) return KPX_ERR_ARG;
    int dev = 0, lds_max = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return bfail(b, KPX_ERR_DEVICE, "device query failed");
    for (auto& g : b->groups) {
        if (g.dyn != dynamics) continue;
        const int rc = allow_lds(propagate_kernel(g.dyn, g.cost, true, false, threads == kPropBlockWide), g.lds, lds_max);
        if (rc != KPX_OK) return bfail(b, rc, "propagate does not fit the LDS at this block size");
        g.nt = threads;
    }
    // captured iterations hold the old launches
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (auto& e : b->exec)
        if (e) {
            (void)hipGraphExecDestroy(e);
            e = nullptr;
        }
    return KPX_OK;
}

int kpx_batch_set_graph(kpx_batch* b, int32_t enable)
{
    if (!b || (enable != 0 && enable != 1)) return KPX_ERR_ARG;
    b->graph_on = enable == 1;
    return KPX_OK;
}

int kpx_batch_iterate(kpx_batch* b, int32_t n_iters)
{
    if (!b || n_iters < 0) return KPX_ERR_ARG;
    for (size_t q = 0; q < b->hs.size(); ++q) {
        const kpx_handle* h = b->hs[q];
        if (h->cur != b->cur || h->polish_steps > 0 || (h->dump_on ? 1 : 0) != b->dump[q])
            return bfail(b, KPX_ERR_STATE,
                         "a handle left the batch's step, has edge polish on or changed its recording");
    }
    for (size_t q = 0; q < b->hs.size(); ++q)
        if (b->hs[q]->z.n_cells != b->cells[q]) return bfail(b, KPX_ERR_STATE, "a handle was refined");
    if (n_iters == 0) return KPX_OK;
    // order the batch stream after the work already on the handles' stream
    if (hipEventRecord(b->ev_in, b->user) != hipSuccess || hipStreamWaitEvent(b->stream, b->ev_in, 0) != hipSuccess)
        return bfail(b, KPX_ERR_DEVICE, "stream ordering failed");
    int i = 0;
    if (b->graph_on) {
        for (; i + 2 <= n_iters; i += 2) {
            if (!b->exec[b->cur]) {
                const int rc = batch_capture(b, b->cur);
                if (rc != KPX_OK) return rc;
            }
            if (hipGraphLaunch(b->exec[b->cur], b->stream) != hipSuccess)
                return bfail(b, KPX_ERR_DEVICE, "hipGraphLaunch failed");
        }
    }
    if (i < n_iters) {
        batch_fork(b);
        for (; i < n_iters; ++i) batch_enqueue(b, b->cur ^ (i & 1));
        batch_join(b);
    }
    // parity after n_iters iterations
    if (n_iters & 1) b->cur ^= 1;
    for (kpx_handle* h : b->hs) {
        h->cur = b->cur;
        h->enq_iter += n_iters;
    }
    if (hipGetLastError() != hipSuccess) return bfail(b, KPX_ERR_DEVICE, "a batched launch failed");
    if (hipEventRecord(b->ev_out, b->stream) != hipSuccess || hipStreamWaitEvent(b->user, b->ev_out, 0) != hipSuccess)
        return bfail(b, KPX_ERR_DEVICE, "stream ordering failed");
    return KPX_OK;
}

int kpx_batch_destroy(kpx_batch* b)
{
    batch_free(b);
    return KPX_OK;
}

const char* kpx_batch_last_error(const kpx_batch* b)
{
    return b ? b->err.c_str() : "";
}

}  // extern "C"
