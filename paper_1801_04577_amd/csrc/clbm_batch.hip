// clbm_batch.hip -- many independent lattices (sizes and parameters per instance)
// advanced together: one kernel launch per time step walks a device list of
// (instance, tile) entries covering every running instance. Convergence checks,
// retirement of converged or diverged instances and compaction of the tile list
// run on the device, between the steps of a replayed HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "clbm_host.h"
#include "clbm_aux_kernels.h"

namespace clbm {

struct BatchInst {
    LatticeConst c;
    unsigned long long buf[2];  // device addresses of the two population buffers
    unsigned long long snap;    // device address of the (u_x, u_y, T) snapshot
    int tiles_x, tile_off, tile_count, pad;
};

constexpr int kBP = 6;  // per-tile partials: du2, u2, dT2, T2, bad, max|u|

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

// One time step of every instance on the active tile list (grid-stride over tiles); S is
// the storage type of every instance's populations.
template <typename S>
__global__ void __launch_bounds__(1024) k_batch_step(const BatchInst* __restrict__ insts,
                                                     const int2* __restrict__ list,
                                                     const int* __restrict__ count, int parity,
                                                     int tile_x, int tile_y)
{
    const int n = uniform_int(*count);
    for (int t = blockIdx.x; t < n; t += gridDim.x) {
        const int2 e = list[t];
        const int inst = uniform_int(e.x), tile = uniform_int(e.y);
        const BatchInst& I = insts[inst];
        const LatticeConst c = I.c;
        const int tiles_x = uniform_int(I.tiles_x);
        const int x = (tile % tiles_x) * tile_x + threadIdx.x;
        // a tile taller than the block is covered by looping over its rows
        for (int ly = threadIdx.y; ly < tile_y; ly += blockDim.y) {
        const int y = (tile / tiles_x) * tile_y + ly;
        if (x < c.nx && y < c.ny) {
            typedef typename Wide<S>::type W;
            const S* src = reinterpret_cast<const S*>(I.buf[parity]);
            S* dst = reinterpret_cast<S*>(I.buf[parity ^ 1]);
            float a[9], b[5];
            W fa[9], tb[5];
            NodeMacro m;
            switch (runtime_src(c)) {
                case kSrcVisc: gather_node<S, kSrcVisc, unsigned>(src, c, x, y, a, b); break;
                case kSrcField: gather_node<S, kSrcField, unsigned>(src, c, x, y, a, b); break;
                case kSrcVisc | kSrcField:
                    gather_node<S, kSrcVisc | kSrcField, unsigned>(src, c, x, y, a, b);
                    break;
                default: gather_node<S, 0, unsigned>(src, c, x, y, a, b); break;
            }
            collide_any(c, a, b, fa, tb, m, x, y);
            store_node<S, unsigned>(dst, c, x, y, fa, tb);
        }
        }
    }
}

// Tile k of this workgroup among n active tiles (n when there is none). With at least 8
// workgroups, the workgroups of XCD x (blockIdx % 8 == x) sweep the x-th of eight
// contiguous bands of the list (instance by instance, row by row), so the ring nodes that
// neighbouring tiles of an instance share stay in that XCD's L2.
__device__ __forceinline__ int banded_tile(int k, int n)
{
    const int b = blockIdx.x, G = gridDim.x;
    if (G < 8) {
        const int t = b + k * G;
        return t < n ? t : n;
    }
    const int x = b & 7, i = b >> 3, per = (G - x + 7) >> 3, band = (n + 7) >> 3;
    const int j = i + k * per, t = x * band + j;
    return j < band && t < n ? t : n;
}

// Waves per SIMD the LDS tile allows (160 KB per CU), at most four.
template <typename S, int TY, int NT>
constexpr int step2_waves_per_eu()
{
    constexpr int lds = 14 * Tile2<TY>::XE * Tile2<TY>::YE * (int)sizeof(S);
    constexpr int w = (160 * 1024 / lds) * (NT / 64) / 4;
    return w < 4 ? w : 4;
}

// Two time steps of every instance on the active tile list (tiles of kBlock x TY nodes,
// NT threads, grid-stride over tiles; the LDS tile is reused by each tile a workgroup
// takes). Per tile it runs the phases of k_step2, so two steps here are two steps of
// k_batch_step bit for bit. MODE: 0 = no instance has viscous heating or a source field,
// 1 = all have viscous heating and none a field, 2 = anything else (every combination of
// source terms compiled in, chosen per tile; the register budget is held at the waves
// per SIMD the LDS tile allows, at most four).
// bands != 0 deals the list to the XCDs in contiguous bands (banded_tile), else every
// workgroup strides over the whole list.
template <typename S, int MODE, int TY, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(step2_waves_per_eu<S, TY, NT>())))
k_batch_step2(const BatchInst* __restrict__ insts, const int2* __restrict__ list, const int* __restrict__ count,
              int parity, int bands)
{
    __shared__ S tile[14 * Tile2<TY>::P];
    const int n = uniform_int(*count);
    const int tid = (int)threadIdx.x;
    for (int k = 0;; ++k) {
        int t = (int)blockIdx.x + k * (int)gridDim.x;
        if (bands) t = banded_tile(k, n);
        if (t >= n) break;
        const int2 e = list[t];
        const int inst = uniform_int(e.x), id = uniform_int(e.y);
        const BatchInst& I = insts[inst];
        const LatticeConst c = I.c;
        const int tiles_x = uniform_int(I.tiles_x);
        const int X0 = (id % tiles_x) * (int)kBlock, Y0 = (id / tiles_x) * TY;
        const S* src = reinterpret_cast<const S*>(I.buf[parity]);
        S* dst = reinterpret_cast<S*>(I.buf[parity ^ 1]);
        const int src_terms = MODE == 0 ? 0 : MODE == 1 ? kSrcVisc : uniform_int(runtime_src(c));
        if (src_terms == kSrcVisc) {
            step2_phase1<S, kSrcVisc, TY, NT, unsigned>(src, c, tile, X0, Y0, tid);
            __syncthreads();
            step2_phase2<S, kSrcVisc, TY, NT, unsigned>(dst, c, tile, X0, Y0, tid);
        } else if (MODE == 2 && src_terms == kSrcField) {
            step2_phase1<S, kSrcField, TY, NT, unsigned>(src, c, tile, X0, Y0, tid);
            __syncthreads();
            step2_phase2<S, kSrcField, TY, NT, unsigned>(dst, c, tile, X0, Y0, tid);
        } else if (MODE == 2 && src_terms == (kSrcVisc | kSrcField)) {
            step2_phase1<S, kSrcVisc | kSrcField, TY, NT, unsigned>(src, c, tile, X0, Y0, tid);
            __syncthreads();
            step2_phase2<S, kSrcVisc | kSrcField, TY, NT, unsigned>(dst, c, tile, X0, Y0, tid);
        } else {
            step2_phase1<S, 0, TY, NT, unsigned>(src, c, tile, X0, Y0, tid);
            __syncthreads();
            step2_phase2<S, 0, TY, NT, unsigned>(dst, c, tile, X0, Y0, tid);
        }
        __syncthreads();  // the next tile overwrites the LDS tile
    }
}

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max_d(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    return v;
}

// Residual partials per active tile (compared with the snapshot when compare != 0),
// then the snapshot is replaced by the current fields. Partials go to the tile's
// fixed slot (its index in the full list), so the per-instance sums are formed in a
// fixed order by k_batch_finalize.
template <typename S>
__global__ void __launch_bounds__(1024) k_batch_diag(const BatchInst* __restrict__ insts,
                                                     const int2* __restrict__ list,
                                                     const int* __restrict__ count, int parity,
                                                     int tile_x, int tile_y, int compare,
                                                     double* __restrict__ part)
{
    __shared__ double lds[16][kBP];
    const int n = uniform_int(*count);
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6, nwaves = (blockDim.x * blockDim.y + 63) >> 6;
    for (int t = blockIdx.x; t < n; t += gridDim.x) {
        const int2 e = list[t];
        const int inst = uniform_int(e.x), tile = uniform_int(e.y);
        const BatchInst& I = insts[inst];
        const LatticeConst c = I.c;
        const int tiles_x = uniform_int(I.tiles_x);
        const int x = (tile % tiles_x) * tile_x + threadIdx.x;
        double acc[kBP] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        // a tile taller than the block is covered by looping over its rows
        for (int ly = threadIdx.y; ly < tile_y; ly += blockDim.y) {
        const int y = (tile / tiles_x) * tile_y + ly;
        if (x < c.nx && y < c.ny) {
            const S* src = reinterpret_cast<const S*>(I.buf[parity]);
            float* snap = reinterpret_cast<float*>(I.snap);
            float a[9], b[5];
            load_own(src, c, node_off(c, x, y), a, b);
            const NodeMacro m = macros_any(c, a, b, x, y);
            const float T = c.T0 + m.theta;
            const size_t k = (size_t)y * c.nx + x, np = (size_t)c.nx * c.ny;
            const double u2 = (double)m.ux * m.ux + (double)m.uy * m.uy;
            if (compare) {
                const double dx = m.ux - snap[k], dy = m.uy - snap[np + k], dt = T - snap[2 * np + k];
                acc[0] += dx * dx + dy * dy;
                acc[2] += dt * dt;
            }
            acc[1] += u2;
            acc[3] += (double)T * T;
            const bool ok = isfinite(m.drho) && isfinite(m.ux) && isfinite(m.uy) && isfinite(T);
            acc[4] += ok ? 0.0 : 1.0;
            acc[5] = fmax(acc[5], ok ? sqrt(u2) : 1e30);
            snap[k] = m.ux;
            snap[np + k] = m.uy;
            snap[2 * np + k] = T;
        }
        }
#pragma unroll
        for (int q = 0; q < kBP; ++q) {
            const double v = q == 5 ? wave_max_d(acc[q]) : wave_sum_d(acc[q]);
            if (lane == 0) lds[wave][q] = v;
        }
        __syncthreads();
        if (tid < kBP) {
            double v = 0.0;
            for (int w = 0; w < nwaves; ++w) v = tid == 5 ? fmax(v, lds[w][tid]) : v + lds[w][tid];
            part[(size_t)(I.tile_off + tile) * kBP + tid] = v;
        }
        __syncthreads();
    }
}

// One workgroup per instance: sums its tile partials in order, updates its step count
// and residuals, and retires it when converged, diverged or out of steps.
__global__ void __launch_bounds__(256) k_batch_finalize(const BatchInst* __restrict__ insts,
                                                        const double* __restrict__ part,
                                                        int* __restrict__ status,
                                                        long long* __restrict__ steps,
                                                        double* __restrict__ res, int K, double tol,
                                                        long long max_steps)
{
    const int i = blockIdx.x;
    if (status[i] != CLBM_INST_RUNNING) return;
    const BatchInst& I = insts[i];
    __shared__ double lds[256][kBP];
    double acc[kBP] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int t = threadIdx.x; t < I.tile_count; t += blockDim.x) {
        const double* p = part + (size_t)(I.tile_off + t) * kBP;
        for (int q = 0; q < 5; ++q) acc[q] += p[q];
        acc[5] = fmax(acc[5], p[5]);
    }
    for (int q = 0; q < kBP; ++q) lds[threadIdx.x][q] = acc[q];
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int q = 0; q < kBP; ++q)
                lds[threadIdx.x][q] = q == 5 ? fmax(lds[threadIdx.x][q], lds[threadIdx.x + s][q])
                                             : lds[threadIdx.x][q] + lds[threadIdx.x + s][q];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double* r = lds[0];
        const long long st = steps[i] + K;
        steps[i] = st;
        const double ru = r[1] > 0.0 ? sqrt(r[0] / r[1]) / K : 0.0;
        const double rT = r[3] > 0.0 ? sqrt(r[2] / r[3]) / K : 0.0;
        res[2 * i] = ru;
        res[2 * i + 1] = rT;
        int s = CLBM_INST_RUNNING;
        if (r[4] > 0.0 || !(r[5] <= 0.5)) s = CLBM_INST_DIVERGED;
        else if (fmax(ru, rT) < tol) s = CLBM_INST_CONVERGED;
        else if (st >= max_steps) s = CLBM_INST_MAX_STEPS;
        status[i] = s;
    }
}

// Compaction, phase 1 (one workgroup): exclusive scan of the running instances'
// tile counts into newoff[] and the new list length into *count.
__global__ void __launch_bounds__(1024) k_batch_scan(const BatchInst* __restrict__ insts,
                                                     const int* __restrict__ status, int n,
                                                     int* __restrict__ newoff, int* __restrict__ count)
{
    __shared__ int lds[1024];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < n; base += blockDim.x) {
        const int i = base + threadIdx.x;
        const int v = (i < n && status[i] == CLBM_INST_RUNNING) ? insts[i].tile_count : 0;
        lds[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < (int)blockDim.x; off <<= 1) {
            const int add = threadIdx.x >= (unsigned)off ? lds[threadIdx.x - off] : 0;
            __syncthreads();
            lds[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < n) newoff[i] = carry + lds[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) carry += lds[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = carry;
}

// Compaction, phase 2: every entry of the full list belonging to a running instance
// moves to its new place; entries keep their order.
__global__ void __launch_bounds__(256) k_batch_scatter(const BatchInst* __restrict__ insts,
                                                       const int* __restrict__ status,
                                                       const int* __restrict__ newoff,
                                                       const int2* __restrict__ full, int total,
                                                       int2* __restrict__ active)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= total) return;
    const int2 e = full[f];
    if (status[e.x] != CLBM_INST_RUNNING) return;
    active[newoff[e.x] + e.y] = e;
}

// Every instance on the active list (statuses and step counts unchanged).
__global__ void k_batch_activate_all(const int2* __restrict__ full, int total, int2* __restrict__ active,
                                     int* __restrict__ count)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < total) active[k] = full[k];
    if (k == 0) *count = total;
}

__global__ void k_batch_reset(int* __restrict__ status, long long* __restrict__ steps,
                              double* __restrict__ res, int n, const int2* __restrict__ full,
                              int total, int2* __restrict__ active, int* __restrict__ count)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) {
        status[k] = CLBM_INST_RUNNING;
        steps[k] = 0;
        res[2 * k] = 0.0;
        res[2 * k + 1] = 0.0;
    }
    if (k < total) active[k] = full[k];
    if (k == 0) *count = total;
}

}  // namespace clbm

using namespace clbm;

struct clbm_batch {
    int n;
    int precision;   // storage of every instance: CLBM_FP32 or CLBM_FP16_SHIFTED
    std::vector<clbm_params> p;
    std::vector<BatchInst> inst;
    std::vector<int2> full_host;
    hipStream_t stream;
    BatchInst* d_inst;
    int* d_status;
    long long* d_steps;
    double* d_res;
    int* d_newoff;
    int* d_count;
    int2* d_full;
    int2* d_active;
    double* d_part;
    double* d_dpart;   // per-instance diagnostics scratch
    double* d_dres;
    int cap_tiles;
    int total_tiles;
    int parity;
    long step;
    clbm_batch_launch launch;
    hipGraph_t graph;
    hipGraphExec_t gexec;
    int graph_K;
    double graph_tol;
    long graph_max;
};

namespace {

constexpr int kMinTileX = 64;

struct BatchLayout {
    size_t inst, status, steps, res, newoff, count, full, active, part, dpart, dres, total;
    std::vector<size_t> buf0, buf1, snap;
    int cap_tiles;
};


bool batch_launch_ok(const clbm_batch_launch& L)
{
    if (L.persistent_wgs < 0 || (L.xcd_bands != 0 && L.xcd_bands != 1)) return false;
    if (L.steps_per_launch == 2) return L.tile_x == (int)kBlock && two_step_rows_ok(L.tile_y);
    if (L.steps_per_launch != 1) return false;
    return L.tile_x >= kMinTileX && L.tile_x % 64 == 0 && L.tile_y >= 1 && L.tile_x * L.tile_y <= 1024;
}

clbm_batch_launch default_batch_launch()
{
    clbm_batch_launch L;
    L.tile_x = (int)kBlock;
    L.tile_y = kTwoStepRows;
    L.persistent_wgs = 0;
    L.steps_per_launch = 2;
    L.xcd_bands = 1;
    return L;
}

clbm_status batch_layout(int n, const clbm_params* p, BatchLayout* L)
{
    if (n < 1 || !p) return CLBM_ERR_INVALID_ARG;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, kAlign);
        return o;
    };
    long long cap = 0;
    // one storage type for the whole batch
    if (p[0].precision != CLBM_FP32 && p[0].precision != CLBM_FP16_SHIFTED) return CLBM_ERR_UNSUPPORTED;
    const size_t elem = p[0].precision == CLBM_FP16_SHIFTED ? 2 : 4;
    for (int i = 0; i < n; ++i) {
        if (p[i].precision != p[0].precision) return CLBM_ERR_UNSUPPORTED;
        clbm_status st = validate(&p[i], nullptr);
        if (st != CLBM_OK) return st;
        // the batched kernels address an instance with 32-bit element offsets
        if (buffer_elems(p[i].nx, p[i].ny) >= 0xFFFFFFFFull) return CLBM_ERR_UNSUPPORTED;
        cap += (long long)((p[i].nx + kMinTileX - 1) / kMinTileX) * p[i].ny;
    }
    if (cap >= (1LL << 30)) return CLBM_ERR_UNSUPPORTED;
    L->cap_tiles = (int)cap;
    L->inst = take(sizeof(BatchInst) * n);
    L->status = take(sizeof(int) * n);
    L->steps = take(sizeof(long long) * n);
    L->res = take(sizeof(double) * 2 * n);
    L->newoff = take(sizeof(int) * n);
    L->count = take(sizeof(int));
    L->full = take(sizeof(int2) * cap);
    L->active = take(sizeof(int2) * cap);
    L->part = take(sizeof(double) * kBP * cap);
    L->dpart = take(sizeof(double) * kDiagMaxBlocks * kDiagSums);
    L->dres = take(sizeof(double) * kDiagSums);
    L->buf0.resize(n);
    L->buf1.resize(n);
    L->snap.resize(n);
    for (int i = 0; i < n; ++i) {
        const size_t elems = buffer_elems(p[i].nx, p[i].ny);
        L->buf0[i] = take(elems * elem);
        L->buf1[i] = take(elems * elem);
        L->snap[i] = take(3 * (size_t)p[i].nx * p[i].ny * sizeof(float));
    }
    L->total = off;
    return CLBM_OK;
}

void drop_batch_graph(clbm_batch* b)
{
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
}

// Rebuild the full tile list and the per-instance tile fields for the current shape.
clbm_status apply_shape(clbm_batch* b)
{
    const clbm_batch_launch& L = b->launch;
    b->full_host.clear();
    int off = 0;
    for (int i = 0; i < b->n; ++i) {
        BatchInst& I = b->inst[i];
        const int tx = (I.c.nx + L.tile_x - 1) / L.tile_x;
        const int ty = (I.c.ny + L.tile_y - 1) / L.tile_y;
        I.tiles_x = tx;
        I.tile_off = off;
        I.tile_count = tx * ty;
        for (int t = 0; t < tx * ty; ++t) b->full_host.push_back(make_int2(i, t));
        off += tx * ty;
    }
    if (off > b->cap_tiles) return CLBM_ERR_INVALID_ARG;
    b->total_tiles = off;
    CLBM_HIP(hipMemcpyAsync(b->d_inst, b->inst.data(), sizeof(BatchInst) * b->n,
                            hipMemcpyHostToDevice, b->stream));
    CLBM_HIP(hipMemcpyAsync(b->d_full, b->full_host.data(), sizeof(int2) * off,
                            hipMemcpyHostToDevice, b->stream));
    // every instance running, active list = full list
    const int m = std::max(b->n, b->total_tiles);
    hipLaunchKernelGGL(k_batch_reset, dim3((m + 255) / 256), dim3(256), 0, b->stream, b->d_status,
                       b->d_steps, b->d_res, b->n, b->d_full, b->total_tiles, b->d_active, b->d_count);
    CLBM_HIP(hipGetLastError());
    CLBM_HIP(hipStreamSynchronize(b->stream));  // host vectors may change after return
    drop_batch_graph(b);
    return CLBM_OK;
}

dim3 step_grid(const clbm_batch* b)
{
    const int g = b->launch.persistent_wgs > 0 ? std::min(b->launch.persistent_wgs, b->total_tiles)
                                                : b->total_tiles;
    return dim3(std::max(g, 1));
}

// Adds a kernel node depending on *prev; argument values are copied by the runtime.
clbm_status add_node(hipGraph_t g, hipGraphNode_t* prev, const void* fn, dim3 grid, dim3 block,
                     void** args)
{
    hipKernelNodeParams kp;
    std::memset(&kp, 0, sizeof kp);
    kp.func = const_cast<void*>(fn);
    kp.gridDim = grid;
    kp.blockDim = block;
    kp.kernelParams = args;
    hipGraphNode_t node;
    CLBM_HIP(hipGraphAddKernelNode(&node, g, *prev ? prev : nullptr, *prev ? 1 : 0, &kp));
    *prev = node;
    return CLBM_OK;
}

template <typename S, int MODE>
const void* step2_rows(int rows)
{
    if (rows == 6) return reinterpret_cast<const void*>(&k_batch_step2<S, MODE, 6, 256>);
    if (rows == 22) return reinterpret_cast<const void*>(&k_batch_step2<S, MODE, 22, 512>);
    if (rows == 30) return reinterpret_cast<const void*>(&k_batch_step2<S, MODE, 30, 1024>);
    return reinterpret_cast<const void*>(&k_batch_step2<S, MODE, 14, 512>);
}

template <typename S>
const void* step2_for(int vh, int rows)
{
    return vh == 0 ? step2_rows<S, 0>(rows) : vh == 1 ? step2_rows<S, 1>(rows) : step2_rows<S, 2>(rows);
}

// The two-step kernel for the batch's storage type, tile height and mix of source terms
// (viscous heating, source fields) over its instances.
const void* step2_kernel(const clbm_batch* b)
{
    int vh = 0, qf = 0;
    for (int i = 0; i < b->n; ++i) {
        vh += b->p[i].viscous_heating ? 1 : 0;
        qf += b->inst[i].c.qfield ? 1 : 0;
    }
    const int mix = qf > 0 ? 2 : vh == 0 ? 0 : (vh == b->n ? 1 : 2);
    return b->precision == CLBM_FP16_SHIFTED ? step2_for<__half>(mix, b->launch.tile_y)
                                             : step2_for<float>(mix, b->launch.tile_y);
}

const void* step1_kernel(const clbm_batch* b)
{
    return b->precision == CLBM_FP16_SHIFTED ? reinterpret_cast<const void*>(&k_batch_step<__half>)
                                             : reinterpret_cast<const void*>(&k_batch_step<float>);
}

const void* diag_kernel(const clbm_batch* b)
{
    return b->precision == CLBM_FP16_SHIFTED ? reinterpret_cast<const void*>(&k_batch_diag<__half>)
                                             : reinterpret_cast<const void*>(&k_batch_diag<float>);
}

// Block shape of the one-step and diagnostics kernels (a two-step tile of kBlock x rows
// nodes is covered by kBlock x min(rows, 16) threads, rows looped).
dim3 tile_block(const clbm_batch* b)
{
    return dim3(b->launch.tile_x, std::min(b->launch.tile_y, 1024 / b->launch.tile_x));
}

clbm_status launch_batch_steps(clbm_batch* b, int nsteps)
{
    while (nsteps > 0) {
        if (b->launch.steps_per_launch == 2 && nsteps >= 2) {
            int parity = b->parity, bands = b->launch.xcd_bands;
            void* args[] = {&b->d_inst, &b->d_active, &b->d_count, &parity, &bands};
            CLBM_HIP(hipLaunchKernel(step2_kernel(b), step_grid(b), dim3(two_step_threads(b->launch.tile_y)),
                                     args, 0, b->stream));
            b->step += 2;
            nsteps -= 2;
        } else {
            int parity = b->parity, tx = b->launch.tile_x, ty = b->launch.tile_y;
            void* args[] = {&b->d_inst, &b->d_active, &b->d_count, &parity, &tx, &ty};
            CLBM_HIP(hipLaunchKernel(step1_kernel(b), step_grid(b), tile_block(b), args, 0, b->stream));
            b->step += 1;
            nsteps -= 1;
        }
        CLBM_HIP(hipGetLastError());
        b->parity ^= 1;
    }
    return CLBM_OK;
}

clbm_status launch_diag(clbm_batch* b, int compare)
{
    int parity = b->parity, tx = b->launch.tile_x, ty = b->launch.tile_y;
    void* args[] = {&b->d_inst, &b->d_active, &b->d_count, &parity, &tx, &ty, &compare, &b->d_part};
    CLBM_HIP(hipLaunchKernel(diag_kernel(b), step_grid(b), tile_block(b), args, 0, b->stream));
    return CLBM_OK;
}

// Graph: K steps, residual partials, per-instance finalize, compaction (scan, scatter).
clbm_status build_run_graph(clbm_batch* b, int K, double tol, long max_steps)
{
    drop_batch_graph(b);
    hipGraph_t g = nullptr;
    CLBM_HIP(hipGraphCreate(&g, 0));
    hipGraphNode_t prev = nullptr;
    const dim3 blk = tile_block(b);
    const dim3 grid = step_grid(b);
    int parity = b->parity, bands = b->launch.xcd_bands;
    int tx = b->launch.tile_x, ty = b->launch.tile_y;
    clbm_status st = CLBM_OK;
    // The graph is replayed from the same buffer, so it must flip the buffers an even
    // number of times: K one-step launches, or two-step launches with two one-step
    // launches in place of one of them when K/2 is odd.
    int pairs = 0, singles = K;
    if (b->launch.steps_per_launch == 2) {
        pairs = (K / 2) % 2 == 0 ? K / 2 : K / 2 - 1;
        singles = K - 2 * pairs;
    }
    for (int k = 0; k < pairs && st == CLBM_OK; ++k) {
        void* args[] = {&b->d_inst, &b->d_active, &b->d_count, &parity, &bands};
        st = add_node(g, &prev, step2_kernel(b), grid, dim3(two_step_threads(b->launch.tile_y)), args);
        parity ^= 1;
    }
    for (int k = 0; k < singles && st == CLBM_OK; ++k) {
        void* args[] = {&b->d_inst, &b->d_active, &b->d_count, &parity, &tx, &ty};
        st = add_node(g, &prev, step1_kernel(b), grid, blk, args);
        parity ^= 1;
    }
    int compare = 1;
    if (st == CLBM_OK) {
        void* args[] = {&b->d_inst, &b->d_active, &b->d_count, &parity, &tx, &ty, &compare, &b->d_part};
        st = add_node(g, &prev, diag_kernel(b), grid, blk, args);
    }
    long long maxs = max_steps;
    if (st == CLBM_OK) {
        void* args[] = {&b->d_inst, &b->d_part, &b->d_status, &b->d_steps, &b->d_res, &K, &tol, &maxs};
        st = add_node(g, &prev, reinterpret_cast<const void*>(&k_batch_finalize), dim3(b->n),
                      dim3(256), args);
    }
    int n = b->n;
    if (st == CLBM_OK) {
        void* args[] = {&b->d_inst, &b->d_status, &n, &b->d_newoff, &b->d_count};
        st = add_node(g, &prev, reinterpret_cast<const void*>(&k_batch_scan), dim3(1), dim3(1024), args);
    }
    int total = b->total_tiles;
    if (st == CLBM_OK) {
        void* args[] = {&b->d_inst, &b->d_status, &b->d_newoff, &b->d_full, &total, &b->d_active};
        st = add_node(g, &prev, reinterpret_cast<const void*>(&k_batch_scatter),
                      dim3((total + 255) / 256), dim3(256), args);
    }
    if (st != CLBM_OK) {
        (void)hipGraphDestroy(g);
        return st;
    }
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        set_last_hip_error(e, "hipGraphInstantiate", __FILE__, __LINE__);
        return CLBM_ERR_HIP;
    }
    b->graph = g;
    b->gexec = ex;
    b->graph_K = K;
    b->graph_tol = tol;
    b->graph_max = max_steps;
    return CLBM_OK;
}

// Workload signature of a batch for the tuning cache: FNV-1a (64-bit) over the instance
// count, the storage type and each instance's (nx, ny, viscous heating), as 16 hex digits.
void signature(const clbm_batch* b, char out[17])
{
    unsigned long long h = 0xcbf29ce484222325ull;
    auto mix = [&](long long v) {
        for (int k = 0; k < 8; ++k) {
            h ^= (unsigned long long)((v >> (8 * k)) & 0xff);
            h *= 0x100000001b3ull;
        }
    };
    mix(b->n);
    mix(b->precision);
    for (int i = 0; i < b->n; ++i) {
        mix(b->p[i].nx);
        mix(b->p[i].ny);
        mix(b->p[i].viscous_heating ? 1 : 0);
    }
    std::snprintf(out, 17, "%016llx", h);
}

// Integer value of "name": in one line of the cache (the format autotune writes).
bool json_int(const char* line, const char* name, int* v)
{
    char key[40];
    std::snprintf(key, sizeof key, "\"%s\": ", name);
    const char* p = std::strstr(line, key);
    return p && std::sscanf(p + std::strlen(key), "%d", v) == 1;
}

}  // namespace

extern "C" {

clbm_status clbm_batch_workspace_bytes(int n, const clbm_params* p, size_t* bytes)
{
    if (!bytes) return CLBM_ERR_INVALID_ARG;
    BatchLayout L;
    clbm_status st = batch_layout(n, p, &L);
    if (st != CLBM_OK) return st;
    *bytes = L.total;
    return CLBM_OK;
}

clbm_status clbm_batch_create(int n, const clbm_params* p, void* d_workspace, size_t bytes,
                              void* hip_stream, const clbm_batch_launch* launch, clbm_batch** out)
{
    if (!out) return CLBM_ERR_INVALID_ARG;
    *out = nullptr;
    BatchLayout L;
    clbm_status st = batch_layout(n, p, &L);
    if (st != CLBM_OK) return st;
    if (!d_workspace || ((uintptr_t)d_workspace) % kAlign != 0) return CLBM_ERR_INVALID_ARG;
    if (bytes < L.total) return CLBM_ERR_BUFFER_TOO_SMALL;
    clbm_batch_launch lc = launch ? *launch : default_batch_launch();
    if (!batch_launch_ok(lc)) return CLBM_ERR_INVALID_ARG;
    clbm_batch* b = new (std::nothrow) clbm_batch();
    if (!b) return CLBM_ERR_INVALID_ARG;
    char* ws = (char*)d_workspace;
    b->n = n;
    b->precision = p[0].precision;
    b->p.assign(p, p + n);
    b->inst.resize(n);
    b->stream = (hipStream_t)hip_stream;
    b->d_inst = (BatchInst*)(ws + L.inst);
    b->d_status = (int*)(ws + L.status);
    b->d_steps = (long long*)(ws + L.steps);
    b->d_res = (double*)(ws + L.res);
    b->d_newoff = (int*)(ws + L.newoff);
    b->d_count = (int*)(ws + L.count);
    b->d_full = (int2*)(ws + L.full);
    b->d_active = (int2*)(ws + L.active);
    b->d_part = (double*)(ws + L.part);
    b->d_dpart = (double*)(ws + L.dpart);
    b->d_dres = (double*)(ws + L.dres);
    b->cap_tiles = L.cap_tiles;
    b->launch = lc;
    for (int i = 0; i < n; ++i) {
        Rates r;
        (void)derive_rates(&p[i], &r);
        BatchInst& I = b->inst[i];
        std::memset(&I, 0, sizeof I);
        I.c = make_const(&p[i], r);
        I.buf[0] = (unsigned long long)(uintptr_t)(ws + L.buf0[i]);
        I.buf[1] = (unsigned long long)(uintptr_t)(ws + L.buf1[i]);
        I.snap = (unsigned long long)(uintptr_t)(ws + L.snap[i]);
    }
    st = apply_shape(b);
    if (st == CLBM_OK)
        for (int i = 0; i < n && st == CLBM_OK; ++i)
            st = clbm_batch_init(b, i, nullptr, nullptr, nullptr, nullptr);
    if (st != CLBM_OK) {
        delete b;
        return st;
    }
    *out = b;
    return CLBM_OK;
}

void clbm_batch_destroy(clbm_batch* b)
{
    if (!b) return;
    drop_batch_graph(b);
    delete b;
}

clbm_status clbm_batch_init(clbm_batch* b, int i, const float* d_rho, const float* d_ux,
                            const float* d_uy, const float* d_T)
{
    if (!b || i < 0 || i >= b->n) return CLBM_ERR_INVALID_ARG;
    const BatchInst& I = b->inst[i];
    const dim3 blk(64, 4);
    const dim3 grd = node_grid(I.c, blk);
    // the current buffer of the batch (all instances share the parity)
    if (b->precision == CLBM_FP16_SHIFTED)
        hipLaunchKernelGGL(k_init<__half>, grd, blk, 0, b->stream, (__half*)(uintptr_t)I.buf[b->parity],
                           I.c, d_rho, d_ux, d_uy, d_T);
    else
        hipLaunchKernelGGL(k_init<float>, grd, blk, 0, b->stream, (float*)(uintptr_t)I.buf[b->parity],
                           I.c, d_rho, d_ux, d_uy, d_T);
    CLBM_HIP(hipGetLastError());
    return CLBM_OK;
}

clbm_status clbm_batch_step(clbm_batch* b, int nsteps)
{
    if (!b || nsteps < 0) return CLBM_ERR_INVALID_ARG;
    if (nsteps == 0) return CLBM_OK;
    // Every instance advances, the ones a run has retired included: all instances share
    // the buffer parity, which flips with every launch. The active list is widened to
    // the full list for these steps and rebuilt from the run's statuses afterwards.
    hipLaunchKernelGGL(k_batch_activate_all, dim3((b->total_tiles + 255) / 256), dim3(256), 0, b->stream,
                       b->d_full, b->total_tiles, b->d_active, b->d_count);
    CLBM_HIP(hipGetLastError());
    clbm_status st = launch_batch_steps(b, nsteps);
    if (st != CLBM_OK) return st;
    int n = b->n, total = b->total_tiles;
    hipLaunchKernelGGL(k_batch_scan, dim3(1), dim3(1024), 0, b->stream, b->d_inst, b->d_status, n,
                       b->d_newoff, b->d_count);
    CLBM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_batch_scatter, dim3((total + 255) / 256), dim3(256), 0, b->stream, b->d_inst,
                       b->d_status, b->d_newoff, b->d_full, total, b->d_active);
    CLBM_HIP(hipGetLastError());
    return CLBM_OK;
}

clbm_status clbm_batch_reset(clbm_batch* b)
{
    if (!b) return CLBM_ERR_INVALID_ARG;
    const int m = std::max(b->n, b->total_tiles);
    hipLaunchKernelGGL(k_batch_reset, dim3((m + 255) / 256), dim3(256), 0, b->stream, b->d_status,
                       b->d_steps, b->d_res, b->n, b->d_full, b->total_tiles, b->d_active, b->d_count);
    CLBM_HIP(hipGetLastError());
    return launch_diag(b, 0);  // snapshot for the first residual window
}

clbm_status clbm_batch_run(clbm_batch* b, long max_steps, double tol, int K, long budget_steps,
                           long* steps_out, int* status_out)
{
    if (!b || K < 2 || (K % 2) != 0 || max_steps < 0 || !(tol >= 0.0)) return CLBM_ERR_INVALID_ARG;
    if (!b->gexec || b->graph_K != K || b->graph_tol != tol || b->graph_max != max_steps) {
        clbm_status st = build_run_graph(b, K, tol, max_steps);
        if (st != CLBM_OK) return st;
    }
    int count = 0;
    CLBM_HIP(hipMemcpyAsync(&count, b->d_count, sizeof(int), hipMemcpyDeviceToHost, b->stream));
    CLBM_HIP(hipStreamSynchronize(b->stream));
    long done = 0;
    while (count > 0 && done < max_steps + K && (budget_steps <= 0 || done < budget_steps)) {
        CLBM_HIP(hipGraphLaunch(b->gexec, b->stream));
        b->step += K;
        done += K;
        CLBM_HIP(hipMemcpyAsync(&count, b->d_count, sizeof(int), hipMemcpyDeviceToHost, b->stream));
        CLBM_HIP(hipStreamSynchronize(b->stream));
    }
    std::vector<long long> steps(b->n);
    std::vector<int> status(b->n);
    CLBM_HIP(hipMemcpyAsync(steps.data(), b->d_steps, sizeof(long long) * b->n,
                            hipMemcpyDeviceToHost, b->stream));
    CLBM_HIP(hipMemcpyAsync(status.data(), b->d_status, sizeof(int) * b->n, hipMemcpyDeviceToHost,
                            b->stream));
    CLBM_HIP(hipStreamSynchronize(b->stream));
    for (int i = 0; i < b->n; ++i) {
        if (steps_out) steps_out[i] = (long)steps[i];
        if (status_out) status_out[i] = status[i];
    }
    return CLBM_OK;
}

clbm_status clbm_batch_macros(clbm_batch* b, int i, float* d_rho, float* d_ux, float* d_uy, float* d_T)
{
    if (!b || i < 0 || i >= b->n) return CLBM_ERR_INVALID_ARG;
    const BatchInst& I = b->inst[i];
    const dim3 blk(64, 4);
    const dim3 grd = node_grid(I.c, blk);
    if (b->precision == CLBM_FP16_SHIFTED)
        hipLaunchKernelGGL(k_macros<__half>, grd, blk, 0, b->stream,
                           (const __half*)(uintptr_t)I.buf[b->parity], I.c, d_rho, d_ux, d_uy, d_T);
    else
        hipLaunchKernelGGL(k_macros<float>, grd, blk, 0, b->stream,
                           (const float*)(uintptr_t)I.buf[b->parity], I.c, d_rho, d_ux, d_uy, d_T);
    CLBM_HIP(hipGetLastError());
    return CLBM_OK;
}

clbm_status clbm_batch_diagnostics(clbm_batch* b, int i, clbm_diag* out)
{
    if (!b || i < 0 || i >= b->n || !out) return CLBM_ERR_INVALID_ARG;
    const BatchInst& I = b->inst[i];
    const size_t n = (size_t)I.c.nx * I.c.ny;
    const int blocks = (int)std::min<size_t>((n + kDiagBlock - 1) / kDiagBlock, kDiagMaxBlocks);
    if (b->precision == CLBM_FP16_SHIFTED)
        hipLaunchKernelGGL(k_diag<__half>, dim3(blocks), dim3(kDiagBlock), 0, b->stream,
                           (const __half*)(uintptr_t)I.buf[b->parity], I.c, (float*)(uintptr_t)I.snap, 0,
                           b->d_dpart);
    else
        hipLaunchKernelGGL(k_diag<float>, dim3(blocks), dim3(kDiagBlock), 0, b->stream,
                           (const float*)(uintptr_t)I.buf[b->parity], I.c, (float*)(uintptr_t)I.snap, 0,
                           b->d_dpart);
    CLBM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, b->stream, b->d_dpart, blocks, b->d_dres);
    CLBM_HIP(hipGetLastError());
    double r[kDiagSums];
    CLBM_HIP(hipMemcpyAsync(r, b->d_dres, sizeof r, hipMemcpyDeviceToHost, b->stream));
    long long st = 0;
    CLBM_HIP(hipMemcpyAsync(&st, b->d_steps + i, sizeof st, hipMemcpyDeviceToHost, b->stream));
    CLBM_HIP(hipStreamSynchronize(b->stream));
    std::memset(out, 0, sizeof *out);
    out->step = (long)st;
    out->mass = (double)n + r[0];
    out->sum_u2 = r[1];
    out->sum_T2 = r[3];
    const clbm_params& p = b->p[i];
    const int len[4] = {p.ny, p.ny, p.nx, p.nx};
    for (int s = 0; s < 4; ++s) {
        if (p.side[s].kind != CLBM_WALL) continue;
        out->dTdn[s] = r[5 + s] / len[s];
        out->T_wall[s] = r[9 + s] / len[s];
        out->wall_flux[s] = r[15 + s] / len[s];
    }
    out->nan_count = (long)r[13];
    return out->nan_count > 0 ? CLBM_ERR_NAN : CLBM_OK;
}

clbm_status clbm_batch_residual(clbm_batch* b, int i, double out[2])
{
    if (!b || i < 0 || i >= b->n || !out) return CLBM_ERR_INVALID_ARG;
    CLBM_HIP(hipMemcpyAsync(out, b->d_res + 2 * i, 2 * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    CLBM_HIP(hipStreamSynchronize(b->stream));
    return CLBM_OK;
}

clbm_status clbm_batch_set_source_field(clbm_batch* b, int i, const float* d_q)
{
    if (!b || i < 0 || i >= b->n) return CLBM_ERR_INVALID_ARG;
    b->inst[i].c.qfield = d_q;
    CLBM_HIP(hipMemcpyAsync(b->d_inst + i, &b->inst[i], sizeof(BatchInst), hipMemcpyHostToDevice, b->stream));
    CLBM_HIP(hipStreamSynchronize(b->stream));  // the host copy may change after return
    drop_batch_graph(b);                        // the kernel variant may change with the mix
    return CLBM_OK;
}

clbm_status clbm_batch_set_launch(clbm_batch* b, const clbm_batch_launch* launch)
{
    if (!b || !launch || !batch_launch_ok(*launch)) return CLBM_ERR_INVALID_ARG;
    b->launch = *launch;
    return apply_shape(b);
}

clbm_status clbm_batch_autotune(clbm_batch* b, int steps, const char* cache_path,
                                clbm_batch_launch* best)
{
    if (!b || steps < 1) return CLBM_ERR_INVALID_ARG;
    // {tile_x, tile_y, steps per launch}: one-step tiles, then the two-step tile heights
    static const int shapes[][3] = {{64, 1, 1}, {64, 2, 1}, {64, 4, 1}, {64, 8, 1}, {128, 1, 1},
                                    {128, 2, 1}, {128, 4, 1}, {256, 1, 1}, {256, 2, 1}, {256, 4, 1},
                                    {512, 1, 1}, {512, 2, 1}, {(int)kBlock, 6, 2},
                                    {(int)kBlock, 14, 2}, {(int)kBlock, 22, 2}, {(int)kBlock, 30, 2}};
    static const int wgs[] = {0, 2048, 8192};
    char sig[17];
    signature(b, sig);
    FILE* fp = cache_path ? std::fopen(cache_path, "a") : nullptr;
    hipEvent_t e0, e1;
    CLBM_HIP(hipEventCreate(&e0));
    CLBM_HIP(hipEventCreate(&e1));
    double best_ms = 1e300;
    clbm_batch_launch best_L = b->launch;
    long long nodes = 0;
    for (int i = 0; i < b->n; ++i) nodes += (long long)b->p[i].nx * b->p[i].ny;
    clbm_status st = CLBM_OK;
    for (const auto& sh : shapes) {
        for (int bands = 0; bands < (sh[2] == 2 ? 2 : 1); ++bands) {
            for (int w : wgs) {
                clbm_batch_launch L;
                L.tile_x = sh[0];
                L.tile_y = sh[1];
                L.steps_per_launch = sh[2];
                L.persistent_wgs = w;
                L.xcd_bands = sh[2] == 2 ? bands : 0;
                if (!batch_launch_ok(L)) continue;
                b->launch = L;
                st = apply_shape(b);
                if (st != CLBM_OK) break;
                if (w > 0 && w >= b->total_tiles) continue;  // same as one workgroup per tile
                st = launch_batch_steps(b, 2);               // warm-up
                if (st != CLBM_OK) break;
                CLBM_HIP(hipEventRecord(e0, b->stream));
                st = launch_batch_steps(b, 2 * ((steps + 1) / 2));
                if (st != CLBM_OK) break;
                CLBM_HIP(hipEventRecord(e1, b->stream));
                CLBM_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                CLBM_HIP(hipEventElapsedTime(&ms, e0, e1));
                const double per = ms / (2 * ((steps + 1) / 2));
                if (fp)
                    std::fprintf(fp, "{\"signature\": \"%s\", \"tile_x\": %d, \"tile_y\": %d, "
                                     "\"persistent_wgs\": %d, \"steps_per_launch\": %d, \"xcd_bands\": %d, "
                                     "\"instances\": %d, \"nodes\": %lld, \"ms_per_step\": %.6f, "
                                     "\"mlups\": %.1f}\n",
                                 sig, L.tile_x, L.tile_y, L.persistent_wgs, L.steps_per_launch, L.xcd_bands,
                                 b->n, nodes, per, nodes / (per * 1e-3) / 1e6);
                if (per < best_ms) {
                    best_ms = per;
                    best_L = L;
                }
            }
            if (st != CLBM_OK) break;
        }
        if (st != CLBM_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (fp && st == CLBM_OK)
        std::fprintf(fp, "{\"signature\": \"%s\", \"best\": 1, \"tile_x\": %d, \"tile_y\": %d, "
                         "\"persistent_wgs\": %d, \"steps_per_launch\": %d, \"xcd_bands\": %d, "
                         "\"ms_per_step\": %.6f}\n",
                     sig, best_L.tile_x, best_L.tile_y, best_L.persistent_wgs, best_L.steps_per_launch,
                     best_L.xcd_bands, best_ms);
    if (fp) std::fclose(fp);
    b->launch = best_L;
    clbm_status st2 = apply_shape(b);
    if (st != CLBM_OK) return st;
    if (best) *best = best_L;
    return st2;
}

clbm_status clbm_batch_tune_lookup(const clbm_batch* b, const char* cache_path, clbm_batch_launch* out,
                                   int* found)
{
    if (!b || !cache_path || !out || !found) return CLBM_ERR_INVALID_ARG;
    *found = 0;
    char sig[17];
    signature(b, sig);
    FILE* fp = std::fopen(cache_path, "r");
    if (!fp) return CLBM_OK;
    char line[1024];
    char key[48];
    std::snprintf(key, sizeof key, "\"signature\": \"%s\"", sig);
    while (std::fgets(line, sizeof line, fp)) {
        if (!std::strstr(line, key) || !std::strstr(line, "\"best\": 1")) continue;
        clbm_batch_launch L;
        if (json_int(line, "tile_x", &L.tile_x) && json_int(line, "tile_y", &L.tile_y) &&
            json_int(line, "persistent_wgs", &L.persistent_wgs) &&
            json_int(line, "steps_per_launch", &L.steps_per_launch) && json_int(line, "xcd_bands", &L.xcd_bands) &&
            batch_launch_ok(L)) {
            *out = L;  // the last matching line wins
            *found = 1;
        }
    }
    std::fclose(fp);
    return CLBM_OK;
}

}  // extern "C"
