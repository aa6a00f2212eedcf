// clbm_aux_kernels.h -- kernels around the fused step (gfx950): initial state,
// macroscopic fields, population export and the diagnostics reductions.
#pragma once

#include "clbm_kernels.h"

namespace clbm {

// Node (x, y) of this thread under a one-dimensional grid of blockDim.x x blockDim.y
// blocks that cover the lattice row of blocks by row of blocks (a one-dimensional grid
// has no per-dimension limit on the block count).
__device__ __forceinline__ void grid_node(const LatticeConst& c, int& x, int& y)
{
    const unsigned nbx = ((unsigned)c.nx + blockDim.x - 1) / blockDim.x;
    const unsigned by = blockIdx.x / nbx, bx = blockIdx.x - by * nbx;
    x = (int)(bx * blockDim.x + threadIdx.x);
    y = (int)(by * blockDim.y + threadIdx.y);
}

// Equilibrium at the given fields followed by one collision: the stored state is
// the post-collision state at t = 0.
template <typename S>
__global__ void __launch_bounds__(256) k_init(S* __restrict__ dst, const LatticeConst c,
                                              const float* __restrict__ rho,
                                              const float* __restrict__ ux,
                                              const float* __restrict__ uy,
                                              const float* __restrict__ T)
{
    int x, y;
    grid_node(c, x, y);
    if (x >= c.nx || y >= c.ny) return;
    const size_t k = (size_t)y * c.nx + x;
    const float drho = rho ? rho[k] - 1.f : 0.f;
    const float vx = ux ? ux[k] : 0.f;
    const float vy = uy ? uy[k] : 0.f;
    const float th = T ? T[k] - c.T0 : 0.f;
    float a[9], b[5];
    typename Wide<S>::type fa[9], tb[5];
    equilibrium(drho, vx, vy, th, c.T0, a, b);
    NodeMacro m;
    collide_any(c, a, b, fa, tb, m, x, y);
    store_node(dst, c, x, y, fa, tb);
}

template <typename S>
__global__ void __launch_bounds__(256) k_macros(const S* __restrict__ src, const LatticeConst c,
                                                float* __restrict__ rho, float* __restrict__ ux,
                                                float* __restrict__ uy, float* __restrict__ T)
{
    int x, y;
    grid_node(c, x, y);
    if (x >= c.nx || y >= c.ny) return;
    float a[9], b[5];
    load_own(src, c, node_off(c, x, y), a, b);
    const NodeMacro m = macros_any(c, a, b, x, y);
    const size_t k = (size_t)y * c.nx + x;
    if (rho) rho[k] = 1.f + m.drho;
    if (ux) ux[k] = m.ux;
    if (uy) uy[k] = m.uy;
    if (T) T[k] = c.T0 + m.theta;
}

template <typename S>
__global__ void __launch_bounds__(256) k_populations(const S* __restrict__ src, const LatticeConst c,
                                                     float* __restrict__ f, float* __restrict__ g)
{
    int x, y;
    grid_node(c, x, y);
    if (x >= c.nx || y >= c.ny) return;
    const size_t own = node_off(c, x, y);
    const size_t n = (size_t)c.nx * c.ny, k = (size_t)y * c.nx + x;
    if (f)
        for (int i = 0; i < 9; ++i) f[i * n + k] = ld(src + i * kBlock + own);
    if (g)
        for (int i = 0; i < 5; ++i) g[i * n + k] = ld(src + (9 + i) * kBlock + own);
}

// Diagnostics. Per node: rho - 1, |u|^2, |u - u_snap|^2, T^2, (T - T_snap)^2, NaN flag;
// per wall node: outward dT/dn (Eq. 27), T_w (Eq. 28) and the heat flux of the
// bounced link. Sums in FP64: wave64
// shuffles, then LDS across the waves of the workgroup, then one partial per
// workgroup; k_diag_final adds the partials in a fixed order.
constexpr int kDiagSums = 19;  // drho, u2, du2, T2, dT2, dTdn[4], Tw[4], nan, count, flux[4]
constexpr int kDiagBlock = 256;
constexpr int kDiagMaxBlocks = 1024;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

template <typename S>
__global__ void __launch_bounds__(kDiagBlock) k_diag(const S* __restrict__ src, const LatticeConst c,
                                                     float* __restrict__ snap, int have_snap,
                                                     double* __restrict__ partial)
{
    double acc[kDiagSums];
#pragma unroll
    for (int k = 0; k < kDiagSums; ++k) acc[k] = 0.0;
    const size_t n = (size_t)c.nx * c.ny;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        const int y = (int)(k / c.nx), x = (int)(k - (size_t)y * c.nx);
        const size_t own = node_off(c, x, y);
        float a[9], b[5];
        load_own(src, c, own, a, b);
        const NodeMacro m = macros_any(c, a, b, x, y);
        const float T = c.T0 + m.theta;
        const bool bad = !(isfinite(m.drho) && isfinite(m.ux) && isfinite(m.uy) && isfinite(T));
        acc[0] += m.drho;
        acc[1] += (double)m.ux * m.ux + (double)m.uy * m.uy;
        acc[3] += (double)T * T;
        if (have_snap) {
            const double dx = m.ux - snap[k], dy = m.uy - snap[n + k], dt = T - snap[2 * n + k];
            acc[2] += dx * dx + dy * dy;
            acc[4] += dt * dt;
        }
        snap[k] = m.ux;
        snap[n + k] = m.uy;
        snap[2 * n + k] = T;
        acc[13] += bad ? 1.0 : 0.0;
        // Wall nodes: Eq. (27)-(28) with T1 at the node and T2 one node inward.
        const bool wall[4] = {!c.periodic_x && x == 0, !c.periodic_x && x == c.nx - 1,
                              !c.periodic_y && y == 0, !c.periodic_y && y == c.ny - 1};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if (!wall[s]) continue;
            const int x2 = s == 0 ? x + 1 : (s == 1 ? x - 1 : x);
            const int y2 = s == 2 ? y + 1 : (s == 3 ? y - 1 : y);
            const size_t o2 = node_off(c, x2, y2);
            const float th2 = theta_post_any<S>(src, c, o2, x2, y2);
            const float thw = c.a1[s] * m.theta + c.a2[s] * th2 + c.a3[s];
            acc[5 + s] += (8.0 * thw - 9.0 * m.theta + th2) / 3.0;
            acc[9 + s] += (double)c.T0 + thw;
            // Heat carried through the wall by the link that crosses it (Eq. 26): g*
            // leaves, -g* + c_T^2 T_w comes back, a net 2 g* - c_T^2 T_w per step.
            const float gout = b[s == 0 ? 3 : (s == 1 ? 1 : (s == 2 ? 4 : 2))] + 0.2f * c.T0;
            acc[15 + s] += 2.0 * gout - 0.4 * ((double)c.T0 + thw);
        }
        acc[14] += 1.0;
    }
    __shared__ double lds[kDiagBlock / 64][kDiagSums];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kDiagSums; ++k) {
        const double v = wave_sum(acc[k]);
        if (lane == 0) lds[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < kDiagSums) {
        double v = 0.0;
        for (int w = 0; w < kDiagBlock / 64; ++w) v += lds[w][threadIdx.x];
        partial[(size_t)blockIdx.x * kDiagSums + threadIdx.x] = v;
    }
}

static __global__ void __launch_bounds__(256) k_diag_final(const double* __restrict__ partial, int nparts,
                                                    double* __restrict__ out)
{
    __shared__ double lds[256];
    for (int k = 0; k < kDiagSums; ++k) {
        double v = 0.0;
        for (int p = threadIdx.x; p < nparts; p += blockDim.x) v += partial[(size_t)p * kDiagSums + k];
        lds[threadIdx.x] = v;
        __syncthreads();
        for (int s = blockDim.x / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = lds[0];
        __syncthreads();
    }
}

}  // namespace clbm
