// clbm_kernels.h -- fused pull-scheme time step and its helpers (gfx950).
//
// One thread updates one node per row it owns: it gathers the 14 populations
// that stream into the node (Eq. 11, Eq. 21), substitutes the wall links
// (half-way bounce-back for f, Sec. 3; general bounce-back for g, Eq. 26-28),
// collides (clbm_device.h) and stores the 14 post-collision populations at its
// own address in the other buffer. Storage is block-interleaved (clbm_device.h):
// population i of node (x, y) sits at node_off(x, y) + i * kBlock, flow populations
// 0..8 then temperature populations 9..13.
#pragma once

#include "clbm_device.h"

namespace clbm {

// The 14 stored populations of one node.
template <typename S>
__device__ __forceinline__ void load_own(const S* __restrict__ src, const LatticeConst& c,
                                         unsigned own, float a[9], float b[5])
{
    constexpr unsigned P = kBlock;
#pragma unroll
    for (int i = 0; i < 9; ++i) a[i] = ld(src + i * P + own);
#pragma unroll
    for (int i = 0; i < 5; ++i) b[i] = ld(src + (9 + i) * P + own);
}

// T - T0 at time t of the node at element offset off (node_off), from its stored post-collision
// populations: sum g* - Q/2, with Q the node's own source under VH.
template <typename S, bool VH>
__device__ __forceinline__ float theta_post(const S* __restrict__ src, const LatticeConst& c,
                                            unsigned off)
{
    constexpr unsigned P = kBlock;
    const S* gs = src + 9 * P;
    if constexpr (VH) {
        float a[9], b[5];
        load_own(src, c, off, a, b);
        return macros_from_post<true>(c, a, b).theta;
    } else {
        const float s = ld(gs + off) + ld(gs + P + off) + ld(gs + 2 * P + off) + ld(gs + 3 * P + off)
                        + ld(gs + 4 * P + off);
        return s - 0.5f * c.Q;
    }
}

// Gather the pre-collision deviations of node (x, y) at time t+1 from the
// post-collision buffer at time t, with all wall substitutions applied.
// VH: the heat source includes the viscous dissipation (wall temperatures need the
// source of the nodes they are extrapolated from).
template <typename S, bool VH = false>
__device__ __forceinline__ void gather_node(const S* __restrict__ src, const LatticeConst& c, int x,
                                            int y, float a[9], float b[5])
{
    const int nx = c.nx, ny = c.ny;
    constexpr unsigned P = kBlock;
    // Source coordinates of the links; a link whose source lies outside a wall is
    // flagged and its source clamped to the node itself (the address is never used).
    int xm = x - 1, xp = x + 1, ym = y - 1, yp = y + 1;
    bool oxm = false, oxp = false, oym = false, oyp = false;
    if (xm < 0) { if (c.periodic_x) xm = nx - 1; else { oxm = true; xm = x; } }
    if (xp >= nx) { if (c.periodic_x) xp = 0; else { oxp = true; xp = x; } }
    if (ym < 0) { if (c.periodic_y) ym = ny - 1; else { oym = true; ym = y; } }
    if (yp >= ny) { if (c.periodic_y) yp = 0; else { oyp = true; yp = y; } }
    // Offsets of the three source rows and the three source columns (node_off split).
    const unsigned rC = (unsigned)y * c.rowlen, rM = (unsigned)ym * c.rowlen, rP = (unsigned)yp * c.rowlen;
    auto col = [](int xx) { return ((unsigned)xx / kBlock) * kBlockElems + ((unsigned)xx % kBlock); };
    const unsigned cM = col(xm), cC = col(x), cP = col(xp);
    const unsigned own = rC + cC;

    // Eq. (11) pull form f_i(x, t+1) = f_i*(x - e_i, t); a wall link takes the
    // opposite population of the node itself (half-way bounce-back).
    a[0] = ld(src + own);
    a[1] = ld(src + (oxm ? 3 * P + own : 1 * P + rC + cM));
    a[2] = ld(src + (oym ? 4 * P + own : 2 * P + rM + cC));
    a[3] = ld(src + (oxp ? 1 * P + own : 3 * P + rC + cP));
    a[4] = ld(src + (oyp ? 2 * P + own : 4 * P + rP + cC));
    a[5] = ld(src + ((oxm | oym) ? 7 * P + own : 5 * P + rM + cM));
    a[6] = ld(src + ((oxp | oym) ? 8 * P + own : 6 * P + rM + cP));
    a[7] = ld(src + ((oxp | oyp) ? 5 * P + own : 7 * P + rP + cP));
    a[8] = ld(src + ((oxm | oyp) ? 6 * P + own : 8 * P + rP + cM));
    // Eq. (21); a wall link loads the opposite population of the node, completed below.
    const S* gs = src + 9 * P;
    b[0] = ld(gs + own);
    b[1] = ld(gs + (oxm ? 3 * P + own : 1 * P + rC + cM));
    b[2] = ld(gs + (oym ? 4 * P + own : 2 * P + rM + cC));
    b[3] = ld(gs + (oxp ? 1 * P + own : 3 * P + rC + cP));
    b[4] = ld(gs + (oyp ? 2 * P + own : 4 * P + rP + cC));

    if (oxm | oxp | oym | oyp) {
        // Eq. (26): g_i(x_f, t+1) = -g*_opp(i)(x_f, t) + c_T^2 T_w, with T_w from Eq. (28)
        // using T at this node (T1) and one node further from the wall (T2) at time t.
        // Stored post-collision data give T = sum g* - Q/2 (the collision adds Q).
        auto theta_at = [&](unsigned off) { return theta_post<S, VH>(src, c, off); };
        const float th1 = theta_at(own);
        if (oxm) {
            const float tw = c.a1[0] * th1 + c.a2[0] * theta_at(node_off(c, x + 1, y)) + c.a3[0];
            b[1] = -b[1] + CT2 * tw;
        }
        if (oxp) {
            const float tw = c.a1[1] * th1 + c.a2[1] * theta_at(node_off(c, x - 1, y)) + c.a3[1];
            b[3] = -b[3] + CT2 * tw;
        }
        if (oym) {
            const float tw = c.a1[2] * th1 + c.a2[2] * theta_at(own + c.rowlen) + c.a3[2];
            b[2] = -b[2] + CT2 * tw;
        }
        if (oyp) {
            const float tw = c.a1[3] * th1 + c.a2[3] * theta_at(own - c.rowlen) + c.a3[3];
            b[4] = -b[4] + CT2 * tw;
        }
        if (c.moving) {
            // Tangentially moving wall: a bounced link j gains 2 w_j rho (e_j . u_w)/c_s^2,
            // rho of the node at time t; u_w collects the speeds of the walls the link
            // crosses (x component from a y wall, y component from an x wall). Links
            // normal to a wall have e_j . u_w = 0.
            float r = 1.f;
#pragma unroll
            for (int i = 0; i < 9; ++i) r += ld(src + i * P + own);
            const float k = 6.f * r * wgt(5);
            const float u_bot = oym ? c.uw[2] : 0.f, u_top = oyp ? c.uw[3] : 0.f;   // along x
            const float v_lft = oxm ? c.uw[0] : 0.f, v_rgt = oxp ? c.uw[1] : 0.f;   // along y
            if (oxm | oym) a[5] += k * (u_bot + v_lft);
            if (oxp | oym) a[6] += k * (-u_bot + v_rgt);
            if (oxp | oyp) a[7] += k * (-u_top - v_rgt);
            if (oxm | oyp) a[8] += k * (u_top - v_lft);
        }
    }
}

// Store the post-collision state of one node: the deviations, computed wider than the
// storage, with the unbiased rounding of st_sr. One hash per node mixes the bits of all
// 14 results; the k-th store takes h + k * 0x9E3779B9 (a Weyl sequence), each uniform
// on its own.
template <typename S>
__device__ __forceinline__ void store_node(S* __restrict__ dst, const LatticeConst& c, unsigned own,
                                           const typename Wide<S>::type fa[9],
                                           const typename Wide<S>::type tb[5])
{
    constexpr unsigned P = kBlock;
    unsigned acc = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) acc = ((acc << 5) | (acc >> 27)) ^ hash_bits(fa[i]);
#pragma unroll
    for (int i = 0; i < 5; ++i) acc = ((acc << 5) | (acc >> 27)) ^ hash_bits(tb[i]);
    const unsigned h = mix32(acc);
#pragma unroll
    for (int i = 0; i < 9; ++i) st_sr(dst + i * P + own, fa[i], h + (unsigned)i * 0x9E3779B9u);
#pragma unroll
    for (int i = 0; i < 5; ++i) st_sr(dst + (9 + i) * P + own, tb[i], h + (unsigned)(9 + i) * 0x9E3779B9u);
}


// Tile -> workgroup map. With xcd_remap the grid is padded to a multiple of 8 and
// workgroup b (dispatched to XCD b % 8) takes tile (b % 8) * (grid/8) + b/8, so
// each XCD sweeps one contiguous band of tiles.
__device__ __forceinline__ int tile_of_block(int total, int remap)
{
    const int b = blockIdx.x;
    if (!remap) return b;
    const int per = gridDim.x >> 3;
    return (b & 7) * per + (b >> 3);
}

template <typename S, int ROWS, bool VH>
__global__ void __launch_bounds__(1024) k_step(const S* __restrict__ src, S* __restrict__ dst,
                                               const LatticeConst c, int tiles_x, int tiles_total,
                                               int remap)
{
    const int t = tile_of_block(tiles_total, remap);
    if (t >= tiles_total) return;
    const int tx = t % tiles_x, ty = t / tiles_x;
    const int x = tx * blockDim.x + threadIdx.x;
    const int y0 = (ty * blockDim.y + threadIdx.y) * ROWS;
    if (x >= c.nx) return;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int y = y0 + r;
        if (y < c.ny) {
            float a[9], b[5];
            typename Wide<S>::type fa[9], tb[5];
            gather_node<S, VH>(src, c, x, y, a, b);
            NodeMacro m;
            collide<typename Wide<S>::type, VH>(c, a, b, fa, tb, m);
            store_node(dst, c, node_off(c, x, y), fa, tb);
        }
    }
}

}  // namespace clbm
