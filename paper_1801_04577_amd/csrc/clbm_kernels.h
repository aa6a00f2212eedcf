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

// Where a step reads the populations of time t: the stored buffer (GlobalMem) or, in
// the two-step kernel, the workgroup's tile in LDS (TileMem). Each gives the element
// offset of a neighbour's row and column part and the stride P between the populations
// of one node. In a periodic direction GlobalMem wraps the neighbour; TileMem does not,
// since its halo already holds the wrapped nodes. Element offsets into the stored buffer
// have the type O: 32-bit where the buffer holds fewer than 2^32 elements, else 64-bit
// (the host picks the kernel); offsets within a row and in LDS are 32-bit.
template <typename S, typename O = size_t>
struct GlobalMem {
    typedef S Elem;
    typedef O Off;
    const S* __restrict__ p;
    unsigned rowlen;
    int nx, ny;
    static constexpr unsigned P = kBlock;
    __device__ __forceinline__ Off row(int y, int d) const
    {
        int yy = y + d;
        yy = yy < 0 ? ny - 1 : (yy >= ny ? 0 : yy);
        return (Off)(unsigned)yy * rowlen;
    }
    __device__ __forceinline__ unsigned col(int x, int d) const
    {
        int xx = x + d;
        xx = xx < 0 ? nx - 1 : (xx >= nx ? 0 : xx);
        return ((unsigned)xx / kBlock) * kBlockElems + ((unsigned)xx % kBlock);
    }
};

template <typename O = size_t, typename S>
__device__ __forceinline__ GlobalMem<S, O> global_mem(const S* __restrict__ src, const LatticeConst& c)
{
    return GlobalMem<S, O>{src, c.rowlen, c.nx, c.ny};
}

// The 14 populations of the node at offset own.
template <typename S, unsigned P, typename Off>
__device__ __forceinline__ void load_pops(const S* p, Off own, float a[9], float b[5])
{
#pragma unroll
    for (int i = 0; i < 9; ++i) a[i] = ld(p + i * P + own);
#pragma unroll
    for (int i = 0; i < 5; ++i) b[i] = ld(p + (9 + i) * P + own);
}

// The 14 stored populations of one node (own = node_off).
template <typename S>
__device__ __forceinline__ void load_own(const S* __restrict__ src, const LatticeConst& c,
                                         size_t own, float a[9], float b[5])
{
    load_pops<S, kBlock>(src, own, a, b);
}

// T - T0 at time t of the node at element offset off, from its post-collision
// populations: sum g* - Q/2, with Q the node's own source (qx its source-field value).
template <int SRC, typename S, unsigned P, typename Off>
__device__ __forceinline__ float theta_at(const S* p, const LatticeConst& c, Off off, float qx)
{
    const S* gs = p + 9 * P;
    if constexpr ((SRC & kSrcVisc) != 0) {
        float a[9], b[5];
        load_pops<S, P>(p, off, a, b);
        return macros_from_post<SRC>(c, a, b, qx).theta;
    } else {
        const float s = ld(gs + off) + ld(gs + P + off) + ld(gs + 2 * P + off) + ld(gs + 3 * P + off)
                        + ld(gs + 4 * P + off);
        return s - 0.5f * ((SRC & kSrcField) ? c.Q + qx : c.Q);
    }
}

template <typename S, int SRC>
__device__ __forceinline__ float theta_post(const S* __restrict__ src, const LatticeConst& c,
                                            size_t off, float qx)
{
    return theta_at<SRC, S, kBlock>(src, c, off, qx);
}

// theta_post with the source terms decided at run time, for node (x, y) at offset off.
template <typename S>
__device__ __forceinline__ float theta_post_any(const S* __restrict__ src, const LatticeConst& c,
                                                size_t off, int x, int y)
{
    switch (runtime_src(c)) {
        case kSrcVisc: return theta_post<S, kSrcVisc>(src, c, off, 0.f);
        case kSrcField: return theta_post<S, kSrcField>(src, c, off, node_q<kSrcField>(c, x, y));
        case kSrcVisc | kSrcField:
            return theta_post<S, kSrcVisc | kSrcField>(src, c, off, node_q<kSrcField>(c, x, y));
        default: return theta_post<S, 0>(src, c, off, 0.f);
    }
}

// Gather the pre-collision deviations of node (x, y) at time t+1 from the
// post-collision populations at time t, with all wall substitutions applied.
// SRC: the source terms (wall temperatures need the source of the nodes they are
// extrapolated from).
template <int SRC, typename Mem>
__device__ __forceinline__ void gather_mem(const Mem& mem, const LatticeConst& c, int x, int y,
                                           float a[9], float b[5])
{
    constexpr unsigned P = Mem::P;
    typedef typename Mem::Off Off;
    // A link whose source lies outside a wall is flagged, and its source is the node
    // itself (the address is never used).
    const bool oxm = !c.periodic_x && x == 0, oxp = !c.periodic_x && x == c.nx - 1;
    const bool oym = !c.periodic_y && y == 0, oyp = !c.periodic_y && y == c.ny - 1;
    // Offsets of the three source rows and the three source columns.
    const Off rC = mem.row(y, 0);
    const unsigned cC = mem.col(x, 0);
    const Off rM = oym ? rC : mem.row(y, -1), rP = oyp ? rC : mem.row(y, 1);
    const unsigned cM = oxm ? cC : mem.col(x, -1), cP = oxp ? cC : mem.col(x, 1);
    const Off own = rC + cC;
    const auto* src = mem.p;

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
    const auto* gs = src + 9 * P;
    b[0] = ld(gs + own);
    b[1] = ld(gs + (oxm ? 3 * P + own : 1 * P + rC + cM));
    b[2] = ld(gs + (oym ? 4 * P + own : 2 * P + rM + cC));
    b[3] = ld(gs + (oxp ? 1 * P + own : 3 * P + rC + cP));
    b[4] = ld(gs + (oyp ? 2 * P + own : 4 * P + rP + cC));

    if (oxm | oxp | oym | oyp) {
        // Eq. (26): g_i(x_f, t+1) = -g*_opp(i)(x_f, t) + c_T^2 T_w, with T_w from Eq. (28)
        // using T at this node (T1) and one node further from the wall (T2) at time t.
        // Post-collision data give T = sum g* - Q/2 (the collision adds Q).
        auto theta = [&](Off off, int qx, int qy) {
            return theta_at<SRC, typename Mem::Elem, P>(src, c, off, node_q<SRC>(c, qx, qy));
        };
        const float th1 = theta(own, x, y);
        if (oxm) {
            const float tw = c.a1[0] * th1 + c.a2[0] * theta(rC + mem.col(x, 1), x + 1, y) + c.a3[0];
            b[1] = -b[1] + CT2 * tw;
        }
        if (oxp) {
            const float tw = c.a1[1] * th1 + c.a2[1] * theta(rC + mem.col(x, -1), x - 1, y) + c.a3[1];
            b[3] = -b[3] + CT2 * tw;
        }
        if (oym) {
            const float tw = c.a1[2] * th1 + c.a2[2] * theta(mem.row(y, 1) + cC, x, y + 1) + c.a3[2];
            b[2] = -b[2] + CT2 * tw;
        }
        if (oyp) {
            const float tw = c.a1[3] * th1 + c.a2[3] * theta(mem.row(y, -1) + cC, x, y - 1) + c.a3[3];
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

// Gather from the stored buffer.
template <typename S, int SRC = 0, typename O = size_t>
__device__ __forceinline__ void gather_node(const S* __restrict__ src, const LatticeConst& c, int x,
                                            int y, float a[9], float b[5])
{
    gather_mem<SRC>(global_mem<O>(src, c), c, x, y, a, b);
}

// Round the post-collision state of one node (x, y) into the storage type: the
// deviations, formed wider than the storage, go through the unbiased rounding of
// sr_round. One hash per node mixes the node's coordinates with the sum of the bits of
// all 14 results (equal results do not cancel in a sum); the k-th value takes the hash
// xor a constant key of its own (RandBits), each uniform on its own. The coordinates give
// nodes in equal states independent variates: a uniform lattice whose increments are far
// below a unit in the last place would otherwise round every node alike and could keep
// rounding to the same state. A state that no longer changes is still stored identically.
template <typename S>
__device__ __forceinline__ void round_node(const typename Wide<S>::type fa[9],
                                           const typename Wide<S>::type tb[5], S out[14], int x, int y)
{
    unsigned acc = (unsigned)x * 0x9E3779B1u + (unsigned)y * 0x632BE5ABu;
#pragma unroll
    for (int i = 0; i < 9; ++i) acc += hash_bits(fa[i]);
#pragma unroll
    for (int i = 0; i < 5; ++i) acc += hash_bits(tb[i]);
    const unsigned r = RandBits<S>::base(mix32(acc));
#pragma unroll
    for (int i = 0; i < 9; ++i) out[i] = sr_round(fa[i], r ^ RandBits<S>::key(i));
#pragma unroll
    for (int i = 0; i < 5; ++i) out[9 + i] = sr_round(tb[i], r ^ RandBits<S>::key(9 + i));
}

// Store the post-collision state of node (x, y), nontemporal; O as in GlobalMem.
template <typename S, typename O = size_t>
__device__ __forceinline__ void store_node(S* __restrict__ dst, const LatticeConst& c, int x, int y,
                                           const typename Wide<S>::type fa[9],
                                           const typename Wide<S>::type tb[5])
{
    S v[14];
    round_node<S>(fa, tb, v, x, y);
    const O own = (O)node_off(c, x, y);
#pragma unroll
    for (int i = 0; i < 14; ++i) st_nt(dst + i * kBlock + own, v[i]);
}

// Store the post-collision state of node (x, y) given the address of its population 0.
template <typename S>
__device__ __forceinline__ void store_node_at(S* __restrict__ p0, const typename Wide<S>::type fa[9],
                                              const typename Wide<S>::type tb[5], int x, int y)
{
    S v[14];
    round_node<S>(fa, tb, v, x, y);
#pragma unroll
    for (int i = 0; i < 14; ++i) st_nt(p0 + i * kBlock, v[i]);
}

// ---------------------------------------------------------------------------
// Interior nodes. Where a node and the nodes it pulls from all lie strictly inside the
// lattice, no link crosses a wall and no neighbour wraps, so the gather needs neither the
// wall substitutions nor the wrapped offsets. Its sources are then addressed as a row
// pointer (uniform across a wave when the wave works on one row) plus a per-thread byte
// offset of the column, which the loads take as scalar base + 32-bit offset + immediate.
// ---------------------------------------------------------------------------

// Byte offsets, within a row, of the columns x-1, x and x+1.
struct ColBytes {
    unsigned m, c, p;
};

// Columns of the stored layout: population 0 of x sits at (x/kBlock)*kBlockElems + x%kBlock,
// so stepping across a block boundary jumps kBlockElems - kBlock + 1 elements.
template <typename S>
__device__ __forceinline__ ColBytes stored_cols(int x)
{
    const unsigned e = (unsigned)sizeof(S);
    const unsigned xb = (unsigned)x % kBlock;
    const unsigned cc = (((unsigned)x / kBlock) * kBlockElems + xb) * e;
    const unsigned jump = (kBlockElems - kBlock + 1) * e;
    return ColBytes{xb == 0 ? cc - jump : cc - e, cc, xb == kBlock - 1 ? cc + jump : cc + e};
}

// Start of stored row y.
template <typename S>
__device__ __forceinline__ const char* stored_row(const S* p, unsigned rowlen, int y)
{
    return reinterpret_cast<const char*>(p) + (size_t)(unsigned)y * rowlen * sizeof(S);
}
template <typename S>
__device__ __forceinline__ char* stored_row(S* p, unsigned rowlen, int y)
{
    return reinterpret_cast<char*>(p) + (size_t)(unsigned)y * rowlen * sizeof(S);
}

// Pull gather (Eq. 11, Eq. 21) of an interior node from the rows y-1 (rm), y (rc), y+1 (rp)
// of the post-collision populations at time t; P is the population stride in elements.
// The values are loaded as LoadT<S> (binary16 storage keeps them in binary16).
template <typename S, unsigned P>
__device__ __forceinline__ void gather_interior(const char* rm, const char* rc, const char* rp,
                                                const ColBytes k, typename LoadT<S>::type a[9],
                                                typename LoadT<S>::type b[5])
{
    auto at = [&](const char* row, unsigned col, int i) {
        return ld_in(reinterpret_cast<const S*>(row + col) + i * P);
    };
    a[0] = at(rc, k.c, 0);
    a[1] = at(rc, k.m, 1);
    a[2] = at(rm, k.c, 2);
    a[3] = at(rc, k.p, 3);
    a[4] = at(rp, k.c, 4);
    a[5] = at(rm, k.m, 5);
    a[6] = at(rm, k.p, 6);
    a[7] = at(rp, k.p, 7);
    a[8] = at(rp, k.m, 8);
    b[0] = at(rc, k.c, 9);
    b[1] = at(rc, k.m, 10);
    b[2] = at(rm, k.c, 11);
    b[3] = at(rc, k.p, 12);
    b[4] = at(rp, k.c, 13);
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

template <typename S, int ROWS, int SRC, typename O>
__global__ void __launch_bounds__(1024) k_step(const S* __restrict__ src, S* __restrict__ dst,
                                               const LatticeConst c, int tiles_x, int tiles_total,
                                               int remap)
{
    typedef typename Wide<S>::type W;
    const int t = tile_of_block(tiles_total, remap);
    if (t >= tiles_total) return;
    const int tx = t % tiles_x, ty = t / tiles_x;
    const int x = tx * blockDim.x + threadIdx.x;
    const int y0 = (ty * blockDim.y + threadIdx.y) * ROWS;
    // A block whose nodes and their sources all lie strictly inside the lattice takes the
    // interior gather when each wave covers one row (rows are then wave-uniform).
    const int bx0 = tx * (int)blockDim.x, by0 = ty * (int)blockDim.y * ROWS;
    if (blockDim.x % 64 == 0 && bx0 >= 1 && bx0 + (int)blockDim.x < c.nx && by0 >= 1
        && by0 + (int)blockDim.y * ROWS < c.ny) {
        const ColBytes k = stored_cols<S>(x);
        const int yw = __builtin_amdgcn_readfirstlane(y0);
        const size_t rb = (size_t)c.rowlen * sizeof(S);
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const char* rc = stored_row(src, c.rowlen, yw + r);
            typename LoadT<S>::type a[9], b[5];
            W fa[9], tb[5];
            NodeMacro m;
            gather_interior<S, kBlock>(rc - rb, rc, rc + rb, k, a, b);
            collide<float, SRC, W>(c, a, b, fa, tb, m, node_q<SRC>(c, x, yw + r));
            store_node_at(reinterpret_cast<S*>(stored_row(dst, c.rowlen, yw + r) + k.c), fa, tb, x, yw + r);
        }
        return;
    }
    if (x >= c.nx) return;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int y = y0 + r;
        if (y < c.ny) {
            float a[9], b[5];
            W fa[9], tb[5];
            gather_node<S, SRC, O>(src, c, x, y, a, b);
            NodeMacro m;
            collide<float, SRC, W>(c, a, b, fa, tb, m, node_q<SRC>(c, x, y));
            store_node<S, O>(dst, c, x, y, fa, tb);
        }
    }
}

// ---------------------------------------------------------------------------
// Two time steps per launch. A workgroup owns a tile of kBlock columns by TY rows.
// Phase 1 advances the tile and a ring of one node around it from t to t+1 (pulling
// from the stored buffer) and keeps the results in LDS, rounded exactly as the stored
// state would be; phase 2 advances the tile from t+1 to t+2, pulling from LDS, and
// stores it. Both phases run the per-node code of k_step, so one launch equals two
// launches of k_step bit for bit, while each stored population is read about
// (1 + 2/kBlock)(1 + 2/TY) times and written once per two steps.
// ---------------------------------------------------------------------------

template <int TY>
struct Tile2 {
    static constexpr int XE = kBlock + 2, YE = TY + 2;  // with the halo ring
    static constexpr unsigned P = XE * YE;              // LDS population stride
};

// LDS tile [14][YE][XE] of the two-step kernel; element (0, 0) is global node (x0, y0).
template <typename S, int TY>
struct TileMem {
    typedef S Elem;
    typedef unsigned Off;
    const S* p;
    int x0, y0;
    static constexpr unsigned P = Tile2<TY>::P;
    __device__ __forceinline__ unsigned row(int y, int d) const { return (unsigned)(y + d - y0) * Tile2<TY>::XE; }
    __device__ __forceinline__ unsigned col(int x, int d) const { return (unsigned)(x + d - x0); }
};

__device__ __forceinline__ int wrap_index(int g, int n)
{
    g = g < 0 ? g + n : g;
    return g >= n ? g % n : g;
}

// True when a tile, its ring and every node the ring pulls from lie strictly inside the
// lattice: then no node of the tile or ring is a wall node and nothing wraps.
template <int TY>
__device__ __forceinline__ bool tile_interior(const LatticeConst& c, int X0, int Y0)
{
    return X0 >= 2 && X0 + (int)kBlock + 1 < c.nx && Y0 >= 2 && Y0 + TY + 1 < c.ny;
}

// Phase 1 for thread tid of the workgroup whose tile starts at (X0, Y0): node
// (X0 - 1 + lx, Y0 - 1 + ly) of the tile with its ring, advanced from the stored buffer
// into LDS. In a periodic direction a ring node outside the lattice is the wrapped
// node; in a walled one it does not exist and its LDS entry is never read.
template <typename S, int SRC, int TY, int NT, typename O>
__device__ __forceinline__ void step2_phase1(const S* __restrict__ src, const LatticeConst& c, S* tile,
                                             int X0, int Y0, int tid)
{
    typedef typename Wide<S>::type W;
    typedef Tile2<TY> T;
    const int lane = tid % 64;
    const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
    constexpr int nwaves = NT / 64;
    auto finish = [&](const auto* a, const auto* b, int gx, int gy, int lx, int ly) {
        W fa[9], tb[5];
        NodeMacro m;
        collide<float, SRC, W>(c, a, b, fa, tb, m, node_q<SRC>(c, gx, gy));
        S v[14];
        round_node<S>(fa, tb, v, gx, gy);
        const unsigned o = (unsigned)ly * T::XE + lx;
#pragma unroll
        for (int i = 0; i < 14; ++i) tile[i * T::P + o] = v[i];
    };
    auto advance = [&](int lx, int ly) {
        int gx = X0 - 1 + lx, gy = Y0 - 1 + ly;
        if (gx < 0 || gx >= c.nx) {
            if (!c.periodic_x) return;
            gx = wrap_index(gx, c.nx);
        }
        if (gy < 0 || gy >= c.ny) {
            if (!c.periodic_y) return;
            gy = wrap_index(gy, c.ny);
        }
        float a[9], b[5];
        gather_node<S, SRC, O>(src, c, gx, gy, a, b);
        finish(a, b, gx, gy, lx, ly);
    };
    // one wave per row for the kBlock interior columns, then the two ring columns
    static_assert(T::YE % nwaves == 0, "rows of the tile and ring per wave");
    if (tile_interior<TY>(c, X0, Y0)) {
        // all rows of the wave are loaded before the first is collided, so the later rows'
        // loads are in flight during the earlier rows' arithmetic
        constexpr int R = T::YE / nwaves;
        const ColBytes k = stored_cols<S>(X0 + lane);
        const size_t rb = (size_t)c.rowlen * sizeof(S);
        typename LoadT<S>::type a[R][9], b[R][5];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const char* rc = stored_row(src, c.rowlen, Y0 - 1 + wave + j * nwaves);
            gather_interior<S, kBlock>(rc - rb, rc, rc + rb, k, a[j], b[j]);
        }
#pragma unroll
        for (int j = 0; j < R; ++j)
            finish(a[j], b[j], X0 + lane, Y0 - 1 + wave + j * nwaves, lane + 1, wave + j * nwaves);
        // the two ring columns: interior nodes too, each lane with its own row
        for (int q = tid; q < 2 * T::YE; q += NT) {
            const int lx = q < T::YE ? 0 : T::XE - 1, ly = q % T::YE;
            const int gx = X0 - 1 + lx, gy = Y0 - 1 + ly;
            const char* rc = stored_row(src, c.rowlen, gy);
            typename LoadT<S>::type ra[9], rb9[5];
            gather_interior<S, kBlock>(rc - rb, rc, rc + rb, stored_cols<S>(gx), ra, rb9);
            finish(ra, rb9, gx, gy, lx, ly);
        }
    } else {
#pragma unroll
        for (int j = 0; j < T::YE / nwaves; ++j) advance(lane + 1, wave + j * nwaves);
        for (int q = tid; q < 2 * T::YE; q += NT) advance(q < T::YE ? 0 : T::XE - 1, q % T::YE);
    }
}

// Phase 2 of an interior tile with FP32 storage, two nodes per lane: lane L of a
// half-wave advances the nodes 2L and 2L + 1 of one tile row from LDS and stores each
// population of the pair as one aligned 8-byte word (half as many store instructions as
// one node per lane, 2% faster on the 4096^2 cavity; for binary16 storage the 4-byte pair
// word gave nothing).
template <int SRC, int TY, int NT>
__device__ __forceinline__ void step2_phase2_pairs(float* __restrict__ dst, const LatticeConst& c,
                                                   const float* tile, int X0, int Y0, int lane, int wave)
{
    typedef Tile2<TY> T;
    typedef float F2 __attribute__((ext_vector_type(2)));
    constexpr int nwaves = NT / 64;
    const int L = lane & 31, sub = lane >> 5;
    constexpr unsigned e = sizeof(float), rb = T::XE * sizeof(float);
    const unsigned pairb = (((unsigned)X0 / kBlock) * kBlockElems + 2u * (unsigned)L) * e;
#pragma unroll
    for (int j = 0; j < (TY + 2 * nwaves - 1) / (2 * nwaves); ++j) {
        const int ly = 2 * wave + sub + j * 2 * nwaves;
        if (ly >= TY) break;
        const char* rc = reinterpret_cast<const char*>(tile) + (unsigned)(ly + 1) * rb;
        float v[2][14];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            // LDS column of the node is its tile column + 1 (the ring is column 0)
            const unsigned cb = (unsigned)(2 * L + h + 1) * e;
            const ColBytes k{cb - e, cb, cb + e};
            float a[9], b[5];
            double fa[9], tb[5];
            NodeMacro m;
            gather_interior<float, T::P>(rc - rb, rc, rc + rb, k, a, b);
            collide<float, SRC, double>(c, a, b, fa, tb, m, node_q<SRC>(c, X0 + 2 * L + h, Y0 + ly));
            round_node<float>(fa, tb, v[h], X0 + 2 * L + h, Y0 + ly);
        }
        char* out = stored_row(dst, c.rowlen, Y0 + ly) + pairb;
#pragma unroll
        for (int i = 0; i < 14; ++i) {
            F2 w;
            w.x = v[0][i];
            w.y = v[1][i];
            __builtin_nontemporal_store(w, reinterpret_cast<F2*>(out + i * kBlock * e));
        }
    }
}

// Phase 2 for thread tid: the tile's own nodes advanced from LDS and stored.
template <typename S, int SRC, int TY, int NT, typename O>
__device__ __forceinline__ void step2_phase2(S* __restrict__ dst, const LatticeConst& c, const S* tile,
                                             int X0, int Y0, int tid)
{
    typedef typename Wide<S>::type W;
    typedef Tile2<TY> T;
    const int lane = tid % 64;
    const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
    constexpr int nwaves = NT / 64;
    const int gx = X0 + lane;
    if constexpr (sizeof(S) == 4) {
        if (tile_interior<TY>(c, X0, Y0)) {
            step2_phase2_pairs<SRC, TY, NT>(dst, c, tile, X0, Y0, lane, wave);
            return;
        }
    }
    if (tile_interior<TY>(c, X0, Y0)) {
        // LDS column of the node is lane + 1, its row ly + 1 (the ring is row and column 0)
        const unsigned e = (unsigned)sizeof(S), cb = (unsigned)(lane + 1) * e;
        const ColBytes k{cb - e, cb, cb + e};
        const unsigned own = stored_cols<S>(gx).c;
        constexpr unsigned rb = T::XE * sizeof(S);
#pragma unroll
        for (int j = 0; j < (TY + nwaves - 1) / nwaves; ++j) {
            const int ly = wave + j * nwaves;
            if (ly >= TY) break;
            const char* rc = reinterpret_cast<const char*>(tile) + (unsigned)(ly + 1) * rb;
            typename LoadT<S>::type a[9], b[5];
            W fa[9], tb[5];
            NodeMacro m;
            gather_interior<S, T::P>(rc - rb, rc, rc + rb, k, a, b);
            collide<float, SRC, W>(c, a, b, fa, tb, m, node_q<SRC>(c, gx, Y0 + ly));
            store_node_at(reinterpret_cast<S*>(stored_row(dst, c.rowlen, Y0 + ly) + own), fa, tb, gx, Y0 + ly);
        }
    } else if (gx < c.nx) {
        const TileMem<S, TY> mem{tile, X0 - 1, Y0 - 1};
#pragma unroll
        for (int j = 0; j < (TY + nwaves - 1) / nwaves; ++j) {
            const int ly = wave + j * nwaves, gy = Y0 + ly;
            if (ly >= TY || gy >= c.ny) break;
            float a[9], b[5];
            W fa[9], tb[5];
            NodeMacro m;
            gather_mem<SRC>(mem, c, gx, gy, a, b);
            collide<float, SRC, W>(c, a, b, fa, tb, m, node_q<SRC>(c, gx, gy));
            store_node<S, O>(dst, c, gx, gy, fa, tb);
        }
    }
}

template <typename S, int SRC, int TY, int NT, typename O>
__global__ void __launch_bounds__(NT) k_step2(const S* __restrict__ src, S* __restrict__ dst,
                                              const LatticeConst c, int tiles_x, int tiles_total,
                                              int remap)
{
    __shared__ S tile[14 * Tile2<TY>::P];
    // With remap, each XCD takes a contiguous run of tiles, so the ring nodes a tile
    // shares with the previous tile of its row (and of the row of tiles above) are
    // still in that XCD's L2.
    const int t = tile_of_block(tiles_total, remap);
    if (t >= tiles_total) return;
    const int X0 = (t % tiles_x) * (int)kBlock;
    const int Y0 = (t / tiles_x) * TY;
    step2_phase1<S, SRC, TY, NT, O>(src, c, tile, X0, Y0, (int)threadIdx.x);
    __syncthreads();
    step2_phase2<S, SRC, TY, NT, O>(dst, c, tile, X0, Y0, (int)threadIdx.x);
}
}  // namespace clbm
