// clbm_device.h -- per-node arithmetic of the thermal cascaded LBM on gfx950.
//
// Fei & Luo, arXiv:1801.04577. Populations are carried as deviations from the
// rest state: a_i = f_i - w_i (w_0 = 4/9, w_1..4 = 1/9, w_5..8 = 1/36, the rest
// equilibrium of Eq. 9 at rho = 1) and b_i = g_i - T0/5 (the rest equilibrium of
// Eq. 19 with c_T^2 = 2/5). Every moment below is written so that O(1)
// constants cancel analytically and float32 only ever adds small numbers.
//
// The collision is Eq. (7) with S of Eq. (8), Gamma~eq of Eq. (9) and C of
// Eq. (10); the thermal collision is Eq. (23) with Gamma~T,eq of Eq. (19) and R
// of Eq. (24). The raw->central shift is Eq. (6b)/(17), its inverse is the shift
// by -u, and the moment->population map is the inverse of Eq. (6a)/(16) written
// out in closed form.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

namespace clbm {

// Velocity set of Eq. (3); opposite directions 0<->0, 1<->3, 2<->4, 5<->7, 6<->8.
__host__ __device__ constexpr int ex(int i) { return (i == 1 || i == 5 || i == 8) ? 1 : (i == 3 || i == 6 || i == 7) ? -1 : 0; }
__host__ __device__ constexpr int ey(int i) { return (i == 2 || i == 5 || i == 6) ? 1 : (i == 4 || i == 7 || i == 8) ? -1 : 0; }
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : (i <= 4 ? ((i + 1) & 3) + 1 : ((i - 3) & 3) + 5); }
__host__ __device__ constexpr float wgt(int i) { return i == 0 ? 4.f / 9.f : (i <= 4 ? 1.f / 9.f : 1.f / 36.f); }

constexpr float CT2 = 0.4f;  // c_T^2 (Sec. 3)

// Storage layout of a population buffer: each row is cut into blocks of kBlock nodes,
// and a block stores its 14 populations one after the other, kBlock values each
// ([y][x / kBlock][i][x % kBlock]). A wave of 64 lanes then reads and writes 14
// contiguous 256-byte (FP32) segments instead of touching 14 planes a buffer apart.
constexpr unsigned kBlock = 64;
constexpr unsigned kBlockElems = 14 * kBlock;

// Per-lattice constants of one step, passed by value to every kernel.
struct LatticeConst {
    int nx, ny;
    unsigned rowlen;           // elements per stored row: ceil(nx / kBlock) * kBlockElems
    int periodic_x, periodic_y;
    int moving;                // any wall with u_wall != 0
    float sp, sm;              // s_plus, s_minus (Eq. 8 block on k20, k02)
    float snu;                 // s_nu on k11
    float s3, half_s3c;        // s_3 and (1 - s_3/2)/3 (force term on k21, k12)
    float s4;                  // s_4 on k22
    float l1, l2;              // thermal lambda_1, lambda_2
    float src2;                // (1 - lambda_2/2) c_T^2 Q (source on thermal k20, k02)
    float g_beta, Fx, Fy, Q, T0;
    int viscous;               // add the viscous dissipation to Q (Sec. 3.2)
    float vh_pre, vh_post;     // 9 nu s_nu^2, and the same over (1 - s_nu)^2
    float src2_q;              // (1 - lambda_2/2) c_T^2
    float uw[4];               // tangential wall speeds, side order x-, x+, y-, y+
    float a1[4], a2[4], a3[4]; // theta_w = a1 theta_1 + a2 theta_2 + a3  (Eq. 28 in theta = T - T0)
    // The same collision constants in FP64, for the FP64 collision of FP32 storage (kept
    // in scalar registers instead of being converted per node).
    double d_sp, d_sm, d_snu, d_s3, d_h3, d_s4, d_l1, d_l2;
    double d_src2, d_src2_q, d_Q, d_Fx, d_Fy, d_gb, d_T0, d_vh_pre;
    const float* qfield;       // nullptr, or a heat source per node [ny][nx] added to Q
};

// Source terms of a kernel instantiation (SRC bits): kSrcVisc adds the local viscous
// dissipation to Q (Sec. 3.2), kSrcField adds the caller's source field Q(x, y).
constexpr int kSrcVisc = 1, kSrcField = 2;

// The source field at node (x, y) when the instantiation has one, else 0.
template <int SRC>
__device__ __forceinline__ float node_q(const LatticeConst& c, int x, int y)
{
    if constexpr ((SRC & kSrcField) != 0) return c.qfield[(size_t)(unsigned)y * (unsigned)c.nx + (unsigned)x];
    else return 0.f;
}

// A collision constant in the arithmetic type R: the FP64 copy for R = double.
template <typename R> __device__ __forceinline__ R kv(float f, double d);
template <> __device__ __forceinline__ float kv<float>(float f, double) { return f; }
template <> __device__ __forceinline__ double kv<double>(float, double d) { return d; }

// 1/x in the arithmetic type: the hardware reciprocal refined by one Newton step (relative
// error far below the type's rounding for the densities of the lattice, x near 1).
__device__ __forceinline__ double recip(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float recip(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.f), r);
}

// Element offset of population 0 of node (x, y); population i is kBlock * i further.
// 64-bit: a buffer may hold more than 2^32 elements (a row holds fewer).
__device__ __forceinline__ size_t node_off(const LatticeConst& c, int x, int y)
{
    return (size_t)(unsigned)y * c.rowlen + ((unsigned)x / kBlock) * kBlockElems + ((unsigned)x % kBlock);
}

// The populations a node collides, as the fast paths load them: FP32 values, or for
// binary16 storage the binary16 values themselves (In = _Float16). Their conversion to
// FP32 is exact and is folded into the first sums the collision forms (in_add, in_sub)
// and into the final addition of the change, so no separate conversion is issued.
template <typename S> struct LoadT { typedef float type; };
template <> struct LoadT<__half> { typedef _Float16 type; };

template <typename R> __device__ __forceinline__ R in_val(float x) { return (R)x; }
template <typename R> __device__ __forceinline__ R in_val(_Float16 x) { return (R)(float)x; }
// x + y and x - y of two inputs in the arithmetic type R, rounded once (for binary16
// inputs and R = float: one mixed-precision fma, x * 1 + y, on the binary16 operands).
template <typename R> __device__ __forceinline__ R in_add(float x, float y) { return (R)x + (R)y; }
template <typename R> __device__ __forceinline__ R in_sub(float x, float y) { return (R)x - (R)y; }
template <typename R> __device__ __forceinline__ R in_add(_Float16 x, _Float16 y)
{
    return (R)(float)x + (R)(float)y;
}
template <typename R> __device__ __forceinline__ R in_sub(_Float16 x, _Float16 y)
{
    return (R)(float)x - (R)(float)y;
}
template <> __device__ __forceinline__ float in_add<float>(_Float16 x, _Float16 y)
{
    float r;
    asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel_hi:[1,0,1]" : "=v"(r) : "v"(x), "v"(y));
    return r;
}
template <> __device__ __forceinline__ float in_sub<float>(_Float16 x, _Float16 y)
{
    float r;
    asm("v_fma_mix_f32 %0, %2, -1.0, %1 op_sel_hi:[1,0,1]" : "=v"(r) : "v"(x), "v"(y));
    return r;
}
// x + y for an input x and a value y already in R.
template <typename R> __device__ __forceinline__ R in_plus(float x, R y) { return (R)x + y; }
template <typename R> __device__ __forceinline__ R in_plus(_Float16 x, R y) { return (R)(float)x + y; }
template <> __device__ __forceinline__ float in_plus<float>(_Float16 x, float y)
{
    float r;
    asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(x), "v"(y));
    return r;
}

// Storage loads: float32 or binary16.
template <typename S> __device__ __forceinline__ float ld(const S* p);
template <> __device__ __forceinline__ float ld<float>(const float* p) { return *p; }
template <> __device__ __forceinline__ float ld<__half>(const __half* p) { return __half2float(*p); }
// Loads of the fast paths, as LoadT.
template <typename S> __device__ __forceinline__ typename LoadT<S>::type ld_in(const S* p);
template <> __device__ __forceinline__ float ld_in<float>(const float* p) { return *p; }
template <> __device__ __forceinline__ _Float16 ld_in<__half>(const __half* p)
{
    return __builtin_bit_cast(_Float16, *p);
}

// Unbiased rounding into storage. x lies between the nearest storable value f and its
// neighbour g on the other side of x; g is taken with probability |x - f|/|g - f|. The
// uniform variates come from a hash of the node's coordinates and the bits of its
// results (round_node), so the expected stored value is x and the decision is a
// deterministic function of the node and its results: runs are reproducible, and a
// state that no longer changes is stored identically every step.
__device__ __forceinline__ unsigned mix32(unsigned h)
{
    h ^= h >> 16;
    h *= 0x7feb352du;
    h ^= h >> 15;
    h *= 0x846ca68bu;
    h ^= h >> 16;
    return h;
}

// Type of a post-collision value before it is rounded into the storage type S: FP64 for
// FP32 storage, FP32 for binary16 storage. The collision itself is FP32 arithmetic for
// both; it yields the change of every population, and the stored value is the incoming
// population plus its change, formed exactly in this wider type (two FP32 numbers sum
// exactly in FP64, up to exponent gaps beyond 29 bits) and then rounded once, without
// bias, into storage.
template <typename S> struct Wide;
template <> struct Wide<float> { typedef double type; };
template <> struct Wide<__half> { typedef float type; };

// Bits of a result that feed the node's hash: the low word of an FP64 value (it holds
// the 29 bits FP32 drops), all bits of an FP32 value.
__device__ __forceinline__ unsigned hash_bits(double x) { return (unsigned)__double_as_longlong(x); }
__device__ __forceinline__ unsigned hash_bits(float x) { return __float_as_uint(x); }

// Uniform variates of the unbiased rounding into S, from one 32-bit node hash h: value k
// takes base(h) ^ key(k), with distinct constant keys (each variate is uniform when h is).
// FP32 storage needs 29 random bits (the bits FP64 has and FP32 drops), taken from the
// top of h; binary16 storage takes all 32 bits (the conversion reads the top ones).
template <typename S> struct RandBits;
template <> struct RandBits<float> {
    static __device__ __forceinline__ unsigned base(unsigned h) { return h >> 3; }
    static constexpr unsigned key(int k) { return ((unsigned)k * 0x9E3779B9u) >> 3; }
};
template <> struct RandBits<__half> {
    static __device__ __forceinline__ unsigned base(unsigned h) { return h; }
    static constexpr unsigned key(int k) { return (unsigned)k * 0x9E3779B9u; }
};

// x rounded into the storage type S with the unbiased rounding; r is the value's variate.
// FP64 -> FP32: add the 29-bit r below the FP32 part of the 52-bit mantissa and truncate
// the 29 bits FP32 does not keep; the conversion of the truncated value is then exact.
// The magnitude rounds up with probability (discarded bits)/2^29.
__device__ __forceinline__ float sr_round(double x, unsigned r)
{
    unsigned long long bits = (unsigned long long)__double_as_longlong(x);
    bits += (unsigned long long)r;
    bits &= ~0x1FFFFFFFull;
    return (float)__longlong_as_double((long long)bits);
}
// FP32 -> binary16 with gfx950's stochastic-rounding conversion: the magnitude rounds up
// with probability equal to the discarded fraction of a binary16 ulp (subnormal spacing
// 2^-24 included), the random bits taken from the top of r.
__device__ __forceinline__ __half sr_round(float x, unsigned r)
{
    typedef _Float16 half2v __attribute__((ext_vector_type(2)));
    // The conversion writes the low half of its destination and keeps the high half; the
    // destination starts as the bits of x (dead after this), so it needs no cleared
    // register of its own. The high half is not used.
    const half2v v = __builtin_amdgcn_cvt_sr_f16_f32(__builtin_bit_cast(half2v, x), x, r, false);
    __half_raw raw;
    raw.data = v[0];
    return raw;
}

// Nontemporal stores of storage values.
__device__ __forceinline__ void st_nt(float* p, float v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void st_nt(__half* p, __half v)
{
    __builtin_nontemporal_store(__half_raw(v).x, reinterpret_cast<unsigned short*>(p));
}

struct NodeMacro {
    float drho;   // rho - 1
    float ux, uy;
    float theta;  // T - T0
};

// Cascaded collision of the temperature populations (Eq. 13-20 with the heat source
// of Eq. 23-24), in the wide type R. The collision changes the central moments by
// Delta k00 = Q (the zeroth moment relaxes to T + Q/2 whatever lambda_0),
// Delta k10 = -lambda_1 k10, Delta k01 = -lambda_1 k01 and
// Delta k20 = -lambda_2 (k20 - c_T^2 T) + (1 - lambda_2/2) c_T^2 Q (k02 alike); the
// change is shifted back to raw moments (inverse of Eq. 17) and to populations
// (inverse of Eq. 16) and added to the incoming populations, tb = b + Delta g.
template <typename R, typename P, typename In>
__device__ __forceinline__ void collide_thermal(const LatticeConst& c, const In b[5], R t10, R t01,
                                                R t20, R t02, R sb, R ux, R uy, R Q, R src2, P tb[5])
{
    const R T0 = kv<R>(c.T0, c.d_T0);
    // Raw moments of b (Eq. 16), formed by the caller: sb = sum b, t10 = b1 - b3,
    // t01 = b2 - b4, t20 = b1 + b3, t02 = b2 + b4; the rest weights carry
    // [T0, 0, 0, T0 c_T^2, T0 c_T^2].
    const R theta = sb + R(0.5) * Q;               // Eq. (25), minus T0
    const R K00 = T0 + sb;                          // full raw k00 = T - Q/2
    // Central moments (Eq. 17) minus their equilibria (Eq. 19).
    const R e10 = t10 - ux * K00;
    const R e01 = t01 - uy * K00;
    const R m20 = t20 - R(0.4) * theta - R(2.0) * ux * t10 + ux * ux * K00;
    const R m02 = t02 - R(0.4) * theta - R(2.0) * uy * t01 + uy * uy * K00;
    // Eq. (23): changes of the central moments.
    const R l1 = kv<R>(c.l1, c.d_l1), l2 = kv<R>(c.l2, c.d_l2);
    const R d10 = -l1 * e10;
    const R d01 = -l1 * e01;
    const R d20 = src2 - l2 * m20;
    const R d02 = src2 - l2 * m02;
    // Shift by -u (inverse of Eq. 17) with Delta k00 = Q.
    const R r10 = d10 + ux * Q;
    const R r01 = d01 + uy * Q;
    const R r20 = d20 + ux * (R(2.0) * d10 + ux * Q);
    const R r02 = d02 + uy * (R(2.0) * d01 + uy * Q);
    // Inverse of Eq. (16): the change of each population, added to the incoming one in P
    // (the factor 1/2 is exact and applied in P with the sum).
    tb[0] = in_val<P>(b[0]) + P(Q - r20 - r02);
    tb[1] = in_val<P>(b[1]) + P(0.5) * P(r20 + r10);
    tb[3] = in_val<P>(b[3]) + P(0.5) * P(r20 - r10);
    tb[2] = in_val<P>(b[2]) + P(0.5) * P(r02 + r01);
    tb[4] = in_val<P>(b[4]) + P(0.5) * P(r02 - r01);
}

// Viscous dissipation nu [(d_x u_y + d_y u_x)^2 + (d_x u_x - d_y u_y)^2] (Sec. 3.2 uses
// its channel form nu (du/dy)^2) from the non-equilibrium central second moments of the
// flow populations. To first order in the Chapman-Enskog expansion the pre-collision
// k11 = -(rho/(3 s_nu))(d_x u_y + d_y u_x) and k20 - k02 = -(2 rho/(3 s_nu))(d_x u_x - d_y u_y),
// so the dissipation is coef (k11^2 + (k20 - k02)^2/4)/rho^2 with coef = 9 nu s_nu^2.
// The post-collision moments are (1 - s_nu) times the pre-collision ones (the force term
// has no second-order central part), hence coef/(1 - s_nu)^2 on stored data.
template <typename R>
__device__ __forceinline__ R dissipation(R coef, R c11, R c2d, R rho)
{
    const R h = R(0.5) * c2d;
    const R ir = recip(rho);
    return coef * (c11 * c11 + h * h) * (ir * ir);
}

// Cascaded collision of one node. On entry a[9], b[5] hold the pre-collision
// deviations at time t (In: FP32, or binary16 as loaded, see LoadT); on exit fa[9] and tb[5] hold the post-collision flow and
// temperature deviations in the type P, to be rounded into storage by store_node.
// m receives rho - 1, u and T - T0 at time t.
// The arithmetic type R gives the change of each population; the change is added to the
// incoming population in P (FP64 for FP32 storage, exact), so that the only rounding of
// a stored value is the unbiased one into storage: a body force or a heat source adds
// the same non-representable amount every step, and round-to-nearest of the sum in
// storage precision would bias the velocity and the temperature by a fixed fraction of
// an ulp per step. The change itself may carry R's rounding: it is the sum of small
// terms (the moments are taken on deviations and the first central moments are fixed by
// the force), so its error is relative to the change, far below an ulp of the stored
// population, and on the conserved moments it does not accumulate beyond that.
// The collision is evaluated as a change: Eq. (7) changes the central moments by
// Delta = -S (k - k_eq) + (I - S/2) C, which vanishes on the conserved k00 and is the
// force on k10, k01; the change is shifted back to raw moments with N(-u) (the inverse
// of Eq. 6b) and to populations with the inverse of Eq. (6a), and added to the incoming
// populations: f* = f + M^-1 N(-u) Delta.
// SRC & kSrcVisc: the heat source is Q plus the local viscous dissipation (needs
// g_beta = 0, so that the force does not depend on the temperature the source produces).
// SRC & kSrcField: qx, the caller's source at this node, is added to Q.
template <typename R, int SRC = 0, typename P = R, typename In = float>
__device__ __forceinline__ void collide(const LatticeConst& c, const In a[9], const In b[5],
                                        P fa[9], P tb[5], NodeMacro& m, float qx = 0.f)
{
    const R third = R(1) / R(3), ninth = R(1) / R(9);
    // Raw moments of the temperature deviations (Eq. 16).
    const R t20 = in_add<R>(b[1], b[3]), t10 = in_sub<R>(b[1], b[3]);
    const R t02 = in_add<R>(b[2], b[4]), t01 = in_sub<R>(b[2], b[4]);
    // Eq. (25): T = sum g + Q/2; sum g = T0 + sum b.
    const R sb = in_plus<R>(b[0], t20) + t02;
    const float Qloc = (SRC & kSrcField) ? c.Q + qx : c.Q;
    const float theta = (float)sb + 0.5f * Qloc;
    // Eq. (2): gravity along -y.
    const R Fx = kv<R>(c.Fx, c.d_Fx);
    const R Fy = kv<R>(c.Fy, c.d_Fy) + kv<R>(c.g_beta, c.d_gb) * (R)theta;

    // Raw moments of the deviations (Eq. 6a applied to a); the rest weights carry
    // [1, 0, 0, 1/3, 1/3, 0, 0, 0, 1/9].
    const R s13 = in_add<R>(a[1], a[3]), d13 = in_sub<R>(a[1], a[3]);
    const R s24 = in_add<R>(a[2], a[4]), d24 = in_sub<R>(a[2], a[4]);
    const R p56 = in_add<R>(a[5], a[6]), m56 = in_sub<R>(a[5], a[6]);
    const R p78 = in_add<R>(a[7], a[8]), m78 = in_sub<R>(a[7], a[8]);
    const R k22 = p56 + p78;                    // a5 + a6 + a7 + a8
    const R d = in_plus<R>(a[0], s13) + s24 + k22;  // rho - 1
    const R jx = d13 + m56 - m78;               // k10
    const R jy = d24 + p56 - p78;               // k01
    const R k20 = s13 + k22;
    const R k02 = s24 + k22;
    const R k11 = m56 + m78;
    const R k21 = p56 - p78;
    const R k12 = m56 - m78;

    // Eq. (12).
    const R rho = R(1) + d;
    const R inv = recip(rho);
    const R ux = (jx + R(0.5) * Fx) * inv;
    const R uy = (jy + R(0.5) * Fy) * inv;
    const R tx = R(2) * ux, ty = R(2) * uy, ux2 = ux * ux, uy2 = uy * uy;

    // Central moments (Eq. 6b) of the relaxed orders, minus their equilibria (Eq. 9). The
    // shift N(u) factors into one-dimensional binomial shifts: along x on each row of
    // moments, h_mn = sum (e_x - u_x)^m e_y^n f, then along y on each column. The first
    // x moment is h_10 = j_x - u_x rho = -F_x/2 by Eq. (12) (and h_01 = -F_y/2 along y).
    // Terms that cancel against the equilibria are taken from the deviations first.
    const R K02 = third + k02;                  // full raw k02
    const R n20 = (k20 - d * third) - tx * jx + ux2 * rho;    // c20 - rho/3 = h20 - rho/3
    const R h20 = n20 + third * rho;
    const R h10 = R(-0.5) * Fx;
    const R h11 = k11 - ux * jy;
    const R h21 = (k21 - tx * k11) + ux2 * jy;
    const R h12 = k12 - ux * K02;
    const R h22 = ((k22 - d * ninth) - tx * k12) + ux2 * K02;  // h22 - rho/9
    const R n02 = (k02 - d * third) - ty * jy + uy2 * rho;
    const R c11 = h11 - uy * h10;
    const R c21 = h21 - uy * h20;
    const R c12 = (h12 - ty * h11) + uy2 * h10;
    const R n22 = (h22 - ty * h21) + uy2 * h20;

    // Eq. (7): changes of the central moments; on k10, k01 the change is the force.
    const R sp = kv<R>(c.sp, c.d_sp), sm = kv<R>(c.sm, c.d_sm);
    const R s3 = kv<R>(c.s3, c.d_s3), h3 = kv<R>(c.half_s3c, c.d_h3);
    const R D20 = -(sp * n20 + sm * n02);
    const R D02 = -(sp * n02 + sm * n20);
    const R D11 = -kv<R>(c.snu, c.d_snu) * c11;
    const R D21 = h3 * Fy - s3 * c21;
    const R D12 = h3 * Fx - s3 * c12;
    const R D22 = -kv<R>(c.s4, c.d_s4) * n22;

    // Shift by -u (inverse of Eq. 6b), along y on each column of changes, then along x on
    // each row; Delta k00 = 0, Delta k10 = F_x, Delta k01 = F_y.
    const R g11 = D11 + uy * Fx;
    const R g21 = D21 + uy * D20;
    const R g02 = D02 + ty * Fy;
    const R g12 = (D12 + ty * D11) + uy2 * Fx;
    const R g22 = (D22 + ty * D21) + uy2 * D20;
    const R R20 = D20 + tx * Fx;
    const R R02 = g02;
    const R R11 = g11 + ux * Fy;
    const R R21 = (g21 + tx * g11) + ux2 * Fy;
    const R R12 = g12 + ux * g02;
    const R R22 = (g22 + tx * g12) + ux2 * g02;

    // Inverse of Eq. (6a): the change of each population, added to the incoming one in P.
    const R v1 = R20 - R22, u1 = Fx - R12;
    const R v2 = R02 - R22, u2 = Fy - R21;
    const R s1 = R11 + R22, s2 = R21 + R12;
    const R t1 = R22 - R11, t2 = R21 - R12;
    // (the factors 1/2 and 1/4 are exact, so they are applied in P together with the sum)
    fa[0] = in_val<P>(a[0]) - P(v1 + R02);
    fa[1] = in_val<P>(a[1]) + P(0.5) * P(v1 + u1);
    fa[3] = in_val<P>(a[3]) + P(0.5) * P(v1 - u1);
    fa[2] = in_val<P>(a[2]) + P(0.5) * P(v2 + u2);
    fa[4] = in_val<P>(a[4]) + P(0.5) * P(v2 - u2);
    fa[5] = in_val<P>(a[5]) + P(0.25) * P(s1 + s2);
    fa[7] = in_val<P>(a[7]) + P(0.25) * P(s1 - s2);
    fa[6] = in_val<P>(a[6]) + P(0.25) * P(t1 + t2);
    fa[8] = in_val<P>(a[8]) + P(0.25) * P(t1 - t2);

    if constexpr ((SRC & kSrcVisc) != 0) {
        const R Q0 = (SRC & kSrcField) ? R(Qloc) : kv<R>(c.Q, c.d_Q);
        const R Qn = Q0 + dissipation<R>(kv<R>(c.vh_pre, c.d_vh_pre), c11, n20 - n02, rho);
        collide_thermal(c, b, t10, t01, t20, t02, sb, ux, uy, Qn, kv<R>(c.src2_q, c.d_src2_q) * Qn, tb);
        m.theta = (float)(sb + R(0.5) * Qn);
    } else if constexpr ((SRC & kSrcField) != 0) {
        collide_thermal(c, b, t10, t01, t20, t02, sb, ux, uy, R(Qloc), kv<R>(c.src2_q, c.d_src2_q) * R(Qloc),
                        tb);
        m.theta = theta;
    } else {
        collide_thermal(c, b, t10, t01, t20, t02, sb, ux, uy, kv<R>(c.Q, c.d_Q), kv<R>(c.src2, c.d_src2), tb);
        m.theta = theta;
    }
    m.drho = (float)d;
    m.ux = (float)ux;
    m.uy = (float)uy;
}

// Discrete equilibria of Eq. (9) and Eq. (19) at (rho, u, T) as deviations.
// Raw equilibrium moments factor as rho m_a(ux) m_b(uy) with m_0 = 1, m_1 = u,
// m_2 = 1/3 + u^2 (flow) and T m_a m_b with m_2 = c_T^2 + u^2 (thermal).
__device__ __forceinline__ void equilibrium(float drho, float ux, float uy, float theta, float T0,
                                            float a[9], float b[5])
{
    const float rho = 1.f + drho;
    const float ux2 = ux * ux, uy2 = uy * uy;
    const float r10 = rho * ux, r01 = rho * uy;
    const float r20 = drho * (1.f / 3.f) + rho * ux2;
    const float r02 = drho * (1.f / 3.f) + rho * uy2;
    const float r11 = rho * ux * uy;
    const float r21 = rho * ((1.f / 3.f) + ux2) * uy;
    const float r12 = rho * ((1.f / 3.f) + uy2) * ux;
    const float r22 = drho * (1.f / 9.f) + rho * ((ux2 + uy2) * (1.f / 3.f) + ux2 * uy2);
    a[0] = drho - r20 - r02 + r22;
    a[1] = 0.5f * (r10 + r20 - r12 - r22);
    a[3] = 0.5f * (-r10 + r20 + r12 - r22);
    a[2] = 0.5f * (r01 + r02 - r21 - r22);
    a[4] = 0.5f * (-r01 + r02 + r21 - r22);
    a[5] = 0.25f * (r11 + r21 + r12 + r22);
    a[6] = 0.25f * (-r11 + r21 - r12 + r22);
    a[7] = 0.25f * (r11 - r21 - r12 + r22);
    a[8] = 0.25f * (-r11 - r21 + r12 + r22);
    const float T = T0 + theta;
    const float q10 = T * ux, q01 = T * uy;
    const float q20 = CT2 * theta + T * ux2;
    const float q02 = CT2 * theta + T * uy2;
    b[0] = theta - q20 - q02;
    b[1] = 0.5f * (q20 + q10);
    b[3] = 0.5f * (q20 - q10);
    b[2] = 0.5f * (q02 + q01);
    b[4] = 0.5f * (q02 - q01);
}

// Macroscopic values at time t from the stored post-collision deviations at t:
// collision conserves rho, adds F to the momentum and Q to sum g, so
// T = sum g* - Q/2 and u = (sum f* e - F/2)/rho. With a source field, qx (the node's
// value) is part of Q; with viscous heating the dissipation part of the node's Q is
// recovered from the post-collision central moments at that u.
template <int SRC = 0>
__device__ __forceinline__ NodeMacro macros_from_post(const LatticeConst& c, const float a[9],
                                                      const float b[5], float qx = 0.f)
{
    NodeMacro m;
    const float sb = (b[0] + b[1]) + (b[2] + b[3]) + b[4];
    m.theta = sb - 0.5f * ((SRC & kSrcField) ? c.Q + qx : c.Q);
    const float Fx = c.Fx;
    const float Fy = c.Fy + c.g_beta * m.theta;
    const float p56 = a[5] + a[6], m56 = a[5] - a[6];
    const float p78 = a[7] + a[8], m78 = a[7] - a[8];
    const float d = a[0] + (a[1] + a[3]) + (a[2] + a[4]) + (p56 + p78);
    const float jx = (a[1] - a[3]) + m56 - m78;
    const float jy = (a[2] - a[4]) + p56 - p78;
    const float inv = 1.f / (1.f + d);
    m.drho = d;
    m.ux = (jx - 0.5f * Fx) * inv;
    m.uy = (jy - 0.5f * Fy) * inv;
    if constexpr ((SRC & kSrcVisc) != 0) {
        // Central k11 and k20 - k02 of the post-collision deviations (the rest weights
        // contribute to neither).
        const float rho = 1.f + d;
        const float k11 = m56 + m78;
        const float k2d = (a[1] + a[3]) - (a[2] + a[4]);
        const float c11 = k11 - m.uy * jx - m.ux * jy + m.ux * m.uy * rho;
        const float c2d = k2d - 2.f * m.ux * jx + 2.f * m.uy * jy + (m.ux * m.ux - m.uy * m.uy) * rho;
        m.theta -= 0.5f * dissipation<float>(c.vh_post, c11, c2d, rho);
    }
    return m;
}

}  // namespace clbm

namespace clbm {

// The source terms of a lattice as kernels see them at run time (the per-node kernels
// outside the time step dispatch on it).
__device__ __forceinline__ int runtime_src(const LatticeConst& c)
{
    return (c.viscous ? kSrcVisc : 0) | (c.qfield ? kSrcField : 0);
}

// macros_from_post with the source terms decided at run time, for node (x, y).
__device__ __forceinline__ NodeMacro macros_any(const LatticeConst& c, const float a[9], const float b[5],
                                                int x, int y)
{
    switch (runtime_src(c)) {
        case kSrcVisc: return macros_from_post<kSrcVisc>(c, a, b);
        case kSrcField: return macros_from_post<kSrcField>(c, a, b, node_q<kSrcField>(c, x, y));
        case kSrcVisc | kSrcField:
            return macros_from_post<kSrcVisc | kSrcField>(c, a, b, node_q<kSrcField>(c, x, y));
        default: return macros_from_post<0>(c, a, b);
    }
}

// collide with the source terms decided at run time, for node (x, y).
template <typename P>
__device__ __forceinline__ void collide_any(const LatticeConst& c, const float a[9], const float b[5], P fa[9],
                                            P tb[5], NodeMacro& m, int x, int y)
{
    switch (runtime_src(c)) {
        case kSrcVisc: collide<float, kSrcVisc, P>(c, a, b, fa, tb, m); break;
        case kSrcField: collide<float, kSrcField, P>(c, a, b, fa, tb, m, node_q<kSrcField>(c, x, y)); break;
        case kSrcVisc | kSrcField:
            collide<float, kSrcVisc | kSrcField, P>(c, a, b, fa, tb, m, node_q<kSrcField>(c, x, y));
            break;
        default: collide<float, 0, P>(c, a, b, fa, tb, m); break;
    }
}

}  // namespace clbm
