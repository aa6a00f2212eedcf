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

// Per-lattice constants of one step, passed by value to every kernel.
struct LatticeConst {
    int nx, ny, pitch;         // pitch: elements per stored row (multiple of 64)
    unsigned plane;            // elements per population plane = ny * pitch
    int periodic_x, periodic_y;
    int moving;                // any wall with u_wall != 0
    float one_m_sp, sm;        // 1 - s_plus, s_minus  (Eq. 8 block on k20, k02)
    float one_m_snu;           // 1 - s_nu on k11
    float one_m_s3, half_s3c;  // 1 - s_3 and (1 - s_3/2)/3 (force term on k21, k12)
    float one_m_s4;            // 1 - s_4 on k22
    float one_m_l1, one_m_l2;  // thermal 1 - lambda_1, 1 - lambda_2
    float src2;                // (1 - lambda_2/2) c_T^2 Q (source on thermal k20, k02)
    float g_beta, Fx, Fy, Q, T0;
    float uw[4];               // tangential wall speeds, side order x-, x+, y-, y+
    float a1[4], a2[4], a3[4]; // theta_w = a1 theta_1 + a2 theta_2 + a3  (Eq. 28 in theta = T - T0)
};

// Storage loads: float32 or binary16.
template <typename S> __device__ __forceinline__ float ld(const S* p);
template <> __device__ __forceinline__ float ld<float>(const float* p) { return *p; }
template <> __device__ __forceinline__ float ld<__half>(const __half* p) { return __half2float(*p); }

// Unbiased rounding into storage. x lies between the nearest storable value f and its
// neighbour g on the other side of x; g is taken with probability |x - f|/|g - f|, the
// uniform variate being a hash of the bits of x. The expected stored value is x, the
// decision is a deterministic function of x (runs are reproducible, and a state that
// no longer changes is stored identically every step).
__device__ __forceinline__ unsigned mix32(unsigned h)
{
    h ^= h >> 16;
    h *= 0x7feb352du;
    h ^= h >> 15;
    h *= 0x846ca68bu;
    h ^= h >> 16;
    return h;
}

// Flow populations are computed in FP32: stored as is in FP32, and with the dithered
// rounding (hash of the FP32 bits) in binary16, whose rounding error dominates.
template <typename S> __device__ __forceinline__ void st(S* p, float v);
template <> __device__ __forceinline__ void st<float>(float* p, float v) { __builtin_nontemporal_store(v, p); }
template <> __device__ __forceinline__ void st<__half>(__half* p, float v)
{
    // Stochastic rounding in the integer domain: binary16 keeps 10 of the 23 fraction bits
    // of a value with exponent >= -14 and fewer below (its grid spacing is 2^-24 there), so
    // a hashed offset of as many bits as are dropped is added to the magnitude and those
    // bits are cleared; the conversion of the result is exact, and the magnitude rounds up
    // with probability equal to the dropped fraction. Below 2^-24 the two candidates are
    // 0 and 2^-24.
    const unsigned u = __float_as_uint(v);
    const int e = (int)((u >> 23) & 0xffu) - 127;
    const unsigned h = mix32(u);
    float w;
    if (e >= -24) {
        const int drop = 13 + (e < -14 ? -14 - e : 0);
        const unsigned mask = (1u << drop) - 1u;
        w = __uint_as_float((u + (h & mask)) & ~mask);
    } else {
        const float a = fabsf(v) * 16777216.f;
        const float r = (float)(h >> 8) * (1.f / 16777216.f);
        w = copysignf(r < a ? 5.9604644775390625e-8f : 0.f, v);
    }
    *p = __float2half_rn(w);
}

// Storage of the temperature populations: evaluated in FP64 registers for FP32 storage
// and in FP32 for binary16 storage (whose rounding, 2^-11, dominates FP32's).
template <typename S> struct Wide;
template <> struct Wide<float> { typedef double type; };
template <> struct Wide<__half> { typedef float type; };

template <typename S> __device__ __forceinline__ void st_dither(S* p, typename Wide<S>::type x);
// FP64 -> FP32: add a hashed 29-bit offset to the 52-bit mantissa and truncate the 29 bits
// FP32 does not keep; the conversion of the truncated value is then exact. The magnitude
// rounds up with probability (discarded bits)/2^29, so the expected stored value is x.
template <> __device__ __forceinline__ void st_dither<float>(float* p, double x)
{
    unsigned long long bits = (unsigned long long)__double_as_longlong(x);
    bits += (unsigned long long)(mix32((unsigned)bits) >> 3);
    bits &= ~0x1FFFFFFFull;
    __builtin_nontemporal_store((float)__longlong_as_double((long long)bits), p);
}
template <> __device__ __forceinline__ void st_dither<__half>(__half* p, float x) { st<__half>(p, x); }

struct NodeMacro {
    float drho;   // rho - 1
    float ux, uy;
    float theta;  // T - T0
};

// Cascaded collision of the temperature populations (Eq. 13-20 with the heat source
// of Eq. 23-24), evaluated in FP64 registers from the FP32 inputs. The arithmetic is
// done wider than the storage so that the only rounding left in a time step is the
// unbiased one into storage: a heat source adds the same non-representable amount
// every step, and round-to-nearest of that increment onto the storage grid would
// otherwise bias the temperature by a fixed fraction of an ulp per step.
template <typename R>
__device__ __forceinline__ void collide_thermal(const LatticeConst& c, const float b[5], float uxf,
                                                float uyf, R tb[5])
{
    const R ux = uxf, uy = uyf, Q = c.Q, T0 = c.T0;
    const R b0 = b[0], b1 = b[1], b2 = b[2], b3 = b[3], b4 = b[4];
    const R ux2 = ux * ux, uy2 = uy * uy;
    // Raw moments of b (Eq. 16); the rest weights carry [T0, 0, 0, T0 c_T^2, T0 c_T^2].
    const R sb = (b0 + b1) + (b2 + b3) + b4;
    const R theta = sb + R(0.5) * Q;               // Eq. (25), minus T0
    const R t10 = b1 - b3, t01 = b2 - b4, t20 = b1 + b3, t02 = b2 + b4;
    const R K00 = T0 + sb;                      // full raw k00 = T - Q/2
    // Central moments (Eq. 17) minus equilibria (Eq. 19).
    const R e10 = t10 - ux * K00;
    const R e01 = t01 - uy * K00;
    const R m20 = t20 - R(0.4) * theta - R(2.0) * ux * t10 + ux2 * K00;
    const R m02 = t02 - R(0.4) * theta - R(2.0) * uy * t01 + uy2 * K00;
    // Eq. (23): k00 relaxes to T + Q/2 for any lambda_0; lambda_1 on k10, k01;
    // lambda_2 on k20, k02 with the source (1 - lambda_2/2) c_T^2 Q.
    const R e10s = (R)c.one_m_l1 * e10;
    const R e01s = (R)c.one_m_l1 * e01;
    const R m20s = (R)c.one_m_l2 * m20 + (R)c.src2;
    const R m02s = (R)c.one_m_l2 * m02 + (R)c.src2;
    // Back to raw moments (shift by -u): k00* = T + Q/2 = T0 + Th.
    const R Th = theta + R(0.5) * Q;
    const R K00s = T0 + Th;
    const R q10 = e10s + ux * K00s;
    const R q01 = e01s + uy * K00s;
    const R q20 = R(0.4) * theta + m20s + R(2.0) * ux * e10s + ux2 * K00s;   // k20* - T0 c_T^2
    const R q02 = R(0.4) * theta + m02s + R(2.0) * uy * e01s + uy2 * K00s;
    // Inverse of Eq. (16).
    tb[0] = Th - q20 - q02;
    tb[1] = R(0.5) * (q20 + q10);
    tb[3] = R(0.5) * (q20 - q10);
    tb[2] = R(0.5) * (q02 + q01);
    tb[4] = R(0.5) * (q02 - q01);
}

// Cascaded collision of one node. On entry a[9], b[5] hold the pre-collision
// deviations at time t; on exit a[9] holds the post-collision flow deviations and
// tb[5] the post-collision temperature deviations (in the wide type R, to be rounded
// into storage by store_node). m receives rho - 1, u and T - T0 at time t.
template <typename R>
__device__ __forceinline__ void collide(const LatticeConst& c, float a[9], const float b[5], R tb[5],
                                        NodeMacro& m)
{
    // Eq. (25): T = sum g + Q/2; sum g = T0 + sum b.
    const float sb = (b[0] + b[1]) + (b[2] + b[3]) + b[4];
    const float theta = sb + 0.5f * c.Q;
    // Eq. (2): gravity along -y.
    const float Fx = c.Fx;
    const float Fy = c.Fy + c.g_beta * theta;

    // Raw moments of the deviations (Eq. 6a applied to a); the rest weights carry
    // [1, 0, 0, 1/3, 1/3, 0, 0, 0, 1/9].
    const float s13 = a[1] + a[3], d13 = a[1] - a[3];
    const float s24 = a[2] + a[4], d24 = a[2] - a[4];
    const float p56 = a[5] + a[6], m56 = a[5] - a[6];
    const float p78 = a[7] + a[8], m78 = a[7] - a[8];
    const float k22 = p56 + p78;                    // a5 + a6 + a7 + a8
    const float d = a[0] + s13 + s24 + k22;         // rho - 1
    const float jx = d13 + m56 - m78;               // k10
    const float jy = d24 + p56 - p78;               // k01
    const float k20 = s13 + k22;
    const float k02 = s24 + k22;
    const float k11 = m56 + m78;
    const float k21 = p56 - p78;
    const float k12 = m56 - m78;

    // Eq. (12).
    const float rho = 1.f + d;
    const float inv = 1.f / rho;
    const float ux = (jx + 0.5f * Fx) * inv;
    const float uy = (jy + 0.5f * Fy) * inv;
    const float ux2 = ux * ux, uy2 = uy * uy, uxy = ux * uy;

    // Central moments (Eq. 6b), minus their equilibria (Eq. 9).
    const float c10 = jx - ux * rho;
    const float c01 = jy - uy * rho;
    const float K20 = (1.f / 3.f) + k20;           // full raw k20
    const float K02 = (1.f / 3.f) + k02;
    const float n20 = (k20 - d * (1.f / 3.f)) - 2.f * ux * jx + ux2 * rho;
    const float n02 = (k02 - d * (1.f / 3.f)) - 2.f * uy * jy + uy2 * rho;
    const float c11 = k11 - uy * jx - ux * jy + uxy * rho;
    const float c21 = k21 - 2.f * ux * k11 - uy * K20 + 2.f * uxy * jx + ux2 * jy - ux2 * uy * rho;
    const float c12 = k12 - 2.f * uy * k11 - ux * K02 + 2.f * uxy * jy + uy2 * jx - uy2 * ux * rho;
    const float n22 = (k22 - d * (1.f / 9.f)) - 2.f * ux * k12 - 2.f * uy * k21 + 4.f * uxy * k11
                      + uy2 * K20 + ux2 * K02 - 2.f * ux * uy2 * jx - 2.f * ux2 * uy * jy
                      + ux2 * uy2 * rho;

    // Eq. (7): relaxation with the force term (I - S/2) C; rows 0-2 are not relaxed.
    const float c10s = c10 + Fx;
    const float c01s = c01 + Fy;
    const float n20s = c.one_m_sp * n20 - c.sm * n02;
    const float n02s = c.one_m_sp * n02 - c.sm * n20;
    const float c11s = c.one_m_snu * c11;
    const float c21s = c.one_m_s3 * c21 + c.half_s3c * Fy;
    const float c12s = c.one_m_s3 * c12 + c.half_s3c * Fx;
    const float n22s = c.one_m_s4 * n22;

    // Back to raw moments (shift by -u), minus the rest-weight moments.
    const float K20s = (1.f / 3.f) + d * (1.f / 3.f) + n20s;   // full central k20*
    const float K02s = (1.f / 3.f) + d * (1.f / 3.f) + n02s;
    const float r10 = c10s + ux * rho;
    const float r01 = c01s + uy * rho;
    const float r20 = d * (1.f / 3.f) + n20s + 2.f * ux * c10s + ux2 * rho;
    const float r02 = d * (1.f / 3.f) + n02s + 2.f * uy * c01s + uy2 * rho;
    const float r11 = c11s + uy * c10s + ux * c01s + uxy * rho;
    const float r21 = c21s + 2.f * ux * c11s + uy * K20s + 2.f * uxy * c10s + ux2 * c01s + ux2 * uy * rho;
    const float r12 = c12s + 2.f * uy * c11s + ux * K02s + 2.f * uxy * c01s + uy2 * c10s + uy2 * ux * rho;
    const float r22 = d * (1.f / 9.f) + n22s + 2.f * ux * c12s + 2.f * uy * c21s + 4.f * uxy * c11s
                      + uy2 * K20s + ux2 * K02s + 2.f * ux * uy2 * c10s + 2.f * ux2 * uy * c01s
                      + ux2 * uy2 * rho;

    // Inverse of Eq. (6a).
    a[0] = d - r20 - r02 + r22;
    a[1] = 0.5f * (r10 + r20 - r12 - r22);
    a[3] = 0.5f * (-r10 + r20 + r12 - r22);
    a[2] = 0.5f * (r01 + r02 - r21 - r22);
    a[4] = 0.5f * (-r01 + r02 + r21 - r22);
    a[5] = 0.25f * (r11 + r21 + r12 + r22);
    a[6] = 0.25f * (-r11 + r21 - r12 + r22);
    a[7] = 0.25f * (r11 - r21 - r12 + r22);
    a[8] = 0.25f * (-r11 - r21 + r12 + r22);

    collide_thermal(c, b, ux, uy, tb);
    m.drho = d;
    m.ux = ux;
    m.uy = uy;
    m.theta = theta;
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
// T = sum g* - Q/2 and u = (sum f* e - F/2)/rho.
__device__ __forceinline__ NodeMacro macros_from_post(const LatticeConst& c, const float a[9],
                                                      const float b[5])
{
    NodeMacro m;
    const float sb = (b[0] + b[1]) + (b[2] + b[3]) + b[4];
    m.theta = sb - 0.5f * c.Q;
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
    return m;
}

}  // namespace clbm
