// clbm_net.hip -- the warm-start network on gfx950: a four-level convolutional
// encoder-decoder with skip connections, trained and run by the library's own
// kernels. 3x3 convolutions are implicit GEMMs on BF16 MFMA
// (v_mfma_f32_16x16x32_bf16) with FP32 accumulation; activations and activation
// gradients are BF16 in NHWC layout, master weights, weight gradients and the Adam
// state are FP32.
//
// Layer order (15 convolutions, widths w1..w4, input planes cin, output fields cout):
//   0: cin->w1   1: w1->w1 (= s1)                       at H x W
//   2: w1->w2    3: w2->w2 (= s2)      after avg-pool   at H/2
//   4: w2->w3    5: w3->w3 (= s3)      after avg-pool   at H/4
//   6: w3->w4    7: w4->w4             after avg-pool   at H/8
//   8: (w4+w3)->w3  9: w3->w3   on concat[up(h), s3]    at H/4
//  10: (w3+w2)->w2 11: w2->w2   on concat[up(h), s2]    at H/2
//  12: (w2+w1)->w1 13: w1->w1   on concat[up(h), s1]    at H
//  14: w1->cout (no activation)
// Every convolution but the last is followed by ReLU. The concatenations are free:
// the skip tensor is written straight into the upper channel range of the buffer the
// decoder reads. The canonical parameter vector stores, per layer in this order,
// W[cout][cin][3][3] then b[cout] (FP32).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <initializer_list>
#include <new>
#include <vector>

#include "clbm_host.h"

namespace clbm {

typedef __bf16 bf16;
typedef bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kLayers = 15;
constexpr int kKChunk = 32;  // K per MFMA (one 3x3 tap, 32 input channels)

__device__ __forceinline__ float bf2f(bf16 v) { return (float)v; }
__device__ __forceinline__ bf16 f2bf(float v) { return (bf16)v; }

// ---------------------------------------------------------------------------
// Implicit-GEMM 3x3 convolution (zero padding 1), one output pixel row of the GEMM
// per image pixel: M = B*H*W pixels, N = output channels, K = 9 taps x Cin.
// A workgroup of 4 waves covers 64 pixels x (16*NB) channels; each wave 16 pixels.
// MFMA 16x16x32 operand layout: lane l holds row (l % 16) of A and column (l % 16)
// of B, elements k = 8*(l/16) .. 8*(l/16)+7; the result holds column (l % 16),
// rows 4*(l/16) .. 4*(l/16)+3.
// mode 0: y = bf16(relu(acc + bias)); mode 1: y = bf16(acc) (input gradients);
// mode 2: fp32 NCHW output yf = acc + bias (network output, n < N only).
// ---------------------------------------------------------------------------
template <int NB, int MP>
__global__ void __launch_bounds__(256) k_conv(const bf16* __restrict__ x, int xC, int xoff, int Cin,
                                              const bf16* __restrict__ w,
                                              const float* __restrict__ bias, int N, int H, int W,
                                              int mode, bf16* __restrict__ y, int yC, int yoff,
                                              float* __restrict__ yf)
{
    // A wave owns MP blocks of 16 pixels and NB blocks of 16 output channels: per tap and
    // 32-channel chunk it loads MP activation and NB weight fragments and issues MP x NB
    // MFMAs, each fragment reused NB (or MP) times from registers.
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int HW = H * W;
    const int p0 = (blockIdx.x * 4 + wave) * 16 * MP;
    const int n0 = blockIdx.y * (16 * NB);
    const int kq = (lane >> 4) * 8;
    int pb[MP], py[MP], px[MP];
#pragma unroll
    for (int j = 0; j < MP; ++j) {
        const int pa = p0 + 16 * j + (lane & 15);
        pb[j] = pa / HW;
        const int rem = pa - pb[j] * HW;
        py[j] = rem / W;
        px[j] = rem - py[j] * W;
    }
    f32x4 acc[MP][NB];
#pragma unroll
    for (int j = 0; j < MP; ++j)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[j][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16x8 zero = {};
    for (int tap = 0; tap < 9; ++tap) {
        const bf16* xs[MP];
        bool in[MP];
#pragma unroll
        for (int j = 0; j < MP; ++j) {
            const int sy = py[j] + tap / 3 - 1, sx = px[j] + tap % 3 - 1;
            in[j] = sy >= 0 && sy < H && sx >= 0 && sx < W;
            // clamped source so the address is valid even where the value is not used
            const int cy = min(max(sy, 0), H - 1), cx = min(max(sx, 0), W - 1);
            xs[j] = x + (size_t)(pb[j] * HW + cy * W + cx) * xC + xoff + kq;
        }
        for (int c0 = 0; c0 < Cin; c0 += kKChunk) {
            bf16x8 a[MP];
#pragma unroll
            for (int j = 0; j < MP; ++j) {
                a[j] = *reinterpret_cast<const bf16x8*>(xs[j] + c0);
                if (!in[j]) a[j] = zero;
            }
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int n = n0 + 16 * nb + (lane & 15);
                const bf16x8 bw =
                    *reinterpret_cast<const bf16x8*>(w + ((size_t)n * 9 + tap) * Cin + c0 + kq);
#pragma unroll
                for (int j = 0; j < MP; ++j)
                    acc[j][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[j], bw, acc[j][nb], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < MP; ++j)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int n = n0 + 16 * nb + (lane & 15);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int p = p0 + 16 * j + 4 * (lane >> 4) + v;
            float r = acc[j][nb][v];
            if (mode == 2) {
                if (n < N) {
                    const int bb = p / HW, rr = p - bb * HW;
                    yf[((size_t)bb * N + n) * HW + rr] = r + bias[n];
                }
            } else if (n < N) {
                if (mode == 0) r = fmaxf(r + bias[n], 0.f);
                y[(size_t)p * yC + yoff + n] = f2bf(r);
            }
        }
    }
}

// The same convolution with both operands staged in LDS. A workgroup owns a block of
// BH x BW pixels of one image (BH = 256 / BW; wave w owns pixels 64 w .. 64 w + 63 of the
// block in row-major order, as four MFMA blocks of 16) and 16 NB output channels. Per
// chunk of 32 input channels it stages the block with its one-pixel halo and the weights
// of the nine taps in LDS, pixel-major (resp. channel-major) with the 32 channels of the
// chunk contiguous, so each tap reads both operands from LDS at compile-time offsets:
// an activation is fetched from memory once per chunk instead of once per tap, and a
// weight once per workgroup instead of once per wave.
constexpr int kCvLd = 32;   // LDS row: the 32 channels of a chunk

template <int NB, int BW>
__global__ void __launch_bounds__(256) k_conv_lds(const bf16* __restrict__ x, int xC, int xoff, int Cin,
                                                  const bf16* __restrict__ w,
                                                  const float* __restrict__ bias, int N, int H, int W,
                                                  int mode, bf16* __restrict__ y, int yC, int yoff,
                                                  float* __restrict__ yf)
{
    constexpr int BH = 256 / BW, HX = BW + 2, HY = BH + 2, NPIX = HX * HY, NC = 16 * NB;
    __shared__ __attribute__((aligned(16))) bf16 sa[NPIX * kCvLd];
    __shared__ __attribute__((aligned(16))) bf16 sw[9 * NC * kCvLd];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int bx_n = W / BW, by_n = H / BH;
    const int bxi = blockIdx.x % bx_n, byi = (blockIdx.x / bx_n) % by_n, bimg = blockIdx.x / (bx_n * by_n);
    const int x0 = bxi * BW, y0 = byi * BH;
    const int n0 = blockIdx.y * NC;
    const int r16 = lane & 15, k8 = (lane >> 4) * 8;
    // LDS element of the A row of each of the wave's four pixel blocks at tap 0 (the
    // top-left neighbour); tap t adds ((t / 3) HX + t % 3) rows
    int abase[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int q = wave * 64 + 16 * j + r16;
        abase[j] = ((q / BW) * HX + (q % BW)) * kCvLd + k8;
    }
    f32x4 acc[4][NB];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[j][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16x8 zero = {};
    // The next chunk's operands are loaded into registers while the current one is
    // multiplied from LDS.
    constexpr int NA = (NPIX * 4 + 255) / 256, NWT = (9 * NC * 4 + 255) / 256;
    bf16x8 ra[NA], rw[NWT];
    auto load_chunk = [&](int c0) {
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int t = tid + 256 * i;
            ra[i] = zero;
            if (t < NPIX * 4) {
                const int px = t >> 2, oct = t & 3;
                const int hy = px / HX, hx = px - hy * HX;
                const int sy = y0 + hy - 1, sx = x0 + hx - 1;
                if (sy >= 0 && sy < H && sx >= 0 && sx < W)
                    ra[i] = *reinterpret_cast<const bf16x8*>(x + ((size_t)(bimg * H + sy) * W + sx) * xC + xoff + c0 + 8 * oct);
            }
        }
#pragma unroll
        for (int i = 0; i < NWT; ++i) {
            const int t = tid + 256 * i;
            if (t < 9 * NC * 4) {
                const int oct = t & 3, rest = t >> 2;   // rest = tap * NC + channel
                const int tap = rest / NC, nn = rest - tap * NC;
                rw[i] = *reinterpret_cast<const bf16x8*>(w + ((size_t)(n0 + nn) * 9 + tap) * Cin + c0 + 8 * oct);
            }
        }
    };
    load_chunk(0);
    for (int c0 = 0; c0 < Cin; c0 += kKChunk) {
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int t = tid + 256 * i;
            if (t < NPIX * 4) *reinterpret_cast<bf16x8*>(&sa[(t >> 2) * kCvLd + 8 * (t & 3)]) = ra[i];
        }
#pragma unroll
        for (int i = 0; i < NWT; ++i) {
            const int t = tid + 256 * i;
            if (t < 9 * NC * 4) *reinterpret_cast<bf16x8*>(&sw[(t >> 2) * kCvLd + 8 * (t & 3)]) = rw[i];
        }
        __syncthreads();
        if (c0 + kKChunk < Cin) load_chunk(c0 + kKChunk);
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int off = ((tap / 3) * HX + tap % 3) * kCvLd;
            bf16x8 a[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) a[j] = *reinterpret_cast<const bf16x8*>(&sa[abase[j] + off]);
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const bf16x8 bw = *reinterpret_cast<const bf16x8*>(&sw[(tap * NC + 16 * nb + r16) * kCvLd + k8]);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[j][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[j], bw, acc[j][nb], 0, 0, 0);
            }
        }
        __syncthreads();  // the next chunk overwrites the tiles
    }
    const int HW = H * W;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int n = n0 + 16 * nb + r16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int q = wave * 64 + 16 * j + 4 * (lane >> 4) + v;
            const int p = (bimg * H + y0 + q / BW) * W + x0 + q % BW;
            float r = acc[j][nb][v];
            if (mode == 2) {
                if (n < N) {
                    const int bb = p / HW, rr = p - bb * HW;
                    yf[((size_t)bb * N + n) * HW + rr] = r + bias[n];
                }
            } else if (n < N) {
                if (mode == 0) r = fmaxf(r + bias[n], 0.f);
                y[(size_t)p * yC + yoff + n] = f2bf(r);
            }
        }
    }
}

// Weight gradient of one 3x3 convolution over a range of pixels (split-K):
// part[s][co][tap][ci] = sum over the pixels p of split s of dz[p][co] * x[src(p,tap)][ci],
// a GEMM whose reduction runs over pixels, the slow index of NHWC. A workgroup of three
// waves owns a (16 NCO) co x (16 NCI) ci block and one split; wave w takes the three
// taps of kernel row w. Per chunk of 32 pixels the workgroup stages dz and the nine
// shifted input tiles in LDS channel-major (the 32 pixels of one channel contiguous, two
// pixels per 32-bit write), so every MFMA operand - 8 consecutive pixels of one channel -
// is one 16-byte LDS read: A = dz^T (co x pixels), B = shifted x (pixels x ci). Each wave
// reads its NCO dz fragments once per chunk and issues 3 NCO NCI MFMAs. NCO and NCI
// divide the padded channel counts (16-channel blocks), so the block has no padding.
constexpr int kWgP = 32;          // pixels per chunk: the MFMA K
constexpr int kWgLd = kWgP + 8;   // LDS row stride in elements (staggers the banks)
constexpr int kWgThreads = 192;

__device__ __forceinline__ unsigned bf16_bits(bf16 v) { return (unsigned)__builtin_bit_cast(unsigned short, v); }

template <int NCO, int NCI>
__global__ void __launch_bounds__(kWgThreads) k_wgrad(const bf16* __restrict__ dz, int zC, int Cout,
                                                      const bf16* __restrict__ x, int xC, int xoff, int Cin,
                                                      int H, int W, int P, int pix_per_split,
                                                      float* __restrict__ part, float* __restrict__ bpart)
{
    constexpr int CO = 16 * NCO, CI = 16 * NCI;
    __shared__ __attribute__((aligned(16))) bf16 sdz[CO * kWgLd];
    __shared__ __attribute__((aligned(16))) bf16 sx[9][CI * kWgLd];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int cib_n = Cin / CI;
    const int co0 = (blockIdx.x / cib_n) * CO, ci0 = (blockIdx.x % cib_n) * CI;
    const int split = blockIdx.y;
    const int HW = H * W;
    const int pbeg = split * pix_per_split, pend = min(P, pbeg + pix_per_split);
    const int r16 = lane & 15, k8 = (lane >> 4) * 8;
    // The workgroups of the first input-channel block also sum dz over their pixels: the
    // bias gradient's partial for this split (bpart[split][co]), from the staged dz.
    const bool bias = bpart != nullptr && blockIdx.x % cib_n == 0;
    float bsum = 0.f;
    f32x4 acc[3][NCO][NCI];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int i = 0; i < NCO; ++i)
#pragma unroll
            for (int j = 0; j < NCI; ++j) acc[d][i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16x8 zero = {};
    // image, row and column of the chunk's first pixel, advanced with the chunk (no
    // division per staged pixel)
    int cb = pbeg / HW, cy = (pbeg - cb * HW) / W, cx = pbeg - cb * HW - cy * W;
    for (int pk = pbeg; pk < pend; pk += kWgP) {
        // stage dz: 16 pixel pairs x (2 NCO) channel octets
        for (int t = tid; t < 16 * 2 * NCO; t += kWgThreads) {
            const int pair = t / (2 * NCO), oct = t % (2 * NCO);
            const int p = pk + 2 * pair, co = co0 + 8 * oct;
            bf16x8 v0 = zero, v1 = zero;
            if (p < pend) v0 = *reinterpret_cast<const bf16x8*>(dz + (size_t)p * zC + co);
            if (p + 1 < pend) v1 = *reinterpret_cast<const bf16x8*>(dz + (size_t)(p + 1) * zC + co);
#pragma unroll
            for (int c = 0; c < 8; ++c)
                *reinterpret_cast<unsigned*>(&sdz[(8 * oct + c) * kWgLd + 2 * pair]) =
                    bf16_bits(v0[c]) | (bf16_bits(v1[c]) << 16);
        }
        // stage the nine shifted input tiles: 9 taps x 16 pixel pairs x (2 NCI) channel octets
#pragma unroll 2
        for (int t = tid; t < 9 * 16 * 2 * NCI; t += kWgThreads) {
            const int tap = t / (32 * NCI), rest = t % (32 * NCI);
            const int pair = rest / (2 * NCI), oct = rest % (2 * NCI);
            const int ci = ci0 + 8 * oct;
            bf16x8 v[2] = {zero, zero};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int p = pk + 2 * pair + h;
                if (p < pend) {
                    int b = cb, py = cy, px = cx + 2 * pair + h;
                    while (px >= W) {
                        px -= W;
                        if (++py == H) {
                            py = 0;
                            ++b;
                        }
                    }
                    const int sy = py + tap / 3 - 1, sx2 = px + tap % 3 - 1;
                    if (sy >= 0 && sy < H && sx2 >= 0 && sx2 < W)
                        v[h] = *reinterpret_cast<const bf16x8*>(x + (size_t)(b * HW + sy * W + sx2) * xC + xoff + ci);
                }
            }
#pragma unroll
            for (int c = 0; c < 8; ++c)
                *reinterpret_cast<unsigned*>(&sx[tap][(8 * oct + c) * kWgLd + 2 * pair]) =
                    bf16_bits(v[0][c]) | (bf16_bits(v[1][c]) << 16);
        }
        __syncthreads();
        if (bias && tid < CO) {
#pragma unroll 8
            for (int q = 0; q < kWgP; ++q) bsum += bf2f(sdz[tid * kWgLd + q]);
        }
        bf16x8 a[NCO];
#pragma unroll
        for (int i = 0; i < NCO; ++i) a[i] = *reinterpret_cast<const bf16x8*>(&sdz[(16 * i + r16) * kWgLd + k8]);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const bf16* xt = sx[3 * wave + d];
#pragma unroll
            for (int j = 0; j < NCI; ++j) {
                const bf16x8 bv = *reinterpret_cast<const bf16x8*>(&xt[(16 * j + r16) * kWgLd + k8]);
#pragma unroll
                for (int i = 0; i < NCO; ++i)
                    acc[d][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bv, acc[d][i][j], 0, 0, 0);
            }
        }
        __syncthreads();  // the next chunk overwrites the tiles
        cx += kWgP;
        while (cx >= W) {
            cx -= W;
            if (++cy == H) {
                cy = 0;
                ++cb;
            }
        }
    }
    // row of the result = output channel co0 + 16 i + 4 (lane / 16) + v, column = ci
    float* out = part + (size_t)split * Cout * 9 * Cin + (size_t)(co0 + 4 * (lane >> 4)) * 9 * Cin + ci0 + r16;
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int i = 0; i < NCO; ++i)
#pragma unroll
            for (int j = 0; j < NCI; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    out[((size_t)(16 * i + v) * 9 + 3 * wave + d) * Cin + 16 * j] = acc[d][i][j][v];
    if (bias && tid < CO) bpart[(size_t)split * Cout + co0 + tid] = bsum;
}

// Largest 16-channel block count in {4, 2, 1} that divides n16 (channels / 16).
inline int wgrad_blocks16(int n16) { return n16 % 4 == 0 ? 4 : (n16 % 2 == 0 ? 2 : 1); }

// Pixels per split of the weight gradient of a layer with P pixels and the given padded
// channel counts: about 512 workgroups (two per CU), at most 256 splits, at least 8
// chunks each.
inline int wgrad_pixels_per_split(size_t P, int cout16, int cin_pad)
{
    const size_t blocks = (size_t)(cout16 / (16 * wgrad_blocks16(cout16 / 16))) *
                          (cin_pad / (16 * wgrad_blocks16(cin_pad / 16)));
    size_t splits = std::min<size_t>(256, std::max<size_t>(1, 512 / blocks));
    splits = std::min(splits, std::max<size_t>(1, P / (8 * kWgP)));
    const size_t pps = (P + splits - 1) / splits;
    return (int)((pps + kWgP - 1) / kWgP * kWgP);
}

// Sum of the split partials in split order, written in the canonical layout
// grad[co][ci][ky][kx] for co < Cout_real, ci < Cin_real (the partials use the padded
// strides Cout, Cin). Threads run along the partials' own layout [co][tap][ci], so
// the reads of each split are contiguous across a wave.
__global__ void k_wgrad_reduce(const float* __restrict__ part, int splits, int Cout, int Cin,
                               int Cout_real, int Cin_real, float* __restrict__ grad)
{
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t plane = (size_t)Cout * 9 * Cin;
    if (k >= plane) return;
    const int co = (int)(k / (9 * (size_t)Cin)), r = (int)(k - (size_t)co * 9 * Cin);
    const int tap = r / Cin, ci = r - tap * Cin;
    if (co >= Cout_real || ci >= Cin_real) return;
    float s = 0.f;
#pragma unroll 8
    for (int sp = 0; sp < splits; ++sp) s += part[sp * plane + k];
    grad[((size_t)co * Cin_real + ci) * 9 + tap] = s;
}

// Sum of the bias partials of channel blockIdx.x: each thread sums a fixed strided
// subset of the splits, then a fixed-order tree over the 256 threads.
__global__ void __launch_bounds__(256) k_bias_reduce(const float* __restrict__ part, int splits, int C,
                                                     float* __restrict__ g)
{
    __shared__ float lds[256];
    const int c = blockIdx.x, t = threadIdx.x;
    float s = 0.f;
    for (int sp = t; sp < splits; sp += 256) s += part[(size_t)sp * C + c];
    lds[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) lds[t] += lds[t + w];
        __syncthreads();
    }
    if (t == 0) g[c] = lds[0];
}

// Canonical FP32 weights -> BF16 forward layout wf[n][tap][ci] (n < Npad, ci < CinPad,
// zeros outside the real sizes) and the input-gradient layout wb[ci][tap'][co] with
// tap' = 8 - tap (the transposed, flipped kernel).
__global__ void k_weight_prep(const float* __restrict__ Wc, int Cout, int Cin, int NoutPad,
                              int CinPad, int CoutKPad, bf16* __restrict__ wf, bf16* __restrict__ wb)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int nf = NoutPad * 9 * CinPad;
    if (k < nf) {
        const int n = k / (9 * CinPad), r = k - n * 9 * CinPad;
        const int tap = r / CinPad, ci = r - tap * CinPad;
        const float v = (n < Cout && ci < Cin) ? Wc[((size_t)n * Cin + ci) * 9 + tap] : 0.f;
        wf[k] = f2bf(v);
    }
    if (wb) {
        const int nb = CinPad * 9 * CoutKPad;
        if (k < nb) {
            const int ci = k / (9 * CoutKPad), r = k - ci * 9 * CoutKPad;
            const int tp = r / CoutKPad, co = r - tp * CoutKPad;
            const int tap = 8 - tp;
            const float v = (co < Cout && ci < Cin) ? Wc[((size_t)co * Cin + ci) * 9 + tap] : 0.f;
            wb[k] = f2bf(v);
        }
    }
}

// fp32 NCHW input planes -> bf16 NHWC with zero channel padding.
__global__ void k_pack_input(const float* __restrict__ xin, int Cin, int HW, int P,
                             bf16* __restrict__ x, int xC)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P * xC) return;
    const int p = k / xC, c = k - p * xC;
    const int b = p / HW, r = p - b * HW;
    x[k] = f2bf(c < Cin ? xin[((size_t)b * Cin + c) * HW + r] : 0.f);
}

// Elementwise kernels over NHWC channel views. Each thread handles V consecutive
// channels of one pixel: V = 8 (one 16-byte access) where the channel counts, strides
// and offsets are multiples of 8, else V = 1. The arithmetic per channel is the same.
template <int V>
__device__ __forceinline__ void load_v(const bf16* p, float (&out)[V])
{
    if constexpr (V == 8) {
        const bf16x8 t = *reinterpret_cast<const bf16x8*>(p);
#pragma unroll
        for (int i = 0; i < 8; ++i) out[i] = bf2f(t[i]);
    } else {
        out[0] = bf2f(p[0]);
    }
}

template <int V>
__device__ __forceinline__ void store_v(bf16* p, const float (&in)[V])
{
    if constexpr (V == 8) {
        bf16x8 t;
#pragma unroll
        for (int i = 0; i < 8; ++i) t[i] = f2bf(in[i]);
        *reinterpret_cast<bf16x8*>(p) = t;
    } else {
        p[0] = f2bf(in[0]);
    }
}

// 2x2 average pooling and nearest 2x upsampling on channel views.
template <int V>
__global__ void k_avgpool(const bf16* __restrict__ x, int xC, int xoff, int C, int H, int W,
                          int B, bf16* __restrict__ y, int yC, int yoff)
{
    const int Ho = H / 2, Wo = W / 2, CV = C / V;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= B * Ho * Wo * CV) return;
    const int c = (k % CV) * V, p = k / CV;
    const int b = p / (Ho * Wo), r = p - b * Ho * Wo, oy = r / Wo, ox = r - oy * Wo;
    const size_t base = (size_t)b * H * W;
    float v00[V], v01[V], v10[V], v11[V], out[V];
    load_v<V>(x + (base + (2 * oy) * W + 2 * ox) * xC + xoff + c, v00);
    load_v<V>(x + (base + (2 * oy) * W + 2 * ox + 1) * xC + xoff + c, v01);
    load_v<V>(x + (base + (2 * oy + 1) * W + 2 * ox) * xC + xoff + c, v10);
    load_v<V>(x + (base + (2 * oy + 1) * W + 2 * ox + 1) * xC + xoff + c, v11);
#pragma unroll
    for (int i = 0; i < V; ++i) out[i] = 0.25f * (v00[i] + v01[i] + v10[i] + v11[i]);
    store_v<V>(y + (size_t)p * yC + yoff + c, out);
}

template <int V>
__global__ void k_upsample(const bf16* __restrict__ x, int xC, int xoff, int C, int H, int W, int B,
                           bf16* __restrict__ y, int yC, int yoff)
{
    // x is H x W, y is 2H x 2W
    const int Ho = 2 * H, Wo = 2 * W, CV = C / V;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= B * Ho * Wo * CV) return;
    const int c = (k % CV) * V, p = k / CV;
    const int b = p / (Ho * Wo), r = p - b * Ho * Wo, oy = r / Wo, ox = r - oy * Wo;
    const bf16* src = x + ((size_t)b * H * W + (oy / 2) * W + ox / 2) * xC + xoff + c;
    bf16* dst = y + (size_t)p * yC + yoff + c;
    if constexpr (V == 8) *reinterpret_cast<bf16x8*>(dst) = *reinterpret_cast<const bf16x8*>(src);
    else dst[0] = src[0];
}

// Gradient of the nearest upsampling: 2x2 sums (dy is 2H x 2W, dx is H x W).
template <int V>
__global__ void k_upsample_bwd(const bf16* __restrict__ dy, int dyC, int dyoff, int C, int H, int W,
                               int B, bf16* __restrict__ dx, int dxC, int dxoff)
{
    const int Wi = 2 * W, CV = C / V;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= B * H * W * CV) return;
    const int c = (k % CV) * V, p = k / CV;
    const int b = p / (H * W), r = p - b * H * W, oy = r / W, ox = r - oy * W;
    const size_t base = (size_t)b * 4 * H * W;
    float v00[V], v01[V], v10[V], v11[V], out[V];
    load_v<V>(dy + (base + (2 * oy) * Wi + 2 * ox) * dyC + dyoff + c, v00);
    load_v<V>(dy + (base + (2 * oy) * Wi + 2 * ox + 1) * dyC + dyoff + c, v01);
    load_v<V>(dy + (base + (2 * oy + 1) * Wi + 2 * ox) * dyC + dyoff + c, v10);
    load_v<V>(dy + (base + (2 * oy + 1) * Wi + 2 * ox + 1) * dyC + dyoff + c, v11);
#pragma unroll
    for (int i = 0; i < V; ++i) out[i] = v00[i] + v01[i] + v10[i] + v11[i];
    store_v<V>(dx + (size_t)p * dxC + dxoff + c, out);
}

// dz = (dskip + pool_backward(dpool)) * (a > 0), all at H x W; dpool is H/2 x W/2.
// With dskip == nullptr and dpool == nullptr it is the plain ReLU gradient dz = dy * (a > 0)
// where dy is passed as dskip.
template <int V>
__global__ void k_relu_grad(const bf16* __restrict__ dskip, int sC, int soff,
                            const bf16* __restrict__ dpool, int pC, const bf16* __restrict__ a,
                            int aC, int aoff, int C, int H, int W, int B, bf16* __restrict__ dz,
                            int zC)
{
    const int CV = C / V;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= B * H * W * CV) return;
    const int c = (k % CV) * V, p = k / CV;
    float g[V], av[V], out[V];
#pragma unroll
    for (int i = 0; i < V; ++i) g[i] = 0.f;
    if (dskip) load_v<V>(dskip + (size_t)p * sC + soff + c, g);
    if (dpool) {
        const int b = p / (H * W), r = p - b * H * W, py = r / W, px = r - py * W;
        const int Wo = W / 2;
        float d[V];
        load_v<V>(dpool + ((size_t)b * (H / 2) * Wo + (py / 2) * Wo + px / 2) * pC + c, d);
#pragma unroll
        for (int i = 0; i < V; ++i) g[i] += 0.25f * d[i];
    }
    load_v<V>(a + (size_t)p * aC + aoff + c, av);
#pragma unroll
    for (int i = 0; i < V; ++i) out[i] = av[i] > 0.f ? g[i] : 0.f;
    store_v<V>(dz + (size_t)p * zC + c, out);
}

// Mean squared error: dy = 2 (y - t)/n into a bf16 NHWC buffer (zero channel padding),
// per-block sums of (y - t)^2 in FP64.
__global__ void __launch_bounds__(256) k_mse(const float* __restrict__ yv, const float* __restrict__ t,
                                             int Cout, int HW, int P, int zC, double inv_n,
                                             bf16* __restrict__ dz, double* __restrict__ part)
{
    __shared__ double lds[256];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (k < P * zC) {
        const int p = k / zC, c = k - p * zC;
        float g = 0.f;
        if (c < Cout) {
            const int b = p / HW, r = p - b * HW;
            const size_t i = ((size_t)b * Cout + c) * HW + r;
            const double d = (double)yv[i] - (double)t[i];
            s = d * d;
            g = (float)(2.0 * d * inv_n);
        }
        dz[k] = f2bf(g);
    }
    lds[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) lds[threadIdx.x] += lds[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = lds[0];
}

__global__ void k_sum_d(const double* __restrict__ part, int n, double* __restrict__ out)
{
    __shared__ double lds[256];
    double s = 0.0;
    for (int k = threadIdx.x; k < n; k += blockDim.x) s += part[k];
    lds[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) lds[threadIdx.x] += lds[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = lds[0];
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, size_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2)
{
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.f - b1) * gk;
    const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// Bilinear resampling of nf fields [nf][sh][sw] onto [nf][dh][dw] (cell-centred grids,
// edge values held), dst = scale[f] * value + shift[f].
struct FieldAffine {
    float scale[16], shift[16];
};

__global__ void k_resample(const float* __restrict__ src, int sh, int sw, float* __restrict__ dst,
                           int dh, int dw, int nf, FieldAffine af)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nf * dh * dw) return;
    const int f = k / (dh * dw), r = k - f * dh * dw, y = r / dw, x = r - y * dw;
    const float fy = fminf(fmaxf((y + 0.5f) * sh / dh - 0.5f, 0.f), (float)(sh - 1));
    const float fx = fminf(fmaxf((x + 0.5f) * sw / dw - 0.5f, 0.f), (float)(sw - 1));
    const int y0 = (int)fy, x0 = (int)fx;
    const int y1 = min(y0 + 1, sh - 1), x1 = min(x0 + 1, sw - 1);
    const float ty = fy - y0, tx = fx - x0;
    const float* s = src + (size_t)f * sh * sw;
    const float v = (1.f - ty) * ((1.f - tx) * s[y0 * sw + x0] + tx * s[y0 * sw + x1]) +
                    ty * ((1.f - tx) * s[y1 * sw + x0] + tx * s[y1 * sw + x1]);
    dst[k] = af.scale[f] * v + af.shift[f];
}

// Input planes of the warm-start network for one problem per sample (see
// clbm_net_features in include/clbm.h for the channel list).
__global__ void k_features(const clbm_problem_code* __restrict__ codes, int B, int H, int W,
                           float* __restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= B * H * W) return;
    const int b = k / (H * W), r = k - b * H * W, y = r / W, x = r - y * W;
    const clbm_problem_code c = codes[b];
    // boundary cells of the network grid, side order x-, x+, y-, y+
    const bool at[4] = {x == 0, x == W - 1, y == 0, y == H - 1};
    float tw = 0.f, dir = 0.f, neu = 0.f;
    for (int s = 0; s < 4; ++s) {
        if (!at[s]) continue;
        if (c.kind[s] == 1) { dir = 1.f; tw = c.theta_wall[s]; }
        if (c.kind[s] == 2) neu = 1.f;
    }
    float* o = out + (size_t)b * 8 * H * W + r;
    const size_t pl = (size_t)H * W;
    o[0] = (c.log10_ra - 4.5f) / 1.5f;
    o[pl] = (c.pr - 3.85f) / 3.15f;
    o[2 * pl] = c.q_star / 4.f;
    o[3 * pl] = tw;
    o[4 * pl] = dir;
    o[5 * pl] = neu;
    o[6 * pl] = 2.f * (x + 0.5f) / W - 1.f;
    o[7 * pl] = c.log2_aspect;
}

}  // namespace clbm

using namespace clbm;

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

namespace {

struct TView {
    bf16* p;
    int C;    // channel stride
    int off;  // channel offset
};

struct Layer {
    int cin, cout;       // real sizes
    int cin_pad;         // K channels (multiple of 32)
    int nout_pad;        // forward N (multiple of 16 * NB)
    int nb;              // 16-channel blocks per wave in the forward
    int cout_kpad;       // K channels of the input-gradient convolution (multiple of 32)
    int H, W;            // resolution it runs at
    size_t woff, boff;   // offsets of W and b in the canonical vector
    bf16* wf;
    bf16* wb;
    TView in, out;       // forward input and output views
    TView dz;            // gradient w.r.t. the pre-activation (and output) of the layer
    TView din;           // gradient w.r.t. the input (nullptr p for layer 0)
};

int round_up(int v, int a) { return (v + a - 1) / a * a; }

}  // namespace

struct clbm_net {
    clbm_net_desc d;
    hipStream_t stream;
    Layer L[kLayers];
    size_t nparams;
    float *params, *grads, *adam_m, *adam_v;
    float* wpart;      // weight-gradient split partials
    size_t wpart_floats;
    float* bpart;      // bias-gradient partials
    double* lpart;     // loss partials
    double* loss;
    bf16* xin;         // packed input (cin padded)
    float* yout;       // network output fp32 NCHW
    bf16* dyout;       // loss gradient (cout padded to 32)
    // activations
    bf16 *a1, *cat1, *p1, *a2, *cat2, *p2, *a3, *cat3, *p3, *a4, *m4, *d3a, *d3b, *d2a, *d2b, *d1a, *d1b;
    // activation gradients
    bf16 *g_d1b, *g_d1a, *g_cat1, *g_d2b, *g_d2a, *g_cat2, *g_d3b, *g_d3a, *g_cat3, *g_m4, *g_a4, *g_p3,
        *g_a3, *g_p2, *g_a2, *g_p1, *g_a1, *g_z;  // g_z: scratch for dz of the current layer
    size_t zscratch;
    int weights_stale;
};

namespace {

struct Alloc {
    char* base;
    size_t off;
    bool dry;
    template <typename T>
    T* take(size_t count)
    {
        const size_t o = off;
        off = align_up(off + count * sizeof(T), kAlign);
        return dry ? nullptr : reinterpret_cast<T*>(base + o);
    }
};

clbm_status check_desc(const clbm_net_desc* d)
{
    if (!d) return CLBM_ERR_INVALID_ARG;
    if (d->batch < 1 || d->cin < 1 || d->cin > 32 || d->cout < 1 || d->cout > 16)
        return CLBM_ERR_INVALID_ARG;
    if (d->height < 16 || d->width < 16 || d->height % 8 || d->width % 8) return CLBM_ERR_INVALID_ARG;
    // the coarsest level must hold whole 64-pixel tiles
    if (((long)d->batch * (d->height / 8) * (d->width / 8)) % 64 != 0) return CLBM_ERR_INVALID_ARG;
    for (int k = 0; k < 4; ++k)
        if (d->widths[k] < 32 || d->widths[k] % 32) return CLBM_ERR_INVALID_ARG;
    return CLBM_OK;
}

// Lays out every buffer; with a.dry only counts bytes.
void layout_net(clbm_net* n, Alloc& a)
{
    const clbm_net_desc& d = n->d;
    const int B = d.batch, H = d.height, W = d.width;
    const int w1 = d.widths[0], w2 = d.widths[1], w3 = d.widths[2], w4 = d.widths[3];
    const size_t P1 = (size_t)B * H * W, P2 = P1 / 4, P3 = P1 / 16, P4 = P1 / 64;
    const int cinp = round_up(d.cin, 32);
    // activations
    n->xin = a.take<bf16>(P1 * cinp);
    n->a1 = a.take<bf16>(P1 * w1);
    n->cat1 = a.take<bf16>(P1 * (w2 + w1));
    n->p1 = a.take<bf16>(P2 * w1);
    n->a2 = a.take<bf16>(P2 * w2);
    n->cat2 = a.take<bf16>(P2 * (w3 + w2));
    n->p2 = a.take<bf16>(P3 * w2);
    n->a3 = a.take<bf16>(P3 * w3);
    n->cat3 = a.take<bf16>(P3 * (w4 + w3));
    n->p3 = a.take<bf16>(P4 * w3);
    n->a4 = a.take<bf16>(P4 * w4);
    n->m4 = a.take<bf16>(P4 * w4);
    n->d3a = a.take<bf16>(P3 * w3);
    n->d3b = a.take<bf16>(P3 * w3);
    n->d2a = a.take<bf16>(P2 * w2);
    n->d2b = a.take<bf16>(P2 * w2);
    n->d1a = a.take<bf16>(P1 * w1);
    n->d1b = a.take<bf16>(P1 * w1);
    n->yout = a.take<float>(P1 * d.cout);
    n->dyout = a.take<bf16>(P1 * 32);
    // gradients
    n->g_d1b = a.take<bf16>(P1 * w1);
    n->g_d1a = a.take<bf16>(P1 * w1);
    n->g_cat1 = a.take<bf16>(P1 * (w2 + w1));
    n->g_d2b = a.take<bf16>(P2 * w2);
    n->g_d2a = a.take<bf16>(P2 * w2);
    n->g_cat2 = a.take<bf16>(P2 * (w3 + w2));
    n->g_d3b = a.take<bf16>(P3 * w3);
    n->g_d3a = a.take<bf16>(P3 * w3);
    n->g_cat3 = a.take<bf16>(P3 * (w4 + w3));
    n->g_m4 = a.take<bf16>(P4 * w4);
    n->g_a4 = a.take<bf16>(P4 * w4);
    n->g_p3 = a.take<bf16>(P4 * w3);
    n->g_a3 = a.take<bf16>(P3 * w3);
    n->g_p2 = a.take<bf16>(P3 * w2);
    n->g_a2 = a.take<bf16>(P2 * w2);
    n->g_p1 = a.take<bf16>(P2 * w1);
    n->g_a1 = a.take<bf16>(P1 * w1);
    const size_t zmax = std::max({P1 * (size_t)w1, P2 * (size_t)w2, P3 * (size_t)w3, P4 * (size_t)w4});
    n->zscratch = zmax;
    n->g_z = a.take<bf16>(zmax);

    // layers
    const int cin_[kLayers] = {d.cin, w1, w1, w2, w2, w3, w3, w4, w4 + w3, w3, w3 + w2, w2, w2 + w1, w1, w1};
    const int cout_[kLayers] = {w1, w1, w2, w2, w3, w3, w4, w4, w3, w3, w2, w2, w1, w1, d.cout};
    const int res_[kLayers] = {1, 1, 2, 2, 4, 4, 8, 8, 4, 4, 2, 2, 1, 1, 1};
    size_t off = 0;
    for (int k = 0; k < kLayers; ++k) {
        Layer& l = n->L[k];
        l.cin = cin_[k];
        l.cout = cout_[k];
        l.cin_pad = round_up(l.cin, 32);
        l.nb = (l.cout % 64 == 0) ? 4 : (l.cout % 32 == 0 ? 2 : 1);
        l.nout_pad = round_up(l.cout, 16 * l.nb);
        l.cout_kpad = round_up(l.cout, 32);
        l.H = H / res_[k];
        l.W = W / res_[k];
        l.woff = off;
        off += (size_t)l.cout * l.cin * 9;
        l.boff = off;
        off += l.cout;
        l.wf = a.take<bf16>((size_t)l.nout_pad * 9 * l.cin_pad);
        l.wb = k == 0 ? nullptr : a.take<bf16>((size_t)l.cin_pad * 9 * l.cout_kpad);
    }
    n->nparams = off;
    n->params = a.take<float>(off);
    n->grads = a.take<float>(off);
    n->adam_m = a.take<float>(off);
    n->adam_v = a.take<float>(off);
    // split-K partials of the weight and bias gradients
    size_t wp = 0, bp = 0;
    for (int k = 0; k < kLayers; ++k) {
        const Layer& l = n->L[k];
        const size_t P = (size_t)B * l.H * l.W;
        const int c16 = round_up(l.cout, 16);
        const size_t pps = (size_t)wgrad_pixels_per_split(P, c16, l.cin_pad);
        wp = std::max(wp, (P + pps - 1) / pps * c16 * 9 * l.cin_pad);
        bp = std::max(bp, (P + pps - 1) / pps * c16);
    }
    n->wpart_floats = wp;
    n->wpart = a.take<float>(wp);
    n->bpart = a.take<float>(bp);
    n->lpart = a.take<double>((P1 * 32 + 255) / 256);
    n->loss = a.take<double>(1);

    // views: forward input/output of each layer
    auto V = [](bf16* p, int C, int off) { return TView{p, C, off}; };
    Layer* L = n->L;
    L[0].in = V(n->xin, cinp, 0);      L[0].out = V(n->a1, w1, 0);
    L[1].in = V(n->a1, w1, 0);         L[1].out = V(n->cat1, w2 + w1, w2);   // s1
    L[2].in = V(n->p1, w1, 0);         L[2].out = V(n->a2, w2, 0);
    L[3].in = V(n->a2, w2, 0);         L[3].out = V(n->cat2, w3 + w2, w3);   // s2
    L[4].in = V(n->p2, w2, 0);         L[4].out = V(n->a3, w3, 0);
    L[5].in = V(n->a3, w3, 0);         L[5].out = V(n->cat3, w4 + w3, w4);   // s3
    L[6].in = V(n->p3, w3, 0);         L[6].out = V(n->a4, w4, 0);
    L[7].in = V(n->a4, w4, 0);         L[7].out = V(n->m4, w4, 0);
    L[8].in = V(n->cat3, w4 + w3, 0);  L[8].out = V(n->d3a, w3, 0);
    L[9].in = V(n->d3a, w3, 0);        L[9].out = V(n->d3b, w3, 0);
    L[10].in = V(n->cat2, w3 + w2, 0); L[10].out = V(n->d2a, w2, 0);
    L[11].in = V(n->d2a, w2, 0);       L[11].out = V(n->d2b, w2, 0);
    L[12].in = V(n->cat1, w2 + w1, 0); L[12].out = V(n->d1a, w1, 0);
    L[13].in = V(n->d1a, w1, 0);       L[13].out = V(n->d1b, w1, 0);
    L[14].in = V(n->d1b, w1, 0);       L[14].out = V(nullptr, 0, 0);
    // gradient w.r.t. each layer's input
    L[0].din = V(nullptr, 0, 0);
    L[1].din = V(n->g_a1, w1, 0);
    L[2].din = V(n->g_p1, w1, 0);
    L[3].din = V(n->g_a2, w2, 0);
    L[4].din = V(n->g_p2, w2, 0);
    L[5].din = V(n->g_a3, w3, 0);
    L[6].din = V(n->g_p3, w3, 0);
    L[7].din = V(n->g_a4, w4, 0);
    L[8].din = V(n->g_cat3, w4 + w3, 0);
    L[9].din = V(n->g_d3a, w3, 0);
    L[10].din = V(n->g_cat2, w3 + w2, 0);
    L[11].din = V(n->g_d2a, w2, 0);
    L[12].din = V(n->g_cat1, w2 + w1, 0);
    L[13].din = V(n->g_d1a, w1, 0);
    L[14].din = V(n->g_d1b, w1, 0);
}

dim3 grid1(size_t n, int block = 256) { return dim3((unsigned)((n + block - 1) / block)); }

// True when every channel count, stride and offset allows 8-channel (16-byte) accesses.
bool vec8(std::initializer_list<int> v)
{
    for (int x : v)
        if (x % 8 != 0) return false;
    return true;
}

// Gradient of the nearest upsampling into a channel view (dy: 2H x 2W, dx: H x W).
clbm_status upsample_bwd(clbm_net* n, TView dy, int C, int H, int W, TView dx)
{
    const int B = n->d.batch;
    if (vec8({C, dy.C, dy.off, dx.C, dx.off}))
        hipLaunchKernelGGL(k_upsample_bwd<8>, grid1((size_t)B * H * W * (C / 8)), dim3(256), 0, n->stream,
                           dy.p, dy.C, dy.off, C, H, W, B, dx.p, dx.C, dx.off);
    else
        hipLaunchKernelGGL(k_upsample_bwd<1>, grid1((size_t)B * H * W * C), dim3(256), 0, n->stream,
                           dy.p, dy.C, dy.off, C, H, W, B, dx.p, dx.C, dx.off);
    CLBM_HIP(hipGetLastError());
    return CLBM_OK;
}

clbm_status conv_launch(clbm_net* n, const Layer& l, TView in, int cin_pad, const bf16* w,
                        const float* bias, int N, int nb, int npad, int mode, TView out, float* yf)
{
    const int P = n->d.batch * l.H * l.W;
    int xC = in.C, xoff = in.off, Cin = cin_pad, H = l.H, W = l.W, yC = out.C, yoff = out.off;
    const bf16* x = in.p;
    bf16* y = out.p;
    void* args[] = {&x, &xC, &xoff, &Cin, (void*)&w, (void*)&bias, &N, &H, &W, &mode, &y, &yC, &yoff, &yf};
    // LDS-staged kernel: pixel blocks of 256 (BW = 64, 32 or 16 columns) that tile the image
    const int bw = W >= 64 ? 64 : W;
    if ((nb == 4 || nb == 2) && (bw == 64 || bw == 32 || bw == 16) && W % bw == 0 && H % (256 / bw) == 0) {
        const void* fl = nb == 4 ? (bw == 64 ? (const void*)&k_conv_lds<4, 64> : bw == 32 ? (const void*)&k_conv_lds<4, 32> : (const void*)&k_conv_lds<4, 16>)
                                 : (bw == 64 ? (const void*)&k_conv_lds<2, 64> : bw == 32 ? (const void*)&k_conv_lds<2, 32> : (const void*)&k_conv_lds<2, 16>);
        CLBM_HIP(hipLaunchKernel(fl, dim3(P / 256, npad / (16 * nb)), dim3(256), args, 0, n->stream));
        return CLBM_OK;
    }
    // four 16-pixel blocks per wave where the pixel count allows (it is a multiple of 64)
    const int mp = P % 256 == 0 ? 4 : 1;
    const dim3 grid(P / (64 * mp), npad / (16 * nb));
    const void* fn =
        mp == 4 ? (nb == 4 ? reinterpret_cast<const void*>(&k_conv<4, 4>)
                  : nb == 2 ? reinterpret_cast<const void*>(&k_conv<2, 4>)
                            : reinterpret_cast<const void*>(&k_conv<1, 4>))
                : (nb == 4 ? reinterpret_cast<const void*>(&k_conv<4, 1>)
                  : nb == 2 ? reinterpret_cast<const void*>(&k_conv<2, 1>)
                            : reinterpret_cast<const void*>(&k_conv<1, 1>));
    CLBM_HIP(hipLaunchKernel(fn, grid, dim3(256), args, 0, n->stream));
    return CLBM_OK;
}

clbm_status prep_weights(clbm_net* n)
{
    for (int k = 0; k < kLayers; ++k) {
        const Layer& l = n->L[k];
        const size_t nf = (size_t)l.nout_pad * 9 * l.cin_pad;
        const size_t nbk = l.wb ? (size_t)l.cin_pad * 9 * l.cout_kpad : 0;
        hipLaunchKernelGGL(k_weight_prep, grid1(std::max(nf, nbk)), dim3(256), 0, n->stream,
                           n->params + l.woff, l.cout, l.cin, l.nout_pad, l.cin_pad, l.cout_kpad,
                           l.wf, l.wb);
        CLBM_HIP(hipGetLastError());
    }
    n->weights_stale = 0;
    return CLBM_OK;
}

clbm_status ew_launch_check() { CLBM_HIP(hipGetLastError()); return CLBM_OK; }

clbm_status pool(clbm_net* n, TView x, int C, int H, int W, TView y)
{
    const int B = n->d.batch;
    if (vec8({C, x.C, x.off, y.C, y.off}))
        hipLaunchKernelGGL(k_avgpool<8>, grid1((size_t)B * (H / 2) * (W / 2) * (C / 8)), dim3(256), 0,
                           n->stream, x.p, x.C, x.off, C, H, W, B, y.p, y.C, y.off);
    else
        hipLaunchKernelGGL(k_avgpool<1>, grid1((size_t)B * (H / 2) * (W / 2) * C), dim3(256), 0, n->stream,
                           x.p, x.C, x.off, C, H, W, B, y.p, y.C, y.off);
    return ew_launch_check();
}

clbm_status upsample(clbm_net* n, TView x, int C, int H, int W, TView y)
{
    const int B = n->d.batch;
    if (vec8({C, x.C, x.off, y.C, y.off}))
        hipLaunchKernelGGL(k_upsample<8>, grid1((size_t)B * 4 * H * W * (C / 8)), dim3(256), 0, n->stream,
                           x.p, x.C, x.off, C, H, W, B, y.p, y.C, y.off);
    else
        hipLaunchKernelGGL(k_upsample<1>, grid1((size_t)B * 4 * H * W * C), dim3(256), 0, n->stream, x.p,
                           x.C, x.off, C, H, W, B, y.p, y.C, y.off);
    return ew_launch_check();
}

// Backward through one convolution: dz (gradient w.r.t. its output pre-activation,
// ReLU already applied) -> weight and bias gradients, and the input gradient when the
// layer has one.
clbm_status conv_backward(clbm_net* n, int k, TView dz)
{
    const Layer& l = n->L[k];
    const int B = n->d.batch;
    const int P = B * l.H * l.W;
    const int cout16 = round_up(l.cout, 16);
    const int pps = wgrad_pixels_per_split((size_t)P, cout16, l.cin_pad);
    const int splits = (P + pps - 1) / pps;
    // weight gradient
    const int nco = wgrad_blocks16(cout16 / 16), nci = wgrad_blocks16(l.cin_pad / 16);
    const void* wg = nco == 4 ? (nci == 4 ? (const void*)&k_wgrad<4, 4> : nci == 2 ? (const void*)&k_wgrad<4, 2> : (const void*)&k_wgrad<4, 1>)
                   : nco == 2 ? (nci == 4 ? (const void*)&k_wgrad<2, 4> : nci == 2 ? (const void*)&k_wgrad<2, 2> : (const void*)&k_wgrad<2, 1>)
                              : (nci == 4 ? (const void*)&k_wgrad<1, 4> : nci == 2 ? (const void*)&k_wgrad<1, 2> : (const void*)&k_wgrad<1, 1>);
    {
        const bf16* zp = dz.p; int zc = dz.C, co = cout16; const bf16* xp = l.in.p; int xc = l.in.C, xo = l.in.off;
        int ci = l.cin_pad, h = l.H, w = l.W, pp = P, ps = pps; float* pt = n->wpart; float* bt = n->bpart;
        void* args[] = {&zp, &zc, &co, &xp, &xc, &xo, &ci, &h, &w, &pp, &ps, &pt, &bt};
        CLBM_HIP(hipLaunchKernel(wg, dim3((cout16 / (16 * nco)) * (l.cin_pad / (16 * nci)), splits),
                                 dim3(kWgThreads), args, 0, n->stream));
    }
    CLBM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_wgrad_reduce, grid1((size_t)cout16 * 9 * l.cin_pad), dim3(256), 0, n->stream,
                       n->wpart, splits, cout16, l.cin_pad, l.cout, l.cin, n->grads + l.woff);
    CLBM_HIP(hipGetLastError());
    // bias gradient: the weight-gradient kernel left one partial per split
    hipLaunchKernelGGL(k_bias_reduce, dim3(l.cout), dim3(256), 0, n->stream, n->bpart, splits, cout16,
                       n->grads + l.boff);
    CLBM_HIP(hipGetLastError());
    // input gradient: convolution of dz with the flipped, transposed kernel
    if (l.din.p) {
        const int nb = (l.cin % 64 == 0) ? 4 : 2;
        return conv_launch(n, l, dz, l.cout_kpad, l.wb, nullptr, l.cin, nb, round_up(l.cin, 16 * nb), 1,
                           l.din, nullptr);
    }
    return CLBM_OK;
}

clbm_status relu_grad(clbm_net* n, TView dy, TView dpool_parent, TView act, int C, int H, int W, TView dz)
{
    const int B = n->d.batch;
    if (vec8({C, dy.C, dy.off, dpool_parent.C, act.C, act.off, dz.C}))
        hipLaunchKernelGGL(k_relu_grad<8>, grid1((size_t)B * H * W * (C / 8)), dim3(256), 0, n->stream,
                           dy.p, dy.C, dy.off, dpool_parent.p, dpool_parent.C, act.p, act.C, act.off, C,
                           H, W, B, dz.p, dz.C);
    else
        hipLaunchKernelGGL(k_relu_grad<1>, grid1((size_t)B * H * W * C), dim3(256), 0, n->stream, dy.p,
                           dy.C, dy.off, dpool_parent.p, dpool_parent.C, act.p, act.C, act.off, C, H,
                           W, B, dz.p, dz.C);
    return ew_launch_check();
}

}  // namespace

extern "C" {

clbm_status clbm_net_param_count(const clbm_net_desc* d, size_t* count)
{
    if (!count) return CLBM_ERR_INVALID_ARG;
    clbm_status st = check_desc(d);
    if (st != CLBM_OK) return st;
    clbm_net tmp;
    std::memset(&tmp, 0, sizeof tmp);
    tmp.d = *d;
    Alloc a{nullptr, 0, true};
    layout_net(&tmp, a);
    *count = tmp.nparams;
    return CLBM_OK;
}

clbm_status clbm_net_workspace_bytes(const clbm_net_desc* d, size_t* bytes)
{
    if (!bytes) return CLBM_ERR_INVALID_ARG;
    clbm_status st = check_desc(d);
    if (st != CLBM_OK) return st;
    clbm_net tmp;
    std::memset(&tmp, 0, sizeof tmp);
    tmp.d = *d;
    Alloc a{nullptr, 0, true};
    layout_net(&tmp, a);
    *bytes = a.off;
    return CLBM_OK;
}

clbm_status clbm_net_create(const clbm_net_desc* d, void* d_workspace, size_t bytes, void* hip_stream,
                            clbm_net** out)
{
    if (!out) return CLBM_ERR_INVALID_ARG;
    *out = nullptr;
    clbm_status st = check_desc(d);
    if (st != CLBM_OK) return st;
    size_t need = 0;
    clbm_net_workspace_bytes(d, &need);
    if (!d_workspace || ((uintptr_t)d_workspace) % kAlign) return CLBM_ERR_INVALID_ARG;
    if (bytes < need) return CLBM_ERR_BUFFER_TOO_SMALL;
    clbm_net* n = new (std::nothrow) clbm_net;
    if (!n) return CLBM_ERR_INVALID_ARG;
    std::memset(n, 0, sizeof *n);
    n->d = *d;
    n->stream = (hipStream_t)hip_stream;
    Alloc a{(char*)d_workspace, 0, false};
    layout_net(n, a);
    // zero everything once (padding channels must read as zeros), Adam moments included
    hipError_t e = hipMemsetAsync(d_workspace, 0, need, n->stream);
    if (e != hipSuccess) {
        delete n;
        set_last_hip_error(e, "hipMemsetAsync", __FILE__, __LINE__);
        return CLBM_ERR_HIP;
    }
    n->weights_stale = 1;
    *out = n;
    return CLBM_OK;
}

void clbm_net_destroy(clbm_net* n) { delete n; }

clbm_status clbm_net_set_params(clbm_net* n, const float* d_params)
{
    if (!n || !d_params) return CLBM_ERR_INVALID_ARG;
    CLBM_HIP(hipMemcpyAsync(n->params, d_params, n->nparams * sizeof(float), hipMemcpyDeviceToDevice,
                            n->stream));
    n->weights_stale = 1;
    return CLBM_OK;
}

clbm_status clbm_net_get_params(clbm_net* n, float* d_params)
{
    if (!n || !d_params) return CLBM_ERR_INVALID_ARG;
    CLBM_HIP(hipMemcpyAsync(d_params, n->params, n->nparams * sizeof(float), hipMemcpyDeviceToDevice,
                            n->stream));
    return CLBM_OK;
}

clbm_status clbm_net_get_grads(clbm_net* n, float* d_grads)
{
    if (!n || !d_grads) return CLBM_ERR_INVALID_ARG;
    CLBM_HIP(hipMemcpyAsync(d_grads, n->grads, n->nparams * sizeof(float), hipMemcpyDeviceToDevice,
                            n->stream));
    return CLBM_OK;
}

clbm_status clbm_net_forward(clbm_net* n, const float* d_x, float* d_y)
{
    if (!n || !d_x) return CLBM_ERR_INVALID_ARG;
    const clbm_net_desc& d = n->d;
    const int B = d.batch, H = d.height, W = d.width;
    const int w1 = d.widths[0], w2 = d.widths[1], w3 = d.widths[2], w4 = d.widths[3];
    clbm_status st = CLBM_OK;
    if (n->weights_stale && (st = prep_weights(n)) != CLBM_OK) return st;
    const int cinp = round_up(d.cin, 32);
    hipLaunchKernelGGL(k_pack_input, grid1((size_t)B * H * W * cinp), dim3(256), 0, n->stream, d_x, d.cin,
                       H * W, B * H * W, n->xin, cinp);
    CLBM_HIP(hipGetLastError());
    Layer* L = n->L;
    auto fwd = [&](int k) {
        const Layer& l = L[k];
        return conv_launch(n, l, l.in, l.cin_pad, l.wf, n->params + l.boff, l.cout, l.nb, l.nout_pad,
                           k == 14 ? 2 : 0, l.out, k == 14 ? n->yout : nullptr);
    };
    auto V = [](bf16* p, int C, int off) { return TView{p, C, off}; };
    if ((st = fwd(0)) || (st = fwd(1))) return st;
    if ((st = pool(n, V(n->cat1, w2 + w1, w2), w1, H, W, V(n->p1, w1, 0)))) return st;
    if ((st = fwd(2)) || (st = fwd(3))) return st;
    if ((st = pool(n, V(n->cat2, w3 + w2, w3), w2, H / 2, W / 2, V(n->p2, w2, 0)))) return st;
    if ((st = fwd(4)) || (st = fwd(5))) return st;
    if ((st = pool(n, V(n->cat3, w4 + w3, w4), w3, H / 4, W / 4, V(n->p3, w3, 0)))) return st;
    if ((st = fwd(6)) || (st = fwd(7))) return st;
    if ((st = upsample(n, V(n->m4, w4, 0), w4, H / 8, W / 8, V(n->cat3, w4 + w3, 0)))) return st;
    if ((st = fwd(8)) || (st = fwd(9))) return st;
    if ((st = upsample(n, V(n->d3b, w3, 0), w3, H / 4, W / 4, V(n->cat2, w3 + w2, 0)))) return st;
    if ((st = fwd(10)) || (st = fwd(11))) return st;
    if ((st = upsample(n, V(n->d2b, w2, 0), w2, H / 2, W / 2, V(n->cat1, w2 + w1, 0)))) return st;
    if ((st = fwd(12)) || (st = fwd(13)) || (st = fwd(14))) return st;
    if (d_y)
        CLBM_HIP(hipMemcpyAsync(d_y, n->yout, (size_t)B * d.cout * H * W * sizeof(float),
                                hipMemcpyDeviceToDevice, n->stream));
    return CLBM_OK;
}

clbm_status clbm_net_backward(clbm_net* n, const float* d_target, double* loss)
{
    if (!n || !d_target) return CLBM_ERR_INVALID_ARG;
    const clbm_net_desc& d = n->d;
    const int B = d.batch, H = d.height, W = d.width;
    const int w1 = d.widths[0], w2 = d.widths[1], w3 = d.widths[2], w4 = d.widths[3];
    const int P1 = B * H * W;
    auto V = [](bf16* p, int C, int off) { return TView{p, C, off}; };
    const TView none = V(nullptr, 0, 0);
    clbm_status st = CLBM_OK;
    // loss and its gradient
    const int nblk = (P1 * 32 + 255) / 256;
    hipLaunchKernelGGL(k_mse, dim3(nblk), dim3(256), 0, n->stream, n->yout, d_target, d.cout, H * W, P1,
                       32, 1.0 / ((double)P1 * d.cout), n->dyout, n->lpart);
    CLBM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum_d, dim3(1), dim3(256), 0, n->stream, n->lpart, nblk, n->loss);
    CLBM_HIP(hipGetLastError());
    auto zv = [&](int C) { return TView{n->g_z, C, 0}; };
    // output layer (no activation)
    if ((st = conv_backward(n, 14, V(n->dyout, 32, 0)))) return st;
    // level-1 decoder
    if ((st = relu_grad(n, V(n->g_d1b, w1, 0), none, V(n->d1b, w1, 0), w1, H, W, zv(w1)))) return st;
    if ((st = conv_backward(n, 13, zv(w1)))) return st;
    if ((st = relu_grad(n, V(n->g_d1a, w1, 0), none, V(n->d1a, w1, 0), w1, H, W, zv(w1)))) return st;
    if ((st = conv_backward(n, 12, zv(w1)))) return st;
    // g_cat1 = [d up(d2b) | d s1]
    if ((st = upsample_bwd(n, V(n->g_cat1, w2 + w1, 0), w2, H / 2, W / 2, V(n->g_d2b, w2, 0)))) return st;
    // level-2 decoder
    if ((st = relu_grad(n, V(n->g_d2b, w2, 0), none, V(n->d2b, w2, 0), w2, H / 2, W / 2, zv(w2)))) return st;
    if ((st = conv_backward(n, 11, zv(w2)))) return st;
    if ((st = relu_grad(n, V(n->g_d2a, w2, 0), none, V(n->d2a, w2, 0), w2, H / 2, W / 2, zv(w2)))) return st;
    if ((st = conv_backward(n, 10, zv(w2)))) return st;
    if ((st = upsample_bwd(n, V(n->g_cat2, w3 + w2, 0), w3, H / 4, W / 4, V(n->g_d3b, w3, 0)))) return st;
    // level-3 decoder
    if ((st = relu_grad(n, V(n->g_d3b, w3, 0), none, V(n->d3b, w3, 0), w3, H / 4, W / 4, zv(w3)))) return st;
    if ((st = conv_backward(n, 9, zv(w3)))) return st;
    if ((st = relu_grad(n, V(n->g_d3a, w3, 0), none, V(n->d3a, w3, 0), w3, H / 4, W / 4, zv(w3)))) return st;
    if ((st = conv_backward(n, 8, zv(w3)))) return st;
    if ((st = upsample_bwd(n, V(n->g_cat3, w4 + w3, 0), w4, H / 8, W / 8, V(n->g_m4, w4, 0)))) return st;
    // bottom level
    if ((st = relu_grad(n, V(n->g_m4, w4, 0), none, V(n->m4, w4, 0), w4, H / 8, W / 8, zv(w4)))) return st;
    if ((st = conv_backward(n, 7, zv(w4)))) return st;
    if ((st = relu_grad(n, V(n->g_a4, w4, 0), none, V(n->a4, w4, 0), w4, H / 8, W / 8, zv(w4)))) return st;
    if ((st = conv_backward(n, 6, zv(w4)))) return st;
    // encoder: skip gradient + pooled gradient, through the ReLU
    if ((st = relu_grad(n, V(n->g_cat3, w4 + w3, w4), V(n->g_p3, w3, 0), V(n->cat3, w4 + w3, w4), w3,
                        H / 4, W / 4, zv(w3)))) return st;
    if ((st = conv_backward(n, 5, zv(w3)))) return st;
    if ((st = relu_grad(n, V(n->g_a3, w3, 0), none, V(n->a3, w3, 0), w3, H / 4, W / 4, zv(w3)))) return st;
    if ((st = conv_backward(n, 4, zv(w3)))) return st;
    if ((st = relu_grad(n, V(n->g_cat2, w3 + w2, w3), V(n->g_p2, w2, 0), V(n->cat2, w3 + w2, w3), w2,
                        H / 2, W / 2, zv(w2)))) return st;
    if ((st = conv_backward(n, 3, zv(w2)))) return st;
    if ((st = relu_grad(n, V(n->g_a2, w2, 0), none, V(n->a2, w2, 0), w2, H / 2, W / 2, zv(w2)))) return st;
    if ((st = conv_backward(n, 2, zv(w2)))) return st;
    if ((st = relu_grad(n, V(n->g_cat1, w2 + w1, w2), V(n->g_p1, w1, 0), V(n->cat1, w2 + w1, w2), w1, H,
                        W, zv(w1)))) return st;
    if ((st = conv_backward(n, 1, zv(w1)))) return st;
    if ((st = relu_grad(n, V(n->g_a1, w1, 0), none, V(n->a1, w1, 0), w1, H, W, zv(w1)))) return st;
    if ((st = conv_backward(n, 0, zv(w1)))) return st;
    if (loss) {
        double sum = 0.0;
        CLBM_HIP(hipMemcpyAsync(&sum, n->loss, sizeof(double), hipMemcpyDeviceToHost, n->stream));
        CLBM_HIP(hipStreamSynchronize(n->stream));
        *loss = sum / ((double)P1 * d.cout);
    }
    return CLBM_OK;
}

clbm_status clbm_net_adam(clbm_net* n, float lr, float beta1, float beta2, float eps, int t)
{
    if (!n || t < 1) return CLBM_ERR_INVALID_ARG;
    const float c1 = 1.f - std::pow(beta1, (float)t), c2 = 1.f - std::pow(beta2, (float)t);
    hipLaunchKernelGGL(k_adam, grid1(n->nparams), dim3(256), 0, n->stream, n->params, n->grads, n->adam_m,
                       n->adam_v, n->nparams, lr, beta1, beta2, eps, c1, c2);
    CLBM_HIP(hipGetLastError());
    n->weights_stale = 1;
    return CLBM_OK;
}

clbm_status clbm_resample_bilinear(const float* d_src, int sh, int sw, float* d_dst, int dh, int dw,
                                   int nfields, const float* scale, const float* shift,
                                   void* hip_stream)
{
    if (!d_src || !d_dst || sh < 1 || sw < 1 || dh < 1 || dw < 1 || nfields < 1 || nfields > 16)
        return CLBM_ERR_INVALID_ARG;
    FieldAffine af;
    for (int f = 0; f < 16; ++f) {
        af.scale[f] = (scale && f < nfields) ? scale[f] : 1.f;
        af.shift[f] = (shift && f < nfields) ? shift[f] : 0.f;
    }
    hipLaunchKernelGGL(k_resample, grid1((size_t)nfields * dh * dw), dim3(256), 0, (hipStream_t)hip_stream,
                       d_src, sh, sw, d_dst, dh, dw, nfields, af);
    CLBM_HIP(hipGetLastError());
    return CLBM_OK;
}

clbm_status clbm_net_features(const clbm_problem_code* d_codes, int batch, int height, int width,
                              float* d_out, void* hip_stream)
{
    if (!d_codes || !d_out || batch < 1 || height < 1 || width < 1) return CLBM_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_features, grid1((size_t)batch * height * width), dim3(256), 0,
                       (hipStream_t)hip_stream, d_codes, batch, height, width, d_out);
    CLBM_HIP(hipGetLastError());
    return CLBM_OK;
}

clbm_status clbm_problem_encode(const clbm_params* p, clbm_problem_code* out)
{
    if (!p || !out) return CLBM_ERR_INVALID_ARG;
    Rates r;
    clbm_status st = derive_rates(p, &r);
    if (st != CLBM_OK) return st;
    // Sec. 3.3: the cavity height H = ny, dT = T(x-) - T(x+) of the Dirichlet side walls
    // (1 when they are not both Dirichlet); Ra = g beta dT H^3/(nu alpha), Pr = nu/alpha.
    const double H = p->ny;
    double dT = 1.0;
    if (p->side[0].kind == CLBM_WALL && p->side[1].kind == CLBM_WALL && p->side[0].b1 == 0.0 &&
        p->side[1].b1 == 0.0 && p->side[0].b2 != 0.0 && p->side[1].b2 != 0.0) {
        const double d = p->side[0].b3 / p->side[0].b2 - p->side[1].b3 / p->side[1].b2;
        if (d != 0.0) dT = std::fabs(d);
    }
    const double Ra = std::max(p->g_beta * dT * H * H * H / (p->nu * p->alpha), 1.0);
    std::memset(out, 0, sizeof *out);
    out->log10_ra = (float)std::log10(Ra);
    out->pr = (float)(p->nu / p->alpha);
    out->q_star = (float)(p->Q * H * H / (p->alpha * dT));
    out->log2_aspect = (float)std::log2((double)p->nx / p->ny);
    for (int s = 0; s < 4; ++s) {
        const clbm_side& sd = p->side[s];
        if (sd.kind != CLBM_WALL) {
            out->kind[s] = 0;
        } else if (sd.b1 == 0.0) {
            out->kind[s] = 1;
            out->theta_wall[s] = (float)((sd.b3 / sd.b2 - p->T0) / dT);
        } else {
            out->kind[s] = (sd.b2 == 0.0 && sd.b3 == 0.0) ? 2 : 3;
        }
    }
    out->u_scale = (float)std::sqrt(p->g_beta * dT * H);
    out->t_scale = (float)dT;
    return CLBM_OK;
}

}  // extern "C"
