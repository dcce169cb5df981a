// Learned initialiser: a U-Net on BF16 MFMA (gfx950) with FP32 accumulation.
//
// Layout: activations NHWC in BF16 (element (n, y, x, c) at
// ((n * H + y) * W + x) * cs + coff + c, so a concatenation is two channel
// ranges of one buffer); 3x3 weights [co][tap][ci] with tap = 3 * ky + kx for
// offsets (ky - 1, kx - 1). Master weights, Adam moments and gradients are FP32.
//
// Kernels:
//   conv3x3_tiled  implicit GEMM for the larger layers, M = pixels, N = out
//                  channels, K = 9 * in channels, v_mfma_f32_32x32x16_bf16, input
//                  patch staged in LDS; forward (bias + SiLU epilogue) and
//                  backward-data (the same GEMM with flipped, transposed weights;
//                  optional SiLU' and accumulation epilogue);
//   conv3x3_mfma   the same GEMM with operands read directly (M = out channels,
//                  N = pixels), for small grids;
//   conv3x3_wgrad  weight gradient, M = out channels, N = in channels per tap,
//                  K = pixels, operands staged transposed in LDS, split over
//                  pixel chunks with a fixed-order reduction (deterministic);
//   pool / upsample / head 1x1 / SiLU' / MSE / bias sums / Adam (optionally
//   with global-norm gradient clipping): kernels on 8-channel vectors.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/ss.h"
#include "../../include/ssn.h"

namespace ssn {

typedef unsigned short bf16_t;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(4))) unsigned u32x4;

__device__ __forceinline__ float bf2f(bf16_t x) { return __uint_as_float(((unsigned)x) << 16); }

// round to nearest even (finite inputs; Inf/NaN keep their class)
__device__ __forceinline__ bf16_t f2bf(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (bf16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_grad_f(float z) {
  const float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// NHWC view
struct TV {
  bf16_t* p;
  int N, H, W;
  int cs;   // channel stride of the buffer
  int coff; // first channel of this view
  int C;    // channels of this view
};

__device__ __forceinline__ long tv_at(const TV& t, int n, int y, int x) {
  return ((long)(n * t.H + y) * t.W + x) * t.cs + t.coff;
}

struct ConvArgs {
  TV in;             // input, in.C a multiple of 16
  const bf16_t* w;   // [rows][9][in.C], rows = Co rounded up to 32
  const float* bias; // [Co] or nullptr
  int Co;
  TV out_z;          // forward: pre-activation (p may be nullptr)
  TV out;            // forward: SiLU(z); backward: gradient w.r.t. the input of the layer
  TV zprev;          // backward: if p != nullptr multiply by SiLU'(zprev)
  int mode;          // 0 forward, 1 backward-data
  int accumulate;    // backward: out += result
};

// Each wave: 32 output channels x (32 * WN) pixels; block: WB waves along pixels.
template <int WN, int WB>
__global__ void __launch_bounds__(64 * WB) conv3x3_mfma(ConvArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 31, half = lane >> 5;
  const int co0 = blockIdx.y * 32;
  const int H = a.in.H, W = a.in.W, Ci = a.in.C;
  const long P = (long)a.in.N * H * W;
  const long pixbase = ((long)blockIdx.x * WB + wave) * (32 * WN);
  int pn[WN], py[WN], px[WN];
  bool pv[WN];
#pragma unroll
  for (int f = 0; f < WN; ++f) {
    const long pix = pixbase + f * 32 + r;
    pv[f] = pix < P;
    const long pp = pv[f] ? pix : 0;
    pn[f] = (int)(pp / ((long)H * W));
    const int rem = (int)(pp - (long)pn[f] * H * W);
    py[f] = rem / W;
    px[f] = rem - py[f] * W;
  }
  f32x16 acc[WN];
#pragma unroll
  for (int f = 0; f < WN; ++f)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[f][v] = 0.0f;
  const bf16_t* wrow = a.w + (long)(co0 + r) * 9 * Ci + half * 8;
  bf16x8 zero;
#pragma unroll
  for (int j = 0; j < 8; ++j) zero[j] = (__bf16)0.0f;
  for (int t = 0; t < 9; ++t) {
    const int dy = t / 3 - 1, dx = t % 3 - 1;
    long boff[WN];
    bool bv[WN];
#pragma unroll
    for (int f = 0; f < WN; ++f) {
      const int yy = py[f] + dy, xx = px[f] + dx;
      bv[f] = pv[f] && yy >= 0 && yy < H && xx >= 0 && xx < W;
      boff[f] = bv[f] ? tv_at(a.in, pn[f], yy, xx) + half * 8 : 0;
    }
    for (int c = 0; c < Ci; c += 16) {
      const bf16x8 A = *reinterpret_cast<const bf16x8*>(wrow + t * Ci + c);
#pragma unroll
      for (int f = 0; f < WN; ++f) {
        const bf16x8 B = bv[f] ? *reinterpret_cast<const bf16x8*>(a.in.p + boff[f] + c) : zero;
        acc[f] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, acc[f], 0, 0, 0);
      }
    }
  }
  // D[row][col]: lane holds col = r (pixel) and rows 8 (v / 4) + 4 half + v % 4 (channels)
#pragma unroll
  for (int f = 0; f < WN; ++f) {
    if (!pv[f]) continue;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int co = co0 + (v >> 2) * 8 + half * 4 + (v & 3);
      if (co >= a.Co) continue;
      float val = acc[f][v];
      if (a.mode == 0) {
        const float z = val + (a.bias ? a.bias[co] : 0.0f);
        if (a.out_z.p) a.out_z.p[tv_at(a.out_z, pn[f], py[f], px[f]) + co] = f2bf(z);
        a.out.p[tv_at(a.out, pn[f], py[f], px[f]) + co] = f2bf(silu_f(z));
      } else {
        if (a.zprev.p) val *= silu_grad_f(bf2f(a.zprev.p[tv_at(a.zprev, pn[f], py[f], px[f]) + co]));
        bf16_t* o = a.out.p + tv_at(a.out, pn[f], py[f], px[f]) + co;
        if (a.accumulate) val += bf2f(*o);
        *o = f2bf(val);
      }
    }
  }
}

// LDS-tiled implicit GEMM for the larger layers. Block: WCO x WPX waves over R
// image rows; wave (i, j) computes 32 output channels (co0 + 32 i ..) x 32 pixels
// (x0 + 32 j ..) of each of the rows y0 .. y0 + R - 1. Input channels are taken
// in chunks of 32: the chunk's input patch (R + 2 rows x (32 WPX + 2) pixels,
// zero outside the image) is staged in LDS, each entry padded to kKP channels
// so that lanes reading neighbouring pixels or rows fall in different banks.
// The weight fragments (a few KB per layer, shared by every workgroup) are read
// straight from global memory through the caches, which leaves LDS to the patch
// (one more workgroup per CU than staging them); each serves R rows. Requires
// W % (32 WPX) == 0, H % R == 0, in.C % 16 == 0 and, for WCO = 2, Co % 64 == 0
// (weight rows exist up to gridDim.y * 32 WCO).
constexpr int kKC = 32, kKP = 40;

template <int WCO, int WPX, int R>
__global__ void __launch_bounds__(64 * WCO * WPX) conv3x3_tiled(ConvArgs a) {
  constexpr int NT = 64 * WCO * WPX, PX = 32 * WPX, PW = PX + 2, CO = 32 * WCO, PR = R + 2;
  __shared__ __align__(16) bf16_t sin_[PR * PW * kKP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave / WPX, wj = wave - wi * WPX;
  const int r = lane & 31, half = lane >> 5;
  const int H = a.in.H, W = a.in.W, Ci = a.in.C;
  const int xt = W / PX, yt = H / R;
  const int bx = blockIdx.x;
  const int n = bx / (yt * xt);
  const int rem = bx - n * yt * xt;
  const int y0 = (rem / xt) * R;
  const int x0 = (rem - (rem / xt) * xt) * PX;
  const int co0 = blockIdx.y * CO;
  bf16x8 zero;
#pragma unroll
  for (int j = 0; j < 8; ++j) zero[j] = (__bf16)0.0f;
  f32x16 acc[R];
#pragma unroll
  for (int q = 0; q < R; ++q)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[q][v] = 0.0f;
  for (int c0 = 0; c0 < Ci; c0 += kKC) {
    const int kc = min(kKC, Ci - c0);  // 32, or 16 for the last chunk
    const int nv = kc >> 3;            // 16-byte vectors per entry
    __syncthreads();
    for (int it = tid; it < PR * PW * nv; it += NT) {
      const int v = it % nv, q = it / nv;
      const int px = q % PW, row = q / PW;
      const int yy = y0 + row - 1, xx = x0 + px - 1;
      bf16x8 val = zero;
      if (yy >= 0 && yy < H && xx >= 0 && xx < W)
        val = *reinterpret_cast<const bf16x8*>(a.in.p + tv_at(a.in, n, yy, xx) + c0 + v * 8);
      *reinterpret_cast<bf16x8*>(sin_ + (row * PW + px) * kKP + v * 8) = val;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int dy = t / 3, dx = t % 3;
      for (int ks = 0; ks < kc; ks += 16) {
        const bf16x8 A =
            *reinterpret_cast<const bf16x8*>(a.w + ((long)(co0 + wi * 32 + r) * 9 + t) * Ci + c0 + ks + half * 8);
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const bf16x8 B =
              *reinterpret_cast<const bf16x8*>(sin_ + ((q + dy) * PW + wj * 32 + r + dx) * kKP + ks + half * 8);
          // D = input x weights^T: rows are pixels, columns output channels
          acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(B, A, acc[q], 0, 0, 0);
        }
      }
    }
  }
  // D[row][col]: lane holds col = r (output channel) and rows 8 (v / 4) + 4 half + v % 4
  // (pixels), so each store of a row writes 32 neighbouring channels of one pixel
  const int co = co0 + wi * 32 + r;
  if (co >= a.Co) return;
  const float bias = (a.mode == 0 && a.bias) ? a.bias[co] : 0.0f;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int y = y0 + q;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int x = x0 + wj * 32 + (v >> 2) * 8 + half * 4 + (v & 3);
      float val = acc[q][v];
      if (a.mode == 0) {
        const float z = val + bias;
        if (a.out_z.p) a.out_z.p[tv_at(a.out_z, n, y, x) + co] = f2bf(z);
        a.out.p[tv_at(a.out, n, y, x) + co] = f2bf(silu_f(z));
      } else {
        if (a.zprev.p) val *= silu_grad_f(bf2f(a.zprev.p[tv_at(a.zprev, n, y, x) + co]));
        bf16_t* o = a.out.p + tv_at(a.out, n, y, x) + co;
        if (a.accumulate) val += bf2f(*o);
        *o = f2bf(val);
      }
    }
  }
}

// Weight gradient: part[split][co][t][ci] = sum over this split's pixel chunks of
// gz[pix][co] * x[pix + d_t][ci]. Block = 9 waves (one per tap), tile 32 co x 32 ci.
// A chunk is R image rows of cw pixels (R * cw <= kChunk): its gz pixels and the
// R + 2 x rows around them (cw + 2 pixels wide) are read as 16-byte vectors of 8
// channels and staged transposed in LDS, then every wave runs R * cw / 16 MFMAs
// on them. Requires 16-byte aligned channel vectors (cs, coff, C multiples of 8),
// cw % 16 == 0, W % cw == 0, H % R == 0 and (R + 2) * 32 * (cw + 8) <= kXLds.
constexpr int kChunk = 256;         // pixels per chunk
constexpr int kGP = kChunk + 8;     // gzT row pitch (elements)
constexpr int kXLds = 13824;        // xT elements: (R + 2) * 32 rows of pitch cw + 8
struct WgradArgs {
  TV gz;        // gradient w.r.t. the layer's pre-activation (C = Co)
  TV x;         // layer input (C = Ci)
  float* part;  // [nsplit][Co][9][Ci]
  int nsplit;
  int cw;       // pixels per chunk row
  int R;        // rows per chunk
};

// 8 channels (16 bytes, channel j in bits 16 (j % 2) of word j / 2)
__device__ __forceinline__ u32x4 load_u32x4(const bf16_t* p) { return *reinterpret_cast<const u32x4*>(p); }

__global__ void __launch_bounds__(576) conv3x3_wgrad(WgradArgs a) {
  __shared__ __align__(16) bf16_t gzT[32 * kGP];  // [co][pix]
  __shared__ __align__(16) bf16_t xT[kXLds];      // [row][ci][pix + 1]
  const int lane = threadIdx.x & 63, tap = threadIdx.x >> 6;
  const int r = lane & 31, half = lane >> 5;
  const int ci0 = blockIdx.x * 32, co0 = blockIdx.y * 32, split = blockIdx.z;
  const int H = a.x.H, W = a.x.W, Ci = a.x.C, Co = a.gz.C, cw = a.cw, R = a.R;
  const int XP = cw + 8;
  const int cpr = W / cw, rpi = H / R;
  const long nchunks = (long)a.x.N * rpi * cpr;
  const int dy = tap / 3 - 1, dx = tap % 3 - 1;
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
  for (long ch = split; ch < nchunks; ch += a.nsplit) {
    const int n = (int)(ch / ((long)rpi * cpr));
    const int rem = (int)(ch - (long)n * rpi * cpr);
    const int y0 = (rem / cpr) * R, x0 = (rem - (rem / cpr) * cpr) * cw;
    // gz: R * cw pixels, 4 vectors of 8 channels each
    for (int e = threadIdx.x; e < R * cw * 4; e += 576) {
      const int p = e >> 2, v = e & 3;
      const int py = p / cw, px = p - py * cw;
      u32x4 val = {0u, 0u, 0u, 0u};
      if (co0 + 8 * v < Co) val = load_u32x4(a.gz.p + tv_at(a.gz, n, y0 + py, x0 + px) + co0 + 8 * v);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        gzT[(8 * v + 2 * j) * kGP + p] = (bf16_t)(val[j] & 0xffffu);
        gzT[(8 * v + 2 * j + 1) * kGP + p] = (bf16_t)(val[j] >> 16);
      }
    }
    // x: rows y0 - 1 .. y0 + R, pixels x0 - 1 .. x0 + cw, 4 vectors of 8 channels each
    for (int e = threadIdx.x; e < (R + 2) * (cw + 2) * 4; e += 576) {
      const int v = e & 3, k = e >> 2;
      const int rr = k / (cw + 2), px = k - rr * (cw + 2);
      const int yy = y0 + rr - 1, xx = x0 + px - 1;
      const bool in = yy >= 0 && yy < H && xx >= 0 && xx < W && ci0 + 8 * v < Ci;
      u32x4 val = {0u, 0u, 0u, 0u};
      if (in) val = load_u32x4(a.x.p + tv_at(a.x, n, yy, xx) + ci0 + 8 * v);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        xT[(rr * 32 + 8 * v + 2 * j) * XP + px] = (bf16_t)(val[j] & 0xffffu);
        xT[(rr * 32 + 8 * v + 2 * j + 1) * XP + px] = (bf16_t)(val[j] >> 16);
      }
    }
    __syncthreads();
    if (tap < 9) {
      // B of tap (dy, dx) starts dx + 1 elements past a 16-byte boundary: it is
      // read as two aligned 16-byte words and shifted by whole elements, so
      // every vector LDS read is aligned
      const int sh = dx + 1;
      for (int rr = 0; rr < R; ++rr) {
        const u32x4* ap = reinterpret_cast<const u32x4*>(gzT + r * kGP + rr * cw + half * 8);
        const u32x4* bp = reinterpret_cast<const u32x4*>(xT + ((rr + dy + 1) * 32 + r) * XP + half * 8);
        for (int kk = 0; kk < cw; kk += 16) {
          const u32x4 a4 = ap[kk >> 3];
          const u32x4 w0 = bp[kk >> 3], w1 = bp[(kk >> 3) + 1];
          u32x4 b4 = w0;
          if (sh == 1) {
            b4.x = __builtin_amdgcn_alignbit(w0.y, w0.x, 16);
            b4.y = __builtin_amdgcn_alignbit(w0.z, w0.y, 16);
            b4.z = __builtin_amdgcn_alignbit(w0.w, w0.z, 16);
            b4.w = __builtin_amdgcn_alignbit(w1.x, w0.w, 16);
          } else if (sh == 2) {
            b4.x = w0.y;
            b4.y = w0.z;
            b4.z = w0.w;
            b4.w = w1.x;
          }
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a4), __builtin_bit_cast(bf16x8, b4),
                                                         acc, 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  if (tap < 9) {
    const int ci = ci0 + r;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int co = co0 + (v >> 2) * 8 + half * 4 + (v & 3);
      if (co < Co && ci < Ci) a.part[(((long)split * Co + co) * 9 + tap) * Ci + ci] = acc[v];
    }
  }
}

// out[k] = sum over s of part[s][k]. A block takes 32 outputs; its 8 groups of
// 32 lanes each sum a contiguous eighth of the splits in order, and the eight
// sums are added in group order (fixed order: deterministic).
__global__ void __launch_bounds__(256) reduce_splits(const float* __restrict__ part, int nsplit, long n,
                                                     float* __restrict__ out) {
  __shared__ float red[256];
  const int kl = threadIdx.x & 31, g = threadIdx.x >> 5;
  const long k = blockIdx.x * 32L + kl;
  const int per = (nsplit + 7) / 8;
  const int s0 = min(nsplit, g * per), s1 = min(nsplit, s0 + per);
  float s = 0.0f;
  if (k < n)
    for (int i = s0; i < s1; ++i) s += part[(long)i * n + k];
  red[threadIdx.x] = s;
  __syncthreads();
  if (g == 0 && k < n) {
    float o = 0.0f;
#pragma unroll
    for (int j = 0; j < 8; ++j) o += red[j * 32 + kl];
    out[k] = o;
  }
}

// 8 bf16 channels of a 16-byte vector as floats
__device__ __forceinline__ void unpack8(const u32x4 v, float (&x)[8]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    x[2 * j] = bf2f((bf16_t)(v[j] & 0xffffu));
    x[2 * j + 1] = bf2f((bf16_t)(v[j] >> 16));
  }
}

// Per-block channel sums of an NHWC view (bf16 g, or fp32 gf with channel
// stride gf_cs) into fp32 partials [nblk][C]. Block y takes channels
// [256 y, 256 y + Cc), Cc = min(C - 256 y, 256). For g (Cc % 8 == 0) thread t
// sums the 8-channel group t % G (G = Cc / 8) over the pixels b0 + t / G, step
// 256 / G, of the block's pixel range; for gf, channel t % Cc over the pixels
// b0 + t / Cc, step 256 / Cc. The lane sums of each channel are then added in
// lane order (deterministic).
__global__ void __launch_bounds__(256) channel_sums(TV g, const float* __restrict__ gf, int gf_cs, long npix, int C,
                                                    float* __restrict__ part) {
  __shared__ float red[256 * 8];
  const int t = threadIdx.x;
  const int c0 = 256 * blockIdx.y;
  const int Cc = min(C - c0, 256);
  const long per = (npix + gridDim.x - 1) / gridDim.x;
  const long b0 = blockIdx.x * per, b1 = std::min(npix, b0 + per);
  if (gf) {
    const int L = 256 / Cc;
    const int c = t % Cc, l = t / Cc;
    float s = 0.0f;
    if (l < L)
      for (long p = b0 + l; p < b1; p += L) s += gf[p * gf_cs + c0 + c];
    red[t] = s;
    __syncthreads();
    if (t < Cc) {
      float a = 0.0f;
      for (int k = 0; k < L; ++k) a += red[k * Cc + t];
      part[(long)blockIdx.x * C + c0 + t] = a;
    }
    return;
  }
  const int G = Cc / 8, L = 256 / G;
  const int e = t % G, l = t / G;
  float s[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  if (l < L)
    for (long p = b0 + l; p < b1; p += L) {
      float v[8];
      unpack8(load_u32x4(g.p + p * g.cs + g.coff + c0 + 8 * e), v);
#pragma unroll
      for (int j = 0; j < 8; ++j) s[j] += v[j];
    }
#pragma unroll
  for (int j = 0; j < 8; ++j) red[t * 8 + j] = s[j];
  __syncthreads();
  if (t < Cc) {
    float a = 0.0f;
    for (int k = 0; k < L; ++k) a += red[(k * G + t / 8) * 8 + t % 8];
    part[(long)blockIdx.x * C + c0 + t] = a;
  }
}

// Pooling, upsampling and SiLU' on NHWC views, one 16-byte vector of 8
// channels per work item (C, cs and coff multiples of 8); item k is channel
// group k % (C / 8) of pixel k / (C / 8).
__device__ __forceinline__ u32x4 pack8(const float (&x)[8]) {
  u32x4 r;
#pragma unroll
  for (int j = 0; j < 4; ++j) r[j] = (unsigned)f2bf(x[2 * j]) | ((unsigned)f2bf(x[2 * j + 1]) << 16);
  return r;
}

__device__ __forceinline__ void store_u32x4(bf16_t* p, const u32x4 v) { *reinterpret_cast<u32x4*>(p) = v; }

// pixel (b, y, x) and first channel c of work item k of a view with C8 groups per pixel
__device__ __forceinline__ void item_of(long k, const TV& t, int C8, int& b, int& y, int& x, int& c) {
  c = 8 * (int)(k % C8);
  long p = k / C8;
  x = (int)(p % t.W);
  p /= t.W;
  y = (int)(p % t.H);
  b = (int)(p / t.H);
}

__global__ void avgpool2_fwd(TV in, TV out) {
  const int C8 = out.C / 8;
  const long n = (long)out.N * out.H * out.W * C8;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    int b, y, x, c;
    item_of(k, out, C8, b, y, x, c);
    float s[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    for (int j = 0; j < 2; ++j)
      for (int i = 0; i < 2; ++i) {
        float v[8];
        unpack8(load_u32x4(in.p + tv_at(in, b, 2 * y + j, 2 * x + i) + c), v);
#pragma unroll
        for (int e = 0; e < 8; ++e) s[e] += v[e];
      }
#pragma unroll
    for (int e = 0; e < 8; ++e) s[e] *= 0.25f;
    store_u32x4(out.p + tv_at(out, b, y, x) + c, pack8(s));
  }
}

// gin (+)= gout / 4 spread over each 2x2 block
__global__ void avgpool2_bwd(TV gout, TV gin, int accumulate) {
  const int C8 = gin.C / 8;
  const long n = (long)gin.N * gin.H * gin.W * C8;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    int b, y, x, c;
    item_of(k, gin, C8, b, y, x, c);
    float v[8];
    unpack8(load_u32x4(gout.p + tv_at(gout, b, y >> 1, x >> 1) + c), v);
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] *= 0.25f;
    bf16_t* o = gin.p + tv_at(gin, b, y, x) + c;
    if (accumulate) {
      float w[8];
      unpack8(load_u32x4(o), w);
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] += w[e];
    }
    store_u32x4(o, pack8(v));
  }
}

__global__ void upsample2_fwd(TV in, TV out) {
  const int C8 = out.C / 8;
  const long n = (long)out.N * out.H * out.W * C8;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    int b, y, x, c;
    item_of(k, out, C8, b, y, x, c);
    store_u32x4(out.p + tv_at(out, b, y, x) + c, load_u32x4(in.p + tv_at(in, b, y >> 1, x >> 1) + c));
  }
}

// gin = sum of gout over each 2x2 block
__global__ void upsample2_bwd(TV gout, TV gin) {
  const int C8 = gin.C / 8;
  const long n = (long)gin.N * gin.H * gin.W * C8;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    int b, y, x, c;
    item_of(k, gin, C8, b, y, x, c);
    float s[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    for (int j = 0; j < 2; ++j)
      for (int i = 0; i < 2; ++i) {
        float v[8];
        unpack8(load_u32x4(gout.p + tv_at(gout, b, 2 * y + j, 2 * x + i) + c), v);
#pragma unroll
        for (int e = 0; e < 8; ++e) s[e] += v[e];
      }
    store_u32x4(gin.p + tv_at(gin, b, y, x) + c, pack8(s));
  }
}

// g *= SiLU'(z) in place
__global__ void silu_bwd_inplace(TV g, TV z) {
  const int C8 = g.C / 8;
  const long n = (long)g.N * g.H * g.W * C8;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    const int c = 8 * (int)(k % C8);
    const long p = k / C8;
    bf16_t* o = g.p + p * g.cs + g.coff + c;
    float v[8], zz[8];
    unpack8(load_u32x4(o), v);
    unpack8(load_u32x4(z.p + p * z.cs + z.coff + c), zz);
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] *= silu_grad_f(zz[e]);
    store_u32x4(o, pack8(v));
  }
}

// The 1x1 head (cout <= 8 outputs, C % 8 == 0 input channels): one pixel per
// thread, channels moved as 16-byte vectors of 8 (load_u32x4).

// head: out[pix][o] = b[o] + sum_ci w[o][ci] a[pix][ci] (fp32 out, ci ascending)
__global__ void __launch_bounds__(256) head_fwd(TV a, const float* __restrict__ w, const float* __restrict__ b,
                                                int cout, float* __restrict__ out, long npix) {
  const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (p >= npix) return;
  const bf16_t* ap = a.p + p * a.cs + a.coff;
  float s[8];
#pragma unroll
  for (int o = 0; o < 8; ++o) s[o] = o < cout ? b[o] : 0.0f;
  for (int c0 = 0; c0 < a.C; c0 += 8) {
    float x[8];
    unpack8(load_u32x4(ap + c0), x);
#pragma unroll
    for (int o = 0; o < 8; ++o)
      if (o < cout) {
#pragma unroll
        for (int j = 0; j < 8; ++j) s[o] += w[o * a.C + c0 + j] * x[j];
      }
  }
  for (int o = 0; o < cout; ++o) out[p * cout + o] = s[o];
}

// head backward to its input, times SiLU'(z): ga[pix][ci] = SiLU'(z) sum_o gout[pix][o] w[o][ci]
__global__ void __launch_bounds__(256) head_bwd_data(const float* __restrict__ gout, const float* __restrict__ w,
                                                     int cout, TV z, TV ga, long npix) {
  const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (p >= npix) return;
  float g[8];
#pragma unroll
  for (int o = 0; o < 8; ++o) g[o] = o < cout ? gout[p * cout + o] : 0.0f;
  const bf16_t* zp = z.p + p * z.cs + z.coff;
  bf16_t* gp = ga.p + p * ga.cs + ga.coff;
  const int C = ga.C;
  for (int c0 = 0; c0 < C; c0 += 8) {
    float zz[8];
    unpack8(load_u32x4(zp + c0), zz);
    u32x4 res;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float lo = 0.0f, hi = 0.0f;
#pragma unroll
      for (int o = 0; o < 8; ++o)
        if (o < cout) {
          lo += g[o] * w[o * C + c0 + 2 * j];
          hi += g[o] * w[o * C + c0 + 2 * j + 1];
        }
      lo *= silu_grad_f(zz[2 * j]);
      hi *= silu_grad_f(zz[2 * j + 1]);
      res[j] = (unsigned)f2bf(lo) | ((unsigned)f2bf(hi) << 16);
    }
    *reinterpret_cast<u32x4*>(gp + c0) = res;
  }
}

// Per-block partials of gw[o][ci] = sum_pix gout[pix][o] a[pix][ci] ([nblk][cout * C],
// cout * C <= 256). Thread t takes the entries (o, 8 channels) e = t % E, E = cout * C / 8,
// over the pixels b0 + t / E, step L = 256 / E, of the block's range; the L lane sums of
// each entry are then added in lane order (deterministic).
__global__ void __launch_bounds__(256) head_wgrad(const float* __restrict__ gout, TV a, int cout, long npix,
                                                  float* __restrict__ part) {
  __shared__ float red[256 * 8];
  const int t = threadIdx.x;
  const int C = a.C, C8 = C / 8, E = cout * C8, L = 256 / E, K = cout * C;
  const int e = t % E, l = t / E;
  const int o = e / C8, c0 = (e - o * C8) * 8;
  const long per = (npix + gridDim.x - 1) / gridDim.x;
  const long b0 = blockIdx.x * per, b1 = std::min(npix, b0 + per);
  float s[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) s[j] = 0.0f;
  if (l < L)
    for (long p = b0 + l; p < b1; p += L) {
      const float g = gout[p * cout + o];
      float x[8];
      unpack8(load_u32x4(a.p + p * a.cs + a.coff + c0), x);
#pragma unroll
      for (int j = 0; j < 8; ++j) s[j] += g * x[j];
    }
#pragma unroll
  for (int j = 0; j < 8; ++j) red[t * 8 + j] = s[j];
  __syncthreads();
  if (t < K) {
    const int oo = t / C, c = t - oo * C;
    const int ee = oo * C8 + c / 8, jj = c % 8;
    float acc = 0.0f;
    for (int q = 0; q < L; ++q) acc += red[(q * E + ee) * 8 + jj];
    part[(long)blockIdx.x * K + t] = acc;
  }
}

// mse: per-block partial sums of (out - t)^2 and gout = 2 (out - t) / count
__global__ void __launch_bounds__(256) mse_fwd_bwd(const float* __restrict__ out, const float* __restrict__ tgt, long n,
                                                   float* __restrict__ gout, double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  const float inv = 2.0f / (float)n;
  for (long k = blockIdx.x * 256L + threadIdx.x; k < n; k += (long)gridDim.x * 256L) {
    const float d = out[k] - tgt[k];
    s += (double)d * d;
    gout[k] = inv * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// gradient clipping by global L2 norm: per-block partial sums of g^2 (FP64,
// grid-stride ranges, tree order), then scale = min(1, max_norm / |g|)
__global__ void __launch_bounds__(256) grad_sq_partials(const float* __restrict__ g, long n,
                                                        double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  for (long k = blockIdx.x * 256L + threadIdx.x; k < n; k += (long)gridDim.x * 256L) s += (double)g[k] * g[k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) grad_clip_scale(const double* __restrict__ part, int nblk, float max_norm,
                                                       float* __restrict__ scale) {
  __shared__ double red[256];
  double s = 0.0;
  for (int k = threadIdx.x; k < nblk; k += 256) s += part[k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double norm = sqrt(red[0]);
    *scale = norm > (double)max_norm ? (float)((double)max_norm / norm) : 1.0f;
  }
}

// Adam (Kingma and Ba 2015) with bias correction on the gradient times *gscale
// (gscale nullable: 1); grads g, moments m, v, master p (fp32)
__global__ void adam_update(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, const float* __restrict__ gscale, long n, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
  const float sc = gscale ? *gscale : 1.0f;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    const float gk = g[k] * sc;
    const float mk = b1 * m[k] + (1.0f - b1) * gk;
    const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
  }
}

// bf16 copies of a 3x3 layer: wf[co][t][ci] (rows padded to 32) and the
// backward-data weights wb[ci][t][co] = w[co][8 - t][ci] (rows padded to 32)
__global__ void pack_conv_weights(const float* __restrict__ w, int Co, int Ci, bf16_t* __restrict__ wf,
                                  bf16_t* __restrict__ wb) {
  const long n = (long)Co * 9 * Ci;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    const int ci = (int)(k % Ci);
    const long q = k / Ci;
    const int t = (int)(q % 9), co = (int)(q / 9);
    const bf16_t b = f2bf(w[k]);
    wf[k] = b;
    if (wb) wb[((long)ci * 9 + (8 - t)) * Co + co] = b;
  }
}

}  // namespace ssn

// ================================================================ host side

using namespace ssn;

namespace {

thread_local std::string g_ssn_err;

int nfail(int code, const std::string& m) {
  g_ssn_err = m;
  return code;
}

#define SN_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) return nfail(SS_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

long rup(long x, long m) { return (x + m - 1) / m * m; }

struct HT {  // host handle of one NHWC bf16 buffer (capacity Ncap)
  bf16_t* p = nullptr;
  int H = 0, W = 0, cs = 0;
  TV view(int n, int coff, int C) const {
    TV t;
    t.p = p;
    t.N = n;
    t.H = H;
    t.W = W;
    t.cs = cs;
    t.coff = coff;
    t.C = C;
    return t;
  }
  TV all(int n) const { return view(n, 0, cs); }
};

struct ConvL {
  int Ci, Ci_real, Co, H, W;
  long w_off, b_off;  // float offsets into the flat parameter arrays
  bf16_t* wf;         // [rup(Co, 32)][9][Ci]
  bf16_t* wb;         // [rup(Ci, 32)][9][Co]
};

constexpr int kPartBlocks = 256;
constexpr long kWgradPartFloats = 1024L * 9 * 1024;

}  // namespace

struct ssn_net {
  int levels, base, cin, cout, cin_pad, Ncap, H, W, L;
  // forward pass captured as a HIP graph for one (x, nb, out) triple
  hipGraphExec_t fgraph = nullptr;
  hipStream_t fcap = nullptr;
  const float* fx = nullptr;
  float* fout = nullptr;
  int fnb = 0;
  int conv_shape;  // 0: by problem size, 1: large direct blocks, 2: small direct blocks, 3: LDS-tiled
  hipStream_t stream;
  float *P, *G, *M, *V;
  long np;
  std::vector<ConvL> conv;  // enc0a enc0b ... mid.a mid.b dec(L-1)a dec(L-1)b ... dec0a dec0b
  long hw_off, hb_off;
  std::vector<int> ch;      // channels per level
  // activations
  HT X0;
  std::vector<HT> ZA, AA, ZB, CAT, Pin;  // Pin[l]: pooled input of level l (l >= 1), Pin[L]: bottleneck input
  HT ZMa, AMa, ZMb, AMb;
  std::vector<HT> ZDa, ADa, ZDb, ADb;
  // gradients
  std::vector<HT> gCAT, gT1, gT2, gT3, gP;  // gT3[l]: gradient at the pre-activation of dec_a(l)
  HT gM1, gM2;
  float *OUT, *GOUT, *part, *cpart;
  double* lpart;
  double* npart;   // per-block partial sums of the squared gradient
  float* gscale;   // gradient scale of the clipped Adam step (device)
  float clip = 0.0f;  // global L2 clipping norm of the Adam step (0: off)
  int adam_t;
  size_t bytes;
};

namespace {

// Carve (or, with base == nullptr, size) the workspace of a network.
size_t net_carve(ssn_net* n, char* base) {
  size_t off = 0;
  auto take = [&](size_t b) -> char* {
    char* p = base ? base + off : nullptr;
    off += (size_t)rup((long)b, 256);
    return p;
  };
  const int L = n->L, N = n->Ncap;
  auto tensor = [&](HT& t, int H, int W, int cs) {
    t.H = H;
    t.W = W;
    t.cs = cs;
    t.p = (bf16_t*)take((size_t)N * H * W * cs * 2);
  };
  n->P = (float*)take(n->np * 4);
  n->G = (float*)take(n->np * 4);
  n->M = (float*)take(n->np * 4);
  n->V = (float*)take(n->np * 4);
  for (ConvL& c : n->conv) {
    c.wf = (bf16_t*)take((size_t)rup(c.Co, 32) * 9 * c.Ci * 2);
    c.wb = (bf16_t*)take((size_t)rup(c.Ci, 32) * 9 * c.Co * 2);
  }
  tensor(n->X0, n->H, n->W, n->cin_pad);
  n->ZA.assign(L, HT()); n->AA.assign(L, HT()); n->ZB.assign(L, HT()); n->CAT.assign(L, HT());
  n->Pin.assign(L + 1, HT());
  n->ZDa.assign(L, HT()); n->ADa.assign(L, HT()); n->ZDb.assign(L, HT()); n->ADb.assign(L, HT());
  n->gCAT.assign(L, HT()); n->gT1.assign(L, HT()); n->gT2.assign(L, HT()); n->gT3.assign(L, HT());
  n->gP.assign(L + 1, HT());
  for (int l = 0; l < L; ++l) {
    const int H = n->H >> l, W = n->W >> l, c = n->ch[l], cn = n->ch[l + 1];
    tensor(n->ZA[l], H, W, c); tensor(n->AA[l], H, W, c); tensor(n->ZB[l], H, W, c);
    tensor(n->CAT[l], H, W, cn + c);
    tensor(n->ZDa[l], H, W, c); tensor(n->ADa[l], H, W, c); tensor(n->ZDb[l], H, W, c); tensor(n->ADb[l], H, W, c);
    tensor(n->gCAT[l], H, W, cn + c); tensor(n->gT1[l], H, W, c); tensor(n->gT2[l], H, W, c);
    tensor(n->gT3[l], H, W, c);
    if (l >= 1) {
      tensor(n->Pin[l], H, W, n->ch[l - 1]);
      tensor(n->gP[l], H, W, n->ch[l - 1]);
    }
  }
  const int HL = n->H >> L, WL = n->W >> L, cL = n->ch[L];
  tensor(n->Pin[L], HL, WL, n->ch[L - 1]);
  tensor(n->gP[L], HL, WL, n->ch[L - 1]);
  tensor(n->ZMa, HL, WL, cL); tensor(n->AMa, HL, WL, cL); tensor(n->ZMb, HL, WL, cL); tensor(n->AMb, HL, WL, cL);
  tensor(n->gM1, HL, WL, cL); tensor(n->gM2, HL, WL, cL);
  n->OUT = (float*)take((size_t)N * n->H * n->W * n->cout * 4);
  n->GOUT = (float*)take((size_t)N * n->H * n->W * n->cout * 4);
  n->part = (float*)take(kWgradPartFloats * 4);
  n->cpart = (float*)take((size_t)kPartBlocks * 1024 * 4);
  n->lpart = (double*)take(256 * 8);
  n->npart = (double*)take(kPartBlocks * 8);
  n->gscale = (float*)take(256);
  return off;
}

// Layer table and parameter offsets (oracle order; layer 0 input padded to 16).
void net_layers(ssn_net* n) {
  n->L = n->levels - 1;
  n->ch.clear();
  for (int l = 0; l < n->levels; ++l) n->ch.push_back(n->base << l);
  n->conv.clear();
  long off = 0;
  auto add = [&](int Ci_real, int Ci, int Co, int H, int W) {
    ConvL c;
    c.Ci = Ci; c.Ci_real = Ci_real; c.Co = Co; c.H = H; c.W = W;
    c.w_off = off; off += (long)Co * 9 * Ci;
    c.b_off = off; off += Co;
    c.wf = c.wb = nullptr;
    n->conv.push_back(c);
  };
  int cprev = n->cin;
  for (int l = 0; l < n->L; ++l) {
    const int H = n->H >> l, W = n->W >> l;
    add(cprev, l == 0 ? n->cin_pad : cprev, n->ch[l], H, W);
    add(n->ch[l], n->ch[l], n->ch[l], H, W);
    cprev = n->ch[l];
  }
  add(cprev, cprev, n->ch[n->L], n->H >> n->L, n->W >> n->L);
  add(n->ch[n->L], n->ch[n->L], n->ch[n->L], n->H >> n->L, n->W >> n->L);
  cprev = n->ch[n->L];
  for (int l = n->L - 1; l >= 0; --l) {
    const int H = n->H >> l, W = n->W >> l;
    add(cprev + n->ch[l], cprev + n->ch[l], n->ch[l], H, W);
    add(n->ch[l], n->ch[l], n->ch[l], H, W);
    cprev = n->ch[l];
  }
  n->hw_off = off; off += (long)n->cout * n->ch[0];
  n->hb_off = off; off += n->cout;
  n->np = off;
}

int enc_a(int l) { return 2 * l; }
int enc_b(int l) { return 2 * l + 1; }
int mid_a(const ssn_net* n) { return 2 * n->L; }
int mid_b(const ssn_net* n) { return 2 * n->L + 1; }
int dec_a(const ssn_net* n, int l) { return 2 * n->L + 2 + 2 * (n->L - 1 - l); }
int dec_b(const ssn_net* n, int l) { return dec_a(n, l) + 1; }

int grid1(long n) { return (int)std::min<long>((n + 255) / 256, 65535); }

template <int WCO, int WPX, int R>
void launch_tiled(const ssn_net* n, const ConvArgs& ca, int Co) {
  const TV& in = ca.in;
  dim3 grid((unsigned)((long)in.N * (in.H / R) * (in.W / (32 * WPX))), (unsigned)((Co + 32 * WCO - 1) / (32 * WCO)));
  hipLaunchKernelGGL((conv3x3_tiled<WCO, WPX, R>), grid, dim3(64 * WCO * WPX), 0, n->stream, ca);
}

// Launch shapes: the LDS-tiled GEMM where rows are at least 32 pixels wide and
// the grid has at least 256 workgroups (2 rows per workgroup on rows of 128 or
// more pixels, 4 on narrower ones); otherwise direct-operand blocks of 4 waves
// with 64 pixels per wave (large grids) or of one wave with 32 pixels (few
// images, deep levels: 8x more workgroups).
void launch_conv(const ssn_net* n, const ConvArgs& ca, long P, int Co) {
  const unsigned gy = (unsigned)((Co + 31) / 32);
  const int W = ca.in.W, H = ca.in.H;
  const int wpx = W >= 128 ? 4 : W >= 64 ? 2 : 1;
  const int wco = Co % 64 == 0 ? 2 : 1;
  const int R = wpx == 4 ? 2 : 4;
  const long tiled_blocks =
      (long)ca.in.N * (H / R) * (W / (32 * wpx)) * ((Co + 32 * wco - 1) / (32 * wco));
  const bool tiled_ok = W >= 32 && W % (32 * wpx) == 0 && H % R == 0;
  const bool tiled = tiled_ok && (n->conv_shape == 3 || (n->conv_shape == 0 && tiled_blocks >= 256));
  if (tiled) {
    if (wco == 2) {
      if (wpx == 4) launch_tiled<2, 4, 2>(n, ca, Co);
      else if (wpx == 2) launch_tiled<2, 2, 4>(n, ca, Co);
      else launch_tiled<2, 1, 4>(n, ca, Co);
    } else {
      if (wpx == 4) launch_tiled<1, 4, 2>(n, ca, Co);
      else if (wpx == 2) launch_tiled<1, 2, 4>(n, ca, Co);
      else launch_tiled<1, 1, 4>(n, ca, Co);
    }
    return;
  }
  const bool large = n->conv_shape == 1 || (n->conv_shape != 2 && (P + 255) / 256 * gy >= 1024);
  if (large) {
    dim3 grid((unsigned)((P + 255) / 256), gy);
    hipLaunchKernelGGL((conv3x3_mfma<2, 4>), grid, dim3(256), 0, n->stream, ca);
  } else {
    dim3 grid((unsigned)((P + 31) / 32), gy);
    hipLaunchKernelGGL((conv3x3_mfma<1, 1>), grid, dim3(64), 0, n->stream, ca);
  }
}

void launch_conv_fwd(const ssn_net* n, const ConvL& c, TV in, TV z, TV a) {
  ConvArgs ca;
  ca.in = in;
  ca.w = c.wf;
  ca.bias = n->P + c.b_off;
  ca.Co = c.Co;
  ca.out_z = z;
  ca.out = a;
  ca.zprev.p = nullptr;
  ca.mode = 0;
  ca.accumulate = 0;
  launch_conv(n, ca, (long)in.N * in.H * in.W, c.Co);
}

// gradient w.r.t. the layer input: out = conv(gz, wb) [* SiLU'(zprev)]
void launch_conv_bwd_data(const ssn_net* n, const ConvL& c, TV gz, TV out, const TV* zprev) {
  ConvArgs ca;
  ca.in = gz;
  ca.w = c.wb;
  ca.bias = nullptr;
  ca.Co = c.Ci;
  ca.out_z.p = nullptr;
  ca.out = out;
  if (zprev) ca.zprev = *zprev;
  else ca.zprev.p = nullptr;
  ca.mode = 1;
  ca.accumulate = 0;
  launch_conv(n, ca, (long)gz.N * gz.H * gz.W, c.Ci);
}

// out[k] = sum over s < nsplit of part[s][k], k < nout
void launch_reduce_splits(const ssn_net* n, const float* part, int nsplit, long nout, float* out) {
  hipLaunchKernelGGL(reduce_splits, dim3((unsigned)((nout + 31) / 32)), dim3(256), 0, n->stream, part, nsplit, nout,
                     out);
}

// Chunk geometry of the weight gradient for a W x H level: cw is the widest
// multiple of 16 up to 64 that divides W; R the largest power of two with
// R * cw <= kChunk, H % R == 0 and the x rows within kXLds.
void wgrad_chunk(int W, int H, int& cw, int& R) {
  cw = 16;
  for (int c = 64; c >= 16; c -= 16)
    if (W % c == 0) {
      cw = c;
      break;
    }
  R = 1;
  while (2 * R * cw <= kChunk && H % (2 * R) == 0 && (2 * R + 2) * 32 * (cw + 8) <= kXLds) R *= 2;
}

void launch_wgrad(ssn_net* n, const ConvL& c, TV gz, TV x) {
  int cw = 16, R = 1;
  wgrad_chunk(x.W, x.H, cw, R);
  const long nchunks = (long)x.N * (x.H / R) * (x.W / cw);
  const int tci = (c.Ci + 31) / 32, tco = (c.Co + 31) / 32;
  // about 1.5 workgroups per CU (measured: 256 and 768 were 1-3% slower overall)
  int nsplit = (int)std::max<long>(1, std::min<long>(nchunks, 384 / (tci * tco)));
  while ((long)nsplit * c.Co * 9 * c.Ci > kWgradPartFloats) nsplit /= 2;
  WgradArgs wa;
  wa.gz = gz;
  wa.x = x;
  wa.part = n->part;
  wa.nsplit = nsplit;
  wa.cw = cw;
  wa.R = R;
  hipLaunchKernelGGL(conv3x3_wgrad, dim3(tci, tco, nsplit), dim3(576), 0, n->stream, wa);
  const long nw = (long)c.Co * 9 * c.Ci;
  launch_reduce_splits(n, n->part, nsplit, nw, n->G + c.w_off);
  // bias gradient: per-channel sums of gz
  hipLaunchKernelGGL(channel_sums, dim3(kPartBlocks, (c.Co + 255) / 256), dim3(256), 0, n->stream, gz,
                     (const float*)nullptr, 0, (long)gz.N * gz.H * gz.W, c.Co, n->cpart);
  launch_reduce_splits(n, n->cpart, kPartBlocks, (long)c.Co, n->G + c.b_off);
}

void pack_all(ssn_net* n) {
  for (const ConvL& c : n->conv) {
    const long nw = (long)c.Co * 9 * c.Ci;
    hipLaunchKernelGGL(pack_conv_weights, dim3(grid1(nw)), dim3(256), 0, n->stream, n->P + c.w_off, c.Co, c.Ci, c.wf,
                       c.wb);
  }
}

__global__ void copy_f32(const float* __restrict__ src, float* __restrict__ dst, long n) {
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) dst[k] = src[k];
}

__global__ void input_to_bf16(const float* __restrict__ x, int cin, long npix, TV X) {
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < npix * X.C; k += (long)gridDim.x * blockDim.x) {
    const long p = k / X.C;
    const int c = (int)(k - p * X.C);
    X.p[p * X.cs + X.coff + c] = f2bf(c < cin ? x[p * cin + c] : 0.0f);
  }
}

int net_forward(ssn_net* n, const float* x, int nb) {
  const int L = n->L;
  const long npix = (long)nb * n->H * n->W;
  hipLaunchKernelGGL(input_to_bf16, dim3(grid1(npix * n->cin_pad)), dim3(256), 0, n->stream, x, n->cin, npix,
                     n->X0.all(nb));
  for (int l = 0; l < L; ++l) {
    const int c = n->ch[l], cn = n->ch[l + 1];
    TV in = l == 0 ? n->X0.all(nb) : n->Pin[l].all(nb);
    launch_conv_fwd(n, n->conv[enc_a(l)], in, n->ZA[l].all(nb), n->AA[l].all(nb));
    TV skip = n->CAT[l].view(nb, cn, c);
    launch_conv_fwd(n, n->conv[enc_b(l)], n->AA[l].all(nb), n->ZB[l].all(nb), skip);
    TV pooled = n->Pin[l + 1].all(nb);
    hipLaunchKernelGGL(avgpool2_fwd, dim3(grid1((long)nb * pooled.H * pooled.W * c / 8)), dim3(256), 0, n->stream, skip,
                       pooled);
  }
  launch_conv_fwd(n, n->conv[mid_a(n)], n->Pin[L].all(nb), n->ZMa.all(nb), n->AMa.all(nb));
  launch_conv_fwd(n, n->conv[mid_b(n)], n->AMa.all(nb), n->ZMb.all(nb), n->AMb.all(nb));
  for (int l = L - 1; l >= 0; --l) {
    const int cn = n->ch[l + 1];
    TV prev = l == L - 1 ? n->AMb.all(nb) : n->ADb[l + 1].all(nb);
    TV up = n->CAT[l].view(nb, 0, cn);
    hipLaunchKernelGGL(upsample2_fwd, dim3(grid1((long)nb * up.H * up.W * cn / 8)), dim3(256), 0, n->stream, prev, up);
    launch_conv_fwd(n, n->conv[dec_a(n, l)], n->CAT[l].all(nb), n->ZDa[l].all(nb), n->ADa[l].all(nb));
    launch_conv_fwd(n, n->conv[dec_b(n, l)], n->ADa[l].all(nb), n->ZDb[l].all(nb), n->ADb[l].all(nb));
  }
  hipLaunchKernelGGL(head_fwd, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, n->stream, n->ADb[0].all(nb),
                     n->P + n->hw_off, n->P + n->hb_off, n->cout, n->OUT, npix);
  SN_HIP(hipGetLastError());
  return SS_OK;
}

int net_backward(ssn_net* n, const float* target, int nb, double* loss) {
  const int L = n->L;
  const long npix = (long)nb * n->H * n->W;
  const long nout = npix * n->cout;
  hipLaunchKernelGGL(mse_fwd_bwd, dim3(256), dim3(256), 0, n->stream, n->OUT, target, nout, n->GOUT, n->lpart);
  // head
  hipLaunchKernelGGL(head_wgrad, dim3(kPartBlocks), dim3(256), 0, n->stream, n->GOUT, n->ADb[0].all(nb), n->cout, npix,
                     n->cpart);
  launch_reduce_splits(n, n->cpart, kPartBlocks, (long)n->cout * n->ch[0], n->G + n->hw_off);
  TV none;
  none.p = nullptr;
  hipLaunchKernelGGL(channel_sums, dim3(kPartBlocks), dim3(256), 0, n->stream, none, n->GOUT, n->cout, npix, n->cout,
                     n->cpart);
  launch_reduce_splits(n, n->cpart, kPartBlocks, (long)n->cout, n->G + n->hb_off);
  hipLaunchKernelGGL(head_bwd_data, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, n->stream, n->GOUT,
                     n->P + n->hw_off, n->cout, n->ZDb[0].all(nb), n->gT1[0].all(nb), npix);
  // decoder, top level first
  for (int l = 0; l < L; ++l) {
    const int cn = n->ch[l + 1];
    const ConvL& cb = n->conv[dec_b(n, l)];
    const ConvL& ca = n->conv[dec_a(n, l)];
    launch_wgrad(n, cb, n->gT1[l].all(nb), n->ADa[l].all(nb));
    TV za = n->ZDa[l].all(nb);
    launch_conv_bwd_data(n, cb, n->gT1[l].all(nb), n->gT3[l].all(nb), &za);
    launch_wgrad(n, ca, n->gT3[l].all(nb), n->CAT[l].all(nb));
    launch_conv_bwd_data(n, ca, n->gT3[l].all(nb), n->gCAT[l].all(nb), nullptr);
    // the upsampled half of the concatenation feeds back to the level below
    TV gup = n->gCAT[l].view(nb, 0, cn);
    TV dst = l == L - 1 ? n->gM2.all(nb) : n->gT1[l + 1].all(nb);
    TV zsrc = l == L - 1 ? n->ZMb.all(nb) : n->ZDb[l + 1].all(nb);
    hipLaunchKernelGGL(upsample2_bwd, dim3(grid1((long)nb * dst.H * dst.W * cn / 8)), dim3(256), 0, n->stream, gup, dst);
    hipLaunchKernelGGL(silu_bwd_inplace, dim3(grid1((long)nb * dst.H * dst.W * cn / 8)), dim3(256), 0, n->stream, dst,
                       zsrc);
  }
  // bottleneck
  {
    const ConvL& cb = n->conv[mid_b(n)];
    const ConvL& ca = n->conv[mid_a(n)];
    launch_wgrad(n, cb, n->gM2.all(nb), n->AMa.all(nb));
    TV za = n->ZMa.all(nb);
    launch_conv_bwd_data(n, cb, n->gM2.all(nb), n->gM1.all(nb), &za);
    launch_wgrad(n, ca, n->gM1.all(nb), n->Pin[L].all(nb));
    launch_conv_bwd_data(n, ca, n->gM1.all(nb), n->gP[L].all(nb), nullptr);
  }
  // encoder, bottom level first
  for (int l = L - 1; l >= 0; --l) {
    const int c = n->ch[l], cn = n->ch[l + 1];
    TV gS = n->gCAT[l].view(nb, cn, c);
    hipLaunchKernelGGL(avgpool2_bwd, dim3(grid1((long)nb * gS.H * gS.W * c / 8)), dim3(256), 0, n->stream,
                       n->gP[l + 1].all(nb), gS, 1);
    hipLaunchKernelGGL(silu_bwd_inplace, dim3(grid1((long)nb * gS.H * gS.W * c / 8)), dim3(256), 0, n->stream, gS,
                       n->ZB[l].all(nb));
    const ConvL& cb = n->conv[enc_b(l)];
    const ConvL& ca = n->conv[enc_a(l)];
    launch_wgrad(n, cb, gS, n->AA[l].all(nb));
    TV za = n->ZA[l].all(nb);
    launch_conv_bwd_data(n, cb, gS, n->gT2[l].all(nb), &za);
    TV in = l == 0 ? n->X0.all(nb) : n->Pin[l].all(nb);
    launch_wgrad(n, ca, n->gT2[l].all(nb), in);
    if (l > 0) launch_conv_bwd_data(n, ca, n->gT2[l].all(nb), n->gP[l].all(nb), nullptr);
  }
  SN_HIP(hipGetLastError());
  if (loss) {
    double parts[256];
    SN_HIP(hipMemcpyAsync(parts, n->lpart, sizeof(parts), hipMemcpyDeviceToHost, n->stream));
    SN_HIP(hipStreamSynchronize(n->stream));
    double s = 0.0;
    for (int k = 0; k < 256; ++k) s += parts[k];
    *loss = s / (double)nout;
  }
  return SS_OK;
}

// oracle-order flat index <-> padded layout, for one parameter block
template <class F>
void for_each_param(const ssn_net* n, F&& f) {
  long o = 0;  // oracle offset
  for (const ConvL& c : n->conv) {
    for (int co = 0; co < c.Co; ++co)
      for (int t = 0; t < 9; ++t)
        for (int ci = 0; ci < c.Ci_real; ++ci) f(o++, c.w_off + ((long)co * 9 + t) * c.Ci + ci);
    for (int co = 0; co < c.Co; ++co) f(o++, c.b_off + co);
  }
  for (int k = 0; k < n->cout * n->ch[0]; ++k) f(o++, n->hw_off + k);
  for (int k = 0; k < n->cout; ++k) f(o++, n->hb_off + k);
}

long oracle_count(const ssn_net* n) {
  long c = 0;
  for_each_param(n, [&](long, long) { ++c; });
  return c;
}

int check_shape(int levels, int base, int cin, int cout, int N, int H, int W) {
  if (levels < 2 || levels > 6) return nfail(SS_EINVAL, "levels must lie in [2, 6]");
  if (base < 16 || base % 16 || (base << (levels - 1)) > 1024) return nfail(SS_EINVAL, "base must be a multiple of 16");
  if (cin < 1 || cin > 16) return nfail(SS_EINVAL, "cin must lie in [1, 16]");
  if (cout < 1 || cout > 8 || cout * base > 256) return nfail(SS_EINVAL, "cout must lie in [1, 8] with cout*base <= 256");
  const int m = 16 << (levels - 1);
  if (N < 1 || H < m || W < m || H % m || W % m)
    return nfail(SS_ESHAPE, "H and W must be multiples of 16 * 2^(levels-1)");
  return SS_OK;
}

}  // namespace

namespace ss_detail {
int ctx_shape(const ss_ctx* c, int* Nx, int* Ny, int* theory);
}

extern "C" {

long ssn_param_count(int levels, int base, int cin, int cout) {
  ssn_net n;
  n.levels = levels; n.base = base; n.cin = cin; n.cout = cout; n.cin_pad = 16;
  n.H = n.W = 16 << (levels - 1);
  net_layers(&n);
  return oracle_count(&n);
}

int ssn_workspace_bytes(int levels, int base, int cin, int cout, int N, int H, int W, size_t* bytes) {
  int rc = check_shape(levels, base, cin, cout, N, H, W);
  if (rc) return rc;
  if (!bytes) return nfail(SS_EINVAL, "bytes is NULL");
  ssn_net n;
  n.levels = levels; n.base = base; n.cin = cin; n.cout = cout; n.cin_pad = 16;
  n.Ncap = N; n.H = H; n.W = W;
  net_layers(&n);
  *bytes = net_carve(&n, nullptr);
  return SS_OK;
}

int ssn_create(int levels, int base, int cin, int cout, int N, int H, int W, void* ws, size_t ws_bytes, void* stream,
               ssn_net** out) {
  if (!out) return nfail(SS_EINVAL, "out is NULL");
  *out = nullptr;
  size_t need = 0;
  int rc = ssn_workspace_bytes(levels, base, cin, cout, N, H, W, &need);
  if (rc) return rc;
  if (!ws || ws_bytes < need || ((uintptr_t)ws) % 256) return nfail(SS_EINVAL, "workspace missing, small or misaligned");
  ssn_net* n = new (std::nothrow) ssn_net();
  if (!n) return nfail(SS_EINVAL, "out of host memory");
  n->levels = levels; n->base = base; n->cin = cin; n->cout = cout; n->cin_pad = 16;
  n->Ncap = N; n->H = H; n->W = W;
  n->stream = (hipStream_t)stream;
  n->adam_t = 0;
  n->conv_shape = 0;
  if (const char* env = std::getenv("SSN_CONV_SHAPE")) {
    const int v = std::atoi(env);
    if (v >= 0 && v <= 3) n->conv_shape = v;
  }
  net_layers(n);
  n->bytes = net_carve(n, (char*)ws);
  hipError_t e = hipMemsetAsync(ws, 0, n->bytes, n->stream);
  if (e != hipSuccess) {
    delete n;
    return nfail(SS_EHIP, std::string("hipMemsetAsync: ") + hipGetErrorString(e));
  }
  *out = n;
  return SS_OK;
}

void ssn_destroy(ssn_net* n) {
  if (!n) return;
  if (n->fgraph) (void)hipGraphExecDestroy(n->fgraph);
  if (n->fcap) (void)hipStreamDestroy(n->fcap);
  delete n;
}

long ssn_num_params(ssn_net* n) { return n ? oracle_count(n) : SS_EINVAL; }

int ssn_set_weights(ssn_net* n, const float* host, long count) {
  if (!n || !host || count != oracle_count(n)) return nfail(SS_EINVAL, "weights: wrong count");
  std::vector<float> flat(n->np, 0.0f);
  for_each_param(n, [&](long o, long d) { flat[d] = host[o]; });
  SN_HIP(hipMemcpyAsync(n->P, flat.data(), n->np * 4, hipMemcpyHostToDevice, n->stream));
  SN_HIP(hipMemsetAsync(n->M, 0, n->np * 4, n->stream));
  SN_HIP(hipMemsetAsync(n->V, 0, n->np * 4, n->stream));
  n->adam_t = 0;
  pack_all(n);
  SN_HIP(hipGetLastError());
  SN_HIP(hipStreamSynchronize(n->stream));
  return SS_OK;
}

static int copy_out(ssn_net* n, const float* dev, float* host, long count) {
  if (!n || !host || count != oracle_count(n)) return nfail(SS_EINVAL, "wrong count");
  std::vector<float> flat(n->np);
  SN_HIP(hipMemcpyAsync(flat.data(), dev, n->np * 4, hipMemcpyDeviceToHost, n->stream));
  SN_HIP(hipStreamSynchronize(n->stream));
  for_each_param(n, [&](long o, long d) { host[o] = flat[d]; });
  return SS_OK;
}

int ssn_get_weights(ssn_net* n, float* host, long count) { return copy_out(n, n ? n->P : nullptr, host, count); }
int ssn_get_grads(ssn_net* n, float* host, long count) { return copy_out(n, n ? n->G : nullptr, host, count); }

}  // extern "C"

namespace {

// The BF16 tensor of kind `kind` of 3x3 layer k (layer order of the parameter
// exchange), as the last forward and backward passes left it.
bool layer_tensor(const ssn_net* n, int kind, int k, int nb, TV* out) {
  const int L = n->L;
  const int nconv = (int)n->conv.size();
  if (k < 0 || k >= nconv) return false;
  // locate the layer: encoder level l (a/b), bottleneck, or decoder level l (a/b)
  int l = -1, part = 0;  // part: 0 enc, 1 mid, 2 dec
  bool second = (k & 1) != 0;
  if (k < 2 * L) { l = k / 2; part = 0; }
  else if (k < 2 * L + 2) { part = 1; }
  else { l = L - 1 - (k - 2 * L - 2) / 2; part = 2; }
  const int c = l >= 0 ? n->ch[l] : n->ch[L], cn = l >= 0 ? n->ch[l + 1] : 0;
  TV t;
  t.p = nullptr;
  switch (kind) {
    case SSN_T_INPUT:
      if (part == 0) t = second ? n->AA[l].all(nb) : (l == 0 ? n->X0.all(nb) : n->Pin[l].all(nb));
      else if (part == 1) t = second ? n->AMa.all(nb) : n->Pin[L].all(nb);
      else t = second ? n->ADa[l].all(nb) : n->CAT[l].all(nb);
      break;
    case SSN_T_PREACT:
      if (part == 0) t = second ? n->ZB[l].all(nb) : n->ZA[l].all(nb);
      else if (part == 1) t = second ? n->ZMb.all(nb) : n->ZMa.all(nb);
      else t = second ? n->ZDb[l].all(nb) : n->ZDa[l].all(nb);
      break;
    case SSN_T_OUTPUT:
      if (part == 0) t = second ? n->CAT[l].view(nb, cn, c) : n->AA[l].all(nb);
      else if (part == 1) t = second ? n->AMb.all(nb) : n->AMa.all(nb);
      else t = second ? n->ADb[l].all(nb) : n->ADa[l].all(nb);
      break;
    case SSN_T_GRAD_PREACT:
      if (part == 0) t = second ? n->gCAT[l].view(nb, cn, c) : n->gT2[l].all(nb);
      else if (part == 1) t = second ? n->gM2.all(nb) : n->gM1.all(nb);
      else t = second ? n->gT1[l].all(nb) : n->gT3[l].all(nb);
      break;
    case SSN_T_GRAD_DATA:
      if (part == 0) {
        if (second) t = n->gT2[l].all(nb);
        else if (l > 0) t = n->gP[l].all(nb);
        else return false;  // the first layer's input gradient is not formed
      } else if (part == 1) {
        t = second ? n->gM1.all(nb) : n->gP[L].all(nb);
      } else {
        t = second ? n->gT3[l].all(nb) : n->gCAT[l].all(nb);
      }
      break;
    default:
      return false;
  }
  *out = t;
  return t.p != nullptr;
}

}  // namespace

extern "C" {

int ssn_tensor_shape(ssn_net* n, int kind, int layer, int* H, int* W, int* C) {
  if (!n || !H || !W || !C) return nfail(SS_EINVAL, "NULL argument");
  TV t;
  if (!layer_tensor(n, kind, layer, 1, &t)) return nfail(SS_EINVAL, "no such tensor");
  *H = t.H;
  *W = t.W;
  *C = t.C;
  return SS_OK;
}

int ssn_read_tensor(ssn_net* n, int kind, int layer, int nb, float* host, long count) {
  if (!n || !host) return nfail(SS_EINVAL, "NULL argument");
  if (nb < 1 || nb > n->Ncap) return nfail(SS_EINVAL, "image count out of range");
  TV t;
  if (!layer_tensor(n, kind, layer, nb, &t)) return nfail(SS_EINVAL, "no such tensor");
  const long npix = (long)nb * t.H * t.W;
  if (count != npix * t.C) return nfail(SS_EINVAL, "count must be n * H * W * C of the tensor");
  std::vector<bf16_t> raw((size_t)npix * t.cs);
  SN_HIP(hipMemcpyAsync(raw.data(), t.p, raw.size() * sizeof(bf16_t), hipMemcpyDeviceToHost, n->stream));
  SN_HIP(hipStreamSynchronize(n->stream));
  for (long p = 0; p < npix; ++p)
    for (int ch = 0; ch < t.C; ++ch) {
      const unsigned u = ((unsigned)raw[(size_t)p * t.cs + t.coff + ch]) << 16;
      float f;
      std::memcpy(&f, &u, 4);
      host[p * t.C + ch] = f;
    }
  return SS_OK;
}

int ssn_forward(ssn_net* n, const float* x, int nb, float* out) {
  if (!n || !x || nb < 1 || nb > n->Ncap) return nfail(SS_EINVAL, "bad forward arguments");
  int rc = net_forward(n, x, nb);
  if (rc) return rc;
  if (out)
    SN_HIP(hipMemcpyAsync(out, n->OUT, (size_t)nb * n->H * n->W * n->cout * 4, hipMemcpyDeviceToDevice, n->stream));
  return SS_OK;
}

int ssn_forward_graph(ssn_net* n, const float* x, int nb, float* out) {
  if (!n || !x || !out || nb < 1 || nb > n->Ncap) return nfail(SS_EINVAL, "bad forward arguments");
  if (!n->fgraph || n->fx != x || n->fout != out || n->fnb != nb) {
    if (n->fgraph) {
      (void)hipGraphExecDestroy(n->fgraph);
      n->fgraph = nullptr;
    }
    if (!n->fcap) SN_HIP(hipStreamCreateWithFlags(&n->fcap, hipStreamNonBlocking));
    hipStream_t s0 = n->stream;
    n->stream = n->fcap;  // the forward's launches go to the capture stream
    hipError_t e = hipStreamBeginCapture(n->fcap, hipStreamCaptureModeRelaxed);
    int rc = e == hipSuccess ? net_forward(n, x, nb) : SS_EHIP;
    if (rc == SS_OK) {
      hipLaunchKernelGGL(copy_f32, dim3(grid1((long)nb * n->H * n->W * n->cout)), dim3(256), 0, n->fcap, n->OUT, out,
                         (long)nb * n->H * n->W * n->cout);
    }
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(n->fcap, &g);
    n->stream = s0;
    if (e != hipSuccess || e2 != hipSuccess || rc != SS_OK)
      return nfail(SS_EHIP, std::string("forward capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    e = hipGraphInstantiate(&n->fgraph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      n->fgraph = nullptr;
      return nfail(SS_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    n->fx = x;
    n->fout = out;
    n->fnb = nb;
  }
  SN_HIP(hipGraphLaunch(n->fgraph, n->stream));
  return SS_OK;
}

int ssn_backward(ssn_net* n, const float* target, int nb, double* loss) {
  if (!n || !target || nb < 1 || nb > n->Ncap) return nfail(SS_EINVAL, "bad backward arguments");
  return net_backward(n, target, nb, loss);
}

int ssn_adam_step(ssn_net* n, float lr) {
  if (!n || !(lr > 0.0f)) return nfail(SS_EINVAL, "bad Adam arguments");
  n->adam_t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - std::pow(b1, (float)n->adam_t), c2 = 1.0f - std::pow(b2, (float)n->adam_t);
  const float* gs = nullptr;
  if (n->clip > 0.0f) {
    hipLaunchKernelGGL(grad_sq_partials, dim3(kPartBlocks), dim3(256), 0, n->stream, n->G, n->np, n->npart);
    hipLaunchKernelGGL(grad_clip_scale, dim3(1), dim3(256), 0, n->stream, n->npart, kPartBlocks, n->clip, n->gscale);
    gs = n->gscale;
  }
  hipLaunchKernelGGL(adam_update, dim3(grid1(n->np)), dim3(256), 0, n->stream, n->P, n->M, n->V, n->G, gs, n->np, lr,
                     b1, b2, 1e-8f, c1, c2);
  pack_all(n);
  SN_HIP(hipGetLastError());
  return SS_OK;
}

int ssn_set_grad_clip(ssn_net* n, float max_norm) {
  if (!n || !(max_norm >= 0.0f) || !std::isfinite(max_norm)) return nfail(SS_EINVAL, "bad clipping norm");
  n->clip = max_norm;
  return SS_OK;
}

int ssn_train_step(ssn_net* n, const float* x, const float* target, int nb, float lr, double* loss) {
  int rc = ssn_forward(n, x, nb, nullptr);
  if (rc) return rc;
  rc = ssn_backward(n, target, nb, loss);
  if (rc) return rc;
  return ssn_adam_step(n, lr);
}

// Forward and backward multiply-add flops of one sample (2 flops per MAC),
// counting the 3x3 and 1x1 convolutions at their real channel counts.
size_t ssn_init_field_workspace_bytes(ssn_net* n) { return n ? (size_t)n->H * n->W * 2 * sizeof(float) : 0; }

int ssn_init_field(ssn_net* n, ss_ctx* ctx, int nv, const double* xy, const double* w, double kappa, double sigma,
                   double pin, uint64_t seed, double noise_amp, void* work, size_t work_bytes) {
  if (!n || !ctx || !work) return nfail(SS_EINVAL, "net, ctx or work is NULL");
  if (n->cin != 2 || n->cout != 4) return nfail(SS_EINVAL, "the learned start needs a network with 2 inputs and 4 outputs");
  int Nx = 0, Ny = 0, theory = -1;
  if (ss_detail::ctx_shape(ctx, &Nx, &Ny, &theory) != SS_OK) return nfail(SS_EINVAL, "ctx is NULL");
  if (theory != SS_THEORY_AH) return nfail(SS_EINVAL, "the learned start exists for the Abelian Higgs model only");
  if (Nx != n->W || Ny != n->H) return nfail(SS_ESHAPE, "the network's image size differs from the lattice");
  if (work_bytes < ssn_init_field_workspace_bytes(n)) return nfail(SS_EINVAL, "work is too small");
  if ((uintptr_t)work % 256) return nfail(SS_EINVAL, "work must be 256-byte aligned");
  // input image on the context's stream (the call synchronises it)
  int rc = ss_learned_input(ctx, nv, xy, kappa, (float*)work);
  if (rc) return nfail(rc, std::string("input image: ") + ss_last_error());
  rc = ssn_forward(n, (const float*)work, 1, nullptr);
  if (rc) return rc;
  // the corrections are read from the network's own output buffer on the
  // context's stream, so the forward pass must have finished
  SN_HIP(hipStreamSynchronize(n->stream));
  rc = ss_init_learned(ctx, nv, xy, w, n->OUT, sigma, pin, seed, noise_amp);  // synchronises the context's stream
  if (rc) return nfail(rc, std::string("corrected ansatz: ") + ss_last_error());
  return SS_OK;
}

int ssn_flops(ssn_net* n, double* fwd, double* bwd) {
  if (!n) return nfail(SS_EINVAL, "net is NULL");
  double f = 0.0, b = 0.0;
  for (size_t k = 0; k < n->conv.size(); ++k) {
    const ConvL& c = n->conv[k];
    const double mac = (double)c.H * c.W * 9.0 * c.Co * c.Ci_real;
    f += 2.0 * mac;
    b += (k == 0 ? 2.0 : 4.0) * mac;  // weight gradient (+ input gradient except for the first layer)
  }
  const double head = (double)n->H * n->W * n->cout * n->ch[0];
  f += 2.0 * head;
  b += 4.0 * head;
  if (fwd) *fwd = f;
  if (bwd) *bwd = b;
  return SS_OK;
}

const char* ssn_last_error(void) { return g_ssn_err.c_str(); }

}  // extern "C"
