// Learned initialiser: a U-Net on BF16 MFMA (gfx950) with FP32 accumulation.
//
// Layout: activations NHWC in BF16 (element (n, y, x, c) at
// ((n * H + y) * W + x) * cs + coff + c, so a concatenation is two channel
// ranges of one buffer); 3x3 weights [co][tap][ci] with tap = 3 * ky + kx for
// offsets (ky - 1, kx - 1). Master weights, Adam moments and gradients are FP32.
//
// Kernels:
//   conv3x3_mfma   implicit GEMM, M = out channels, N = pixels, K = 9 * in channels,
//                  v_mfma_f32_32x32x16_bf16; forward (bias + SiLU epilogue) and
//                  backward-data (the same GEMM with flipped, transposed weights;
//                  optional SiLU' and accumulation epilogue);
//   conv3x3_wgrad  weight gradient, M = out channels, N = in channels per tap,
//                  K = pixels, operands staged transposed in LDS, split over
//                  pixel chunks with a fixed-order reduction (deterministic);
//   pool / upsample / head 1x1 / SiLU' / MSE / bias sums / Adam: plain kernels.
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
// zero outside the image) and its weights (32 WCO rows x 9 taps) are staged in
// LDS, each entry padded to kKP channels so that lanes reading neighbouring
// pixels or rows fall in different banks; every MFMA takes both operands from
// LDS and each weight fragment serves R rows. Requires W % (32 WPX) == 0,
// H % R == 0, in.C % 16 == 0 and, for WCO = 2, Co % 64 == 0 (weight rows exist
// up to gridDim.y * 32 WCO).
constexpr int kKC = 32, kKP = 40;

template <int WCO, int WPX, int R>
__global__ void __launch_bounds__(64 * WCO * WPX) conv3x3_tiled(ConvArgs a) {
  constexpr int NT = 64 * WCO * WPX, PX = 32 * WPX, PW = PX + 2, CO = 32 * WCO, PR = R + 2;
  __shared__ __align__(16) bf16_t sin_[PR * PW * kKP];
  __shared__ __align__(16) bf16_t sw[9 * CO * kKP];
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
    for (int it = tid; it < CO * 9 * nv; it += NT) {
      const int v = it % nv, q = it / nv;
      const int t = q % 9, co = q / 9;
      const bf16x8 val = *reinterpret_cast<const bf16x8*>(a.w + ((long)(co0 + co) * 9 + t) * Ci + c0 + v * 8);
      *reinterpret_cast<bf16x8*>(sw + (t * CO + co) * kKP + v * 8) = val;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int dy = t / 3, dx = t % 3;
      for (int ks = 0; ks < kc; ks += 16) {
        const bf16x8 A = *reinterpret_cast<const bf16x8*>(sw + (t * CO + wi * 32 + r) * kKP + ks + half * 8);
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const bf16x8 B =
              *reinterpret_cast<const bf16x8*>(sin_ + ((q + dy) * PW + wj * 32 + r + dx) * kKP + ks + half * 8);
          acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, acc[q], 0, 0, 0);
        }
      }
    }
  }
  // D[row][col]: lane holds col = r (pixel) and rows 8 (v / 4) + 4 half + v % 4 (channels)
  const int x = x0 + wj * 32 + r;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int y = y0 + q;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int co = co0 + wi * 32 + (v >> 2) * 8 + half * 4 + (v & 3);
      if (co >= a.Co) continue;
      float val = acc[q][v];
      if (a.mode == 0) {
        const float z = val + (a.bias ? a.bias[co] : 0.0f);
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
// A chunk is cw pixels of one image row (cw = 64 or W); its gz rows and the
// three x rows around it (cw + 2 pixels wide) are staged transposed in LDS.
constexpr int kCW = 64;
struct WgradArgs {
  TV gz;        // gradient w.r.t. the layer's pre-activation (C = Co)
  TV x;         // layer input (C = Ci)
  float* part;  // [nsplit][Co][9][Ci]
  int nsplit;
  int cw;       // pixels per chunk (divides W, multiple of 16, <= kCW)
};

__global__ void __launch_bounds__(576) conv3x3_wgrad(WgradArgs a) {
  __shared__ __align__(16) bf16_t gzT[32][kCW + 8];      // [co][pix]
  __shared__ __align__(16) bf16_t xT[3][32][kCW + 8 + 2]; // [row][ci][pix + 1]
  const int lane = threadIdx.x & 63, tap = threadIdx.x >> 6;
  const int r = lane & 31, half = lane >> 5;
  const int ci0 = blockIdx.x * 32, co0 = blockIdx.y * 32, split = blockIdx.z;
  const int H = a.x.H, W = a.x.W, Ci = a.x.C, Co = a.gz.C, cw = a.cw;
  const int chunks_per_row = W / cw;
  const long nchunks = (long)a.x.N * H * chunks_per_row;
  const int dy = tap / 3 - 1, dx = tap % 3 - 1;
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
  for (long ch = split; ch < nchunks; ch += a.nsplit) {
    const int n = (int)(ch / ((long)H * chunks_per_row));
    const int rem = (int)(ch - (long)n * H * chunks_per_row);
    const int y = rem / chunks_per_row, x0 = (rem - y * chunks_per_row) * cw;
    // stage gz[pix][co0..co0+31] transposed
    for (int e = threadIdx.x; e < cw * 32; e += 576) {
      const int pix = e >> 5, c = e & 31;
      gzT[c][pix] = (co0 + c < Co) ? a.gz.p[tv_at(a.gz, n, y, x0 + pix) + co0 + c] : (bf16_t)0;
    }
    // stage x rows y-1..y+1, pixels x0-1..x0+cw, channels ci0..ci0+31, transposed
    for (int e = threadIdx.x; e < 3 * (cw + 2) * 32; e += 576) {
      const int c = e & 31, k = e >> 5;
      const int row = k / (cw + 2), pix = k - row * (cw + 2);
      const int yy = y + row - 1, xx = x0 + pix - 1;
      bf16_t val = 0;
      if (yy >= 0 && yy < H && xx >= 0 && xx < W && ci0 + c < Ci) val = a.x.p[tv_at(a.x, n, yy, xx) + ci0 + c];
      xT[row][c][pix] = val;
    }
    __syncthreads();
    if (tap < 9) {
      for (int kk = 0; kk < cw; kk += 16) {
        bf16x8 A, B;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int pix = kk + half * 8 + j;
          A[j] = __builtin_bit_cast(__bf16, gzT[r][pix]);
          B[j] = __builtin_bit_cast(__bf16, xT[dy + 1][r][pix + dx + 1]);
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, acc, 0, 0, 0);
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

// out[k] = sum over s of part[s][k], in split order
__global__ void reduce_splits(const float* __restrict__ part, int nsplit, long n, float* __restrict__ out) {
  const long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (k >= n) return;
  float s = 0.0f;
  for (int i = 0; i < nsplit; ++i) s += part[(long)i * n + k];
  out[k] = s;
}

// Per-block channel sums of an NHWC view (bf16 g, or fp32 gf with channel
// stride gf_cs) into fp32 partials [nblk][C]. Block y takes channels
// [256 y, 256 y + Cc), Cc = min(C - 256 y, 256); thread t sums channel t % Cc
// over the pixels b0 + t / Cc, step 256 / Cc, of the block's pixel range, and
// the lanes of each channel are then added in lane order (deterministic).
__global__ void __launch_bounds__(256) channel_sums(TV g, const float* __restrict__ gf, int gf_cs, long npix, int C,
                                                    float* __restrict__ part) {
  __shared__ float red[256];
  const int t = threadIdx.x;
  const int c0 = 256 * blockIdx.y;
  const int Cc = min(C - c0, 256);
  const int L = 256 / Cc;
  const int c = t % Cc, l = t / Cc;
  const long per = (npix + gridDim.x - 1) / gridDim.x;
  const long b0 = blockIdx.x * per, b1 = std::min(npix, b0 + per);
  float s = 0.0f;
  if (l < L) {
    if (gf)
      for (long p = b0 + l; p < b1; p += L) s += gf[p * gf_cs + c0 + c];
    else
      for (long p = b0 + l; p < b1; p += L) s += bf2f(g.p[p * g.cs + g.coff + c0 + c]);
  }
  red[t] = s;
  __syncthreads();
  if (t < Cc) {
    float a = 0.0f;
    for (int k = 0; k < L; ++k) a += red[k * Cc + t];
    part[(long)blockIdx.x * C + c0 + t] = a;
  }
}

__global__ void avgpool2_fwd(TV in, TV out) {
  const long n = (long)out.N * out.H * out.W * out.C;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    const int c = (int)(k % out.C);
    long p = k / out.C;
    const int x = (int)(p % out.W);
    p /= out.W;
    const int y = (int)(p % out.H);
    const int b = (int)(p / out.H);
    float s = 0.0f;
    for (int j = 0; j < 2; ++j)
      for (int i = 0; i < 2; ++i) s += bf2f(in.p[tv_at(in, b, 2 * y + j, 2 * x + i) + c]);
    out.p[tv_at(out, b, y, x) + c] = f2bf(0.25f * s);
  }
}

// gin (+)= gout / 4 spread over each 2x2 block
__global__ void avgpool2_bwd(TV gout, TV gin, int accumulate) {
  const long n = (long)gin.N * gin.H * gin.W * gin.C;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    const int c = (int)(k % gin.C);
    long p = k / gin.C;
    const int x = (int)(p % gin.W);
    p /= gin.W;
    const int y = (int)(p % gin.H);
    const int b = (int)(p / gin.H);
    float v = 0.25f * bf2f(gout.p[tv_at(gout, b, y >> 1, x >> 1) + c]);
    bf16_t* o = gin.p + tv_at(gin, b, y, x) + c;
    if (accumulate) v += bf2f(*o);
    *o = f2bf(v);
  }
}

__global__ void upsample2_fwd(TV in, TV out) {
  const long n = (long)out.N * out.H * out.W * out.C;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    const int c = (int)(k % out.C);
    long p = k / out.C;
    const int x = (int)(p % out.W);
    p /= out.W;
    const int y = (int)(p % out.H);
    const int b = (int)(p / out.H);
    out.p[tv_at(out, b, y, x) + c] = in.p[tv_at(in, b, y >> 1, x >> 1) + c];
  }
}

// gin = sum of gout over each 2x2 block
__global__ void upsample2_bwd(TV gout, TV gin) {
  const long n = (long)gin.N * gin.H * gin.W * gin.C;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    const int c = (int)(k % gin.C);
    long p = k / gin.C;
    const int x = (int)(p % gin.W);
    p /= gin.W;
    const int y = (int)(p % gin.H);
    const int b = (int)(p / gin.H);
    float s = 0.0f;
    for (int j = 0; j < 2; ++j)
      for (int i = 0; i < 2; ++i) s += bf2f(gout.p[tv_at(gout, b, 2 * y + j, 2 * x + i) + c]);
    gin.p[tv_at(gin, b, y, x) + c] = f2bf(s);
  }
}

// g *= SiLU'(z) in place
__global__ void silu_bwd_inplace(TV g, TV z) {
  const long n = (long)g.N * g.H * g.W * g.C;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    const int c = (int)(k % g.C);
    const long p = k / g.C;
    bf16_t* o = g.p + p * g.cs + g.coff + c;
    *o = f2bf(bf2f(*o) * silu_grad_f(bf2f(z.p[p * z.cs + z.coff + c])));
  }
}

// head: out[pix][o] = sum_ci w[o][ci] a[pix][ci] + b[o]   (fp32 out, cout <= 8)
__global__ void head_fwd(TV a, const float* __restrict__ w, const float* __restrict__ b, int cout,
                         float* __restrict__ out, long npix) {
  const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (p >= npix) return;
  const bf16_t* ap = a.p + p * a.cs + a.coff;
  for (int o = 0; o < cout; ++o) {
    float s = b[o];
    for (int c = 0; c < a.C; ++c) s += w[o * a.C + c] * bf2f(ap[c]);
    out[p * cout + o] = s;
  }
}

// head backward to its input, times SiLU'(z): ga[pix][ci] = SiLU'(z) sum_o gout[pix][o] w[o][ci]
__global__ void head_bwd_data(const float* __restrict__ gout, const float* __restrict__ w, int cout, TV z, TV ga,
                              long npix) {
  const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (p >= npix) return;
  for (int c = 0; c < ga.C; ++c) {
    float s = 0.0f;
    for (int o = 0; o < cout; ++o) s += gout[p * cout + o] * w[o * ga.C + c];
    s *= silu_grad_f(bf2f(z.p[p * z.cs + z.coff + c]));
    ga.p[p * ga.cs + ga.coff + c] = f2bf(s);
  }
}

// Per-block partials of gw[o][ci] = sum_pix gout[pix][o] a[pix][ci] ([nblk][cout * C],
// cout * C <= 256): thread t takes entry k = t % K, K = cout * C, over the pixels
// b0 + t / K, step 256 / K, of the block's range; lanes are added in order.
__global__ void __launch_bounds__(256) head_wgrad(const float* __restrict__ gout, TV a, int cout, long npix,
                                                  float* __restrict__ part) {
  __shared__ float red[256];
  const int t = threadIdx.x;
  const int K = cout * a.C;
  const int L = 256 / K;
  const int k = t % K, l = t / K;
  const int o = k / a.C, c = k - o * a.C;
  const long per = (npix + gridDim.x - 1) / gridDim.x;
  const long b0 = blockIdx.x * per, b1 = std::min(npix, b0 + per);
  float s = 0.0f;
  if (l < L)
    for (long p = b0 + l; p < b1; p += L) s += gout[p * cout + o] * bf2f(a.p[p * a.cs + a.coff + c]);
  red[t] = s;
  __syncthreads();
  if (t < K) {
    float acc = 0.0f;
    for (int q = 0; q < L; ++q) acc += red[q * K + t];
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

// Adam (Kingma and Ba 2015) with bias correction; grads g, moments m, v, master p (fp32)
__global__ void adam_update(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, long n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    const float gk = g[k];
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
  std::vector<HT> gCAT, gT1, gT2, gP;
  HT gM1, gM2;
  float *OUT, *GOUT, *part, *cpart;
  double* lpart;
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
  n->gCAT.assign(L, HT()); n->gT1.assign(L, HT()); n->gT2.assign(L, HT()); n->gP.assign(L + 1, HT());
  for (int l = 0; l < L; ++l) {
    const int H = n->H >> l, W = n->W >> l, c = n->ch[l], cn = n->ch[l + 1];
    tensor(n->ZA[l], H, W, c); tensor(n->AA[l], H, W, c); tensor(n->ZB[l], H, W, c);
    tensor(n->CAT[l], H, W, cn + c);
    tensor(n->ZDa[l], H, W, c); tensor(n->ADa[l], H, W, c); tensor(n->ZDb[l], H, W, c); tensor(n->ADb[l], H, W, c);
    tensor(n->gCAT[l], H, W, cn + c); tensor(n->gT1[l], H, W, c); tensor(n->gT2[l], H, W, c);
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

void launch_wgrad(ssn_net* n, const ConvL& c, TV gz, TV x) {
  const int cw = std::min(kCW, x.W);
  const long nchunks = (long)x.N * x.H * (x.W / cw);
  const int tci = (c.Ci + 31) / 32, tco = (c.Co + 31) / 32;
  int nsplit = (int)std::max<long>(1, std::min<long>(nchunks, 256 / (tci * tco)));
  while ((long)nsplit * c.Co * 9 * c.Ci > kWgradPartFloats) nsplit /= 2;
  WgradArgs wa;
  wa.gz = gz;
  wa.x = x;
  wa.part = n->part;
  wa.nsplit = nsplit;
  wa.cw = cw;
  hipLaunchKernelGGL(conv3x3_wgrad, dim3(tci, tco, nsplit), dim3(576), 0, n->stream, wa);
  const long nw = (long)c.Co * 9 * c.Ci;
  hipLaunchKernelGGL(reduce_splits, dim3(grid1(nw)), dim3(256), 0, n->stream, n->part, nsplit, nw, n->G + c.w_off);
  // bias gradient: per-channel sums of gz
  hipLaunchKernelGGL(channel_sums, dim3(kPartBlocks, (c.Co + 255) / 256), dim3(256), 0, n->stream, gz,
                     (const float*)nullptr, 0, (long)gz.N * gz.H * gz.W, c.Co, n->cpart);
  hipLaunchKernelGGL(reduce_splits, dim3(grid1(c.Co)), dim3(256), 0, n->stream, n->cpart, kPartBlocks, (long)c.Co,
                     n->G + c.b_off);
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
    hipLaunchKernelGGL(avgpool2_fwd, dim3(grid1((long)nb * pooled.H * pooled.W * c)), dim3(256), 0, n->stream, skip,
                       pooled);
  }
  launch_conv_fwd(n, n->conv[mid_a(n)], n->Pin[L].all(nb), n->ZMa.all(nb), n->AMa.all(nb));
  launch_conv_fwd(n, n->conv[mid_b(n)], n->AMa.all(nb), n->ZMb.all(nb), n->AMb.all(nb));
  for (int l = L - 1; l >= 0; --l) {
    const int cn = n->ch[l + 1];
    TV prev = l == L - 1 ? n->AMb.all(nb) : n->ADb[l + 1].all(nb);
    TV up = n->CAT[l].view(nb, 0, cn);
    hipLaunchKernelGGL(upsample2_fwd, dim3(grid1((long)nb * up.H * up.W * cn)), dim3(256), 0, n->stream, prev, up);
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
  hipLaunchKernelGGL(reduce_splits, dim3(grid1((long)n->cout * n->ch[0])), dim3(256), 0, n->stream, n->cpart,
                     kPartBlocks, (long)n->cout * n->ch[0], n->G + n->hw_off);
  TV none;
  none.p = nullptr;
  hipLaunchKernelGGL(channel_sums, dim3(kPartBlocks), dim3(256), 0, n->stream, none, n->GOUT, n->cout, npix, n->cout,
                     n->cpart);
  hipLaunchKernelGGL(reduce_splits, dim3(1), dim3(256), 0, n->stream, n->cpart, kPartBlocks, (long)n->cout,
                     n->G + n->hb_off);
  hipLaunchKernelGGL(head_bwd_data, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, n->stream, n->GOUT,
                     n->P + n->hw_off, n->cout, n->ZDb[0].all(nb), n->gT1[0].all(nb), npix);
  // decoder, top level first
  for (int l = 0; l < L; ++l) {
    const int cn = n->ch[l + 1];
    const ConvL& cb = n->conv[dec_b(n, l)];
    const ConvL& ca = n->conv[dec_a(n, l)];
    launch_wgrad(n, cb, n->gT1[l].all(nb), n->ADa[l].all(nb));
    TV za = n->ZDa[l].all(nb);
    launch_conv_bwd_data(n, cb, n->gT1[l].all(nb), n->gT2[l].all(nb), &za);
    launch_wgrad(n, ca, n->gT2[l].all(nb), n->CAT[l].all(nb));
    launch_conv_bwd_data(n, ca, n->gT2[l].all(nb), n->gCAT[l].all(nb), nullptr);
    // the upsampled half of the concatenation feeds back to the level below
    TV gup = n->gCAT[l].view(nb, 0, cn);
    TV dst = l == L - 1 ? n->gM2.all(nb) : n->gT1[l + 1].all(nb);
    TV zsrc = l == L - 1 ? n->ZMb.all(nb) : n->ZDb[l + 1].all(nb);
    hipLaunchKernelGGL(upsample2_bwd, dim3(grid1((long)nb * dst.H * dst.W * cn)), dim3(256), 0, n->stream, gup, dst);
    hipLaunchKernelGGL(silu_bwd_inplace, dim3(grid1((long)nb * dst.H * dst.W * cn)), dim3(256), 0, n->stream, dst,
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
    hipLaunchKernelGGL(avgpool2_bwd, dim3(grid1((long)nb * gS.H * gS.W * c)), dim3(256), 0, n->stream,
                       n->gP[l + 1].all(nb), gS, 1);
    hipLaunchKernelGGL(silu_bwd_inplace, dim3(grid1((long)nb * gS.H * gS.W * c)), dim3(256), 0, n->stream, gS,
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
  hipLaunchKernelGGL(adam_update, dim3(grid1(n->np)), dim3(256), 0, n->stream, n->P, n->M, n->V, n->G, n->np, lr, b1,
                     b2, 1e-8f, c1, c2);
  pack_all(n);
  SN_HIP(hipGetLastError());
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
