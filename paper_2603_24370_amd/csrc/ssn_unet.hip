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
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/ss.h"

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

// Each wave: 32 output channels x (32 * WN) pixels; block: 4 waves along pixels.
template <int WN>
__global__ void __launch_bounds__(256) conv3x3_mfma(ConvArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 31, half = lane >> 5;
  const int co0 = blockIdx.y * 32;
  const int H = a.in.H, W = a.in.W, Ci = a.in.C;
  const long P = (long)a.in.N * H * W;
  const long pixbase = ((long)blockIdx.x * 4 + wave) * (32 * WN);
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

// per-block channel sums of an NHWC view (fp32 partials [nblk][C]); C <= 256
__global__ void __launch_bounds__(256) channel_sums(TV g, const float* __restrict__ gf, int gf_cs, long npix, int C,
                                                    float* __restrict__ part) {
  const int c = threadIdx.x;
  if (c >= C) return;
  const long per = (npix + gridDim.x - 1) / gridDim.x;
  const long b0 = blockIdx.x * per, b1 = std::min(npix, b0 + per);
  float s = 0.0f;
  for (long p = b0; p < b1; ++p) s += gf ? gf[p * gf_cs + c] : bf2f(g.p[p * g.cs + g.coff + c]);
  part[(long)blockIdx.x * C + c] = s;
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

// per-block partials of gw[o][ci] = sum_pix gout[pix][o] a[pix][ci]  ([nblk][cout * C])
__global__ void __launch_bounds__(256) head_wgrad(const float* __restrict__ gout, TV a, int cout, long npix,
                                                  float* __restrict__ part) {
  const int k = threadIdx.x;  // o * C + c
  if (k >= cout * a.C) return;
  const int o = k / a.C, c = k - o * a.C;
  const long per = (npix + gridDim.x - 1) / gridDim.x;
  const long b0 = blockIdx.x * per, b1 = std::min(npix, b0 + per);
  float s = 0.0f;
  for (long p = b0; p < b1; ++p) s += gout[p * cout + o] * bf2f(a.p[p * a.cs + a.coff + c]);
  part[(long)blockIdx.x * cout * a.C + k] = s;
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
