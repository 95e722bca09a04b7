// Warm-start network (include/wf_nn.h): bfloat16 matrix-core convolutions
// with float32 accumulation, the encoder-decoder's forward and backward
// passes, Adam, and the C ABI.
//
// Every 3x3 convolution is an implicit GEMM on v_mfma_f32_16x16x32_bf16:
// output pixels are the rows, output channels the columns and (tap, input
// channel) the reduction.  Activations are [pixel][channel] bfloat16 so that
// one lane's eight consecutive reduction values are one 16-byte load; the
// periodic neighbour of each pixel is computed per tap, so no halo copies
// are made.  The weight gradient is the same product with pixels as the
// reduction: 64-pixel slabs of the input and of the output gradient are
// staged transposed in LDS, each block sums one pixel chunk, and a second
// kernel adds the chunks in a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "wf.h"
#include "wf_nn.h"

namespace wfnn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kLevels = 4;
constexpr int kChan[kLevels] = {32, 64, 96, 128};
constexpr int kLayers = 4 * kLevels - 1;
constexpr int kPad = 32;  // channels of the padded input and output

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// round to nearest even; NaN stays NaN
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// ---------------------------------------------------------------------------
// convolution (forward, and the input adjoint with mirrored taps)
// ---------------------------------------------------------------------------

struct ConvArgs {
  const uint16_t* in;  // [P][cin]
  const uint16_t* wt;  // [9][cout][cin]: reduction dimension contiguous
  const float* bias;   // [cout] or null
  uint16_t* out;       // [P][cout] or null
  float* out_f32;      // [P]: channel 0 in float32, or null
  int h, w, cin, cout;
  int flip;            // 1: tap (dy, dx) reads the pixel at (-dy, -dx)
  int relu;
  int64_t P;           // pixels
};

// Block: 256 threads, 128 pixels x COT output channels; wave w owns pixels
// 32w..32w+31 of the block (two 16-row tiles) and every column tile, so each
// weight fragment feeds two MFMAs.  One tap's weights (COT x cin) are staged
// in LDS and shared by the four waves.  Pixels past the end (P not a multiple
// of 128) read a valid pixel and store nothing.
template <int COT>
__global__ __launch_bounds__(256) void conv_kernel(ConvArgs a) {
  constexpr int NJ = COT / 16;
  constexpr int WS = 128 + 8;  // LDS row: up to 128 input channels + pad
  __shared__ __attribute__((aligned(16))) uint16_t ws[COT * WS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, kq = lane >> 4;
  const int64_t pw = (int64_t)blockIdx.x * 128 + wave * 32;
  const int co0 = blockIdx.y * COT;
  const int hw = a.h * a.w;
  int64_t img[2];
  int yy0[2], xx0[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    int64_t p = pw + 16 * u + r;
    if (p >= a.P) p = a.P - 1;
    img[u] = p / hw;
    const int rem = (int)(p - img[u] * hw);
    yy0[u] = rem / a.w;
    xx0[u] = rem - yy0[u] * a.w;
  }
  f32x4 acc[2][NJ];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[u][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int c8 = a.cin / 8;
  for (int t = 0; t < 9; ++t) {
    __syncthreads();  // the previous tap's weights have been consumed
    for (int i = threadIdx.x; i < COT * c8; i += 256) {
      const int co = i / c8, cc = i - co * c8;
      *(uint4*)&ws[co * WS + cc * 8] =
          *(const uint4*)(a.wt + ((int64_t)t * a.cout + co0 + co) * a.cin + cc * 8);
    }
    __syncthreads();
    int dy = t / 3 - 1, dx = t % 3 - 1;
    if (a.flip) {
      dy = -dy;
      dx = -dx;
    }
    const uint16_t* arow[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int yy = wrap(yy0[u] + dy, a.h), xx = wrap(xx0[u] + dx, a.w);
      arow[u] = a.in + (img[u] * hw + (int64_t)yy * a.w + xx) * a.cin + kq * 8;
    }
    for (int c = 0; c < a.cin; c += 32) {
      const bf16x8 a0 = __builtin_bit_cast(bf16x8, *(const uint4*)(arow[0] + c));
      const bf16x8 a1 = __builtin_bit_cast(bf16x8, *(const uint4*)(arow[1] + c));
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const bf16x8 bv = __builtin_bit_cast(bf16x8, *(const uint4*)&ws[(16 * j + r) * WS + c + kq * 8]);
        acc[0][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bv, acc[0][j], 0, 0, 0);
        acc[1][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bv, acc[1][j], 0, 0, 0);
      }
    }
  }
  // lane holds rows 4 kq + v (pixels) of column r (channel) of each tile
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int co = co0 + 16 * j + r;
    const float bb = a.bias ? a.bias[co] : 0.f;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t pp = pw + 16 * u + 4 * kq + v;
        if (pp >= a.P) continue;
        float val = acc[u][j][v] + bb;
        if (a.relu) val = fmaxf(val, 0.f);
        if (a.out) a.out[pp * a.cout + co] = f2bf(val);
        if (a.out_f32 && co == 0) a.out_f32[pp] = val;
      }
  }
}

// ---------------------------------------------------------------------------
// weight gradient: part[chunk][t][ci][co] = sum over the chunk's pixels p of
// in[p + tap t][ci] g[p][co]
// ---------------------------------------------------------------------------

struct WgradArgs {
  const uint16_t* in;  // [P][cin]
  const uint16_t* g;   // [P][cout]
  float* part;         // [nchunk][9][cin][cout]
  int h, w, cin, cout;
  int64_t chunk;       // pixels per block, a multiple of 64
};

// grid (nchunk, (cin/32) * (cout/32)); each block one 32 x 32 (ci, co) tile
// of all nine taps over its pixel chunk.  Per 64-pixel slab the output
// gradient is staged once and the input once per tap (its periodic
// neighbours), both transposed to [channel][pixel] in LDS so that a lane's 8
// consecutive pixels are one 16-byte read; wave w owns the 16 x 16 sub-tile
// (w / 2, w % 2) of every tap.
__global__ __launch_bounds__(256) void wgrad_kernel(WgradArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t xs[9][32][72];  // [tap][ci][pixel]
  __shared__ __attribute__((aligned(16))) uint16_t gs[32][72];     // [co][pixel]
  const int ntc = a.cout / 32;
  const int ci0 = (int)(blockIdx.y / ntc) * 32, co0 = (int)(blockIdx.y % ntc) * 32;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int si = (wave >> 1) * 16, sj = (wave & 1) * 16;
  const int sp = threadIdx.x >> 2;         // staged pixel 0..63
  const int sc = (threadIdx.x & 3) * 8;    // staged channel offset
  const int hw = a.h * a.w;
  f32x4 acc[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int64_t pbeg = (int64_t)blockIdx.x * a.chunk;
  for (int64_t pb = pbeg; pb < pbeg + a.chunk; pb += 64) {
    const int64_t p = pb + sp;
    const int64_t img = p / hw;
    const int rem = (int)(p - img * hw);
    const int y = rem / a.w, x = rem - (rem / a.w) * a.w;
    uint4 xv[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int dy = t / 3 - 1, dx = t % 3 - 1;
      const int64_t q = img * hw + (int64_t)wrap(y + dy, a.h) * a.w + wrap(x + dx, a.w);
      xv[t] = *(const uint4*)(a.in + q * a.cin + ci0 + sc);
    }
    const uint4 gv = *(const uint4*)(a.g + p * a.cout + co0 + sc);
    __syncthreads();  // the previous slab has been consumed
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const uint16_t* xe = (const uint16_t*)&xv[t];
#pragma unroll
      for (int e = 0; e < 8; ++e) xs[t][sc + e][sp] = xe[e];
    }
    const uint16_t* ge = (const uint16_t*)&gv;
#pragma unroll
    for (int e = 0; e < 8; ++e) gs[sc + e][sp] = ge[e];
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 64; ks += 32) {
      const bf16x8 bv = __builtin_bit_cast(bf16x8, *(const uint4*)&gs[sj + (lane & 15)][ks + 8 * (lane >> 4)]);
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        const bf16x8 av =
            __builtin_bit_cast(bf16x8, *(const uint4*)&xs[t][si + (lane & 15)][ks + 8 * (lane >> 4)]);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[t], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    float* dst = a.part + (((int64_t)blockIdx.x * 9 + t) * a.cin + ci0 + si) * a.cout + co0 + sj;
#pragma unroll
    for (int v = 0; v < 4; ++v) dst[(int64_t)(4 * (lane >> 4) + v) * a.cout + (lane & 15)] = acc[t][v];
  }
}

// out[i] = sum_c part[c][i] in a fixed order.  A block takes 32 consecutive
// i and 8 groups of chunks (group g sums chunks g, g+8, ...), so that many
// loads are in flight; the 8 group sums are then added in order.
__global__ __launch_bounds__(256) void chunk_sum_kernel(const float* __restrict__ part, int nchunk, int64_t n,
                                                        float* __restrict__ out) {
  __shared__ float sh[8][32];
  const int li = threadIdx.x & 31, grp = threadIdx.x >> 5;
  const int64_t i = (int64_t)blockIdx.x * 32 + li;
  float s = 0.f;
  if (i < n)
    for (int c = grp; c < nchunk; c += 8) s += part[(int64_t)c * n + i];
  sh[grp][li] = s;
  __syncthreads();
  if (grp == 0 && i < n) {
    float t = 0.f;
#pragma unroll
    for (int g = 0; g < 8; ++g) t += sh[g][li];
    out[i] = t;
  }
}

// bias gradient partials: part[chunk][co] = sum over the chunk of g[p][co].
// A thread reads 8 channels of one pixel per step (16-byte loads, whole
// pixels per step across the block); the per-thread sums are then added
// over the block's pixel lanes in LDS.
__global__ __launch_bounds__(256) void colsum_kernel(const uint16_t* __restrict__ g, int cout,
                                                     int64_t chunk, float* __restrict__ part) {
  __shared__ float red[256 * 8];
  const int vpp = cout / 8;            // 16-byte vectors per pixel
  const int ppi = 256 / vpp;           // pixels per step
  const int lp = threadIdx.x / vpp, v = threadIdx.x - lp * vpp;
  float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  const int64_t pbeg = (int64_t)blockIdx.x * chunk;
  if (lp < ppi) {
    for (int64_t p = pbeg + lp; p < pbeg + chunk; p += ppi) {
      const uint4 u = *(const uint4*)(g + p * cout + 8 * v);
      const uint16_t* h = (const uint16_t*)&u;
#pragma unroll
      for (int e = 0; e < 8; ++e) acc[e] += bf2f(h[e]);
    }
  }
#pragma unroll
  for (int e = 0; e < 8; ++e) red[threadIdx.x * 8 + e] = acc[e];
  __syncthreads();
  for (int co = threadIdx.x; co < cout; co += blockDim.x) {
    const int vv = co / 8, e = co - vv * 8;
    float sum = 0.f;
    for (int l = 0; l < ppi; ++l) sum += red[(l * vpp + vv) * 8 + e];
    part[(int64_t)blockIdx.x * cout + co] = sum;
  }
}

// ---------------------------------------------------------------------------
// resampling and elementwise work on [P][C] bfloat16 (8 channels per thread)
// ---------------------------------------------------------------------------

__device__ __forceinline__ void unpack8(uint4 v, float* f) {
  const uint16_t* h = (const uint16_t*)&v;
#pragma unroll
  for (int e = 0; e < 8; ++e) f[e] = bf2f(h[e]);
}
__device__ __forceinline__ uint4 pack8(const float* f) {
  uint4 v;
  uint16_t* h = (uint16_t*)&v;
#pragma unroll
  for (int e = 0; e < 8; ++e) h[e] = f2bf(f[e]);
  return v;
}

enum Ew { EW_POOL = 0, EW_UP = 1, EW_ADD = 2, EW_RELU_BWD = 3, EW_UP_ADJ = 4, EW_ADD_POOL_ADJ = 5 };

// One thread per 8 channels of one output pixel.  Sizes (oh, ow) are the
// output's; the coarse/fine partner is at half/double resolution.
//   POOL        out[y][x] = mean of in[2y+a][2x+b]
//   UP          out[y][x] = in[y/2][x/2]
//   ADD         out = in + in2
//   RELU_BWD    out = in * (in2 > 0)
//   UP_ADJ      out[y][x] = sum of in[2y+a][2x+b]
//   ADD_POOL_ADJ out[y][x] += in[y/2][x/2] / 4
// (out may alias in: each thread reads its element before writing it)
__global__ void ew_kernel(int op, const uint16_t* in, const uint16_t* in2, uint16_t* out, int64_t npix,
                          int oh, int ow, int c) {
  const int c8 = c / 8;
  const int64_t total = npix * c8;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = i / c8;
    const int cc = (int)(i - p * c8) * 8;
    const int64_t img = p / ((int64_t)oh * ow);
    const int rem = (int)(p - img * oh * ow);
    const int y = rem / ow, x = rem - (rem / ow) * ow;
    float f[8], g[8];
    if (op == EW_POOL || op == EW_UP_ADJ) {
      const int ih = 2 * oh, iw = 2 * ow;
#pragma unroll
      for (int e = 0; e < 8; ++e) f[e] = 0.f;
      for (int a2 = 0; a2 < 2; ++a2)
        for (int b2 = 0; b2 < 2; ++b2) {
          const int64_t q = (img * ih + 2 * y + a2) * iw + 2 * x + b2;
          unpack8(*(const uint4*)(in + q * c + cc), g);
#pragma unroll
          for (int e = 0; e < 8; ++e) f[e] += g[e];
        }
      if (op == EW_POOL)
#pragma unroll
        for (int e = 0; e < 8; ++e) f[e] *= 0.25f;
    } else if (op == EW_UP || op == EW_ADD_POOL_ADJ) {
      const int ih = oh / 2, iw = ow / 2;
      const int64_t q = (img * ih + y / 2) * iw + x / 2;
      unpack8(*(const uint4*)(in + q * c + cc), f);
      if (op == EW_ADD_POOL_ADJ) {
        unpack8(*(const uint4*)(out + p * c + cc), g);
#pragma unroll
        for (int e = 0; e < 8; ++e) f[e] = g[e] + 0.25f * f[e];
      }
    } else {
      unpack8(*(const uint4*)(in + p * c + cc), f);
      unpack8(*(const uint4*)(in2 + p * c + cc), g);
#pragma unroll
      for (int e = 0; e < 8; ++e) f[e] = (op == EW_ADD) ? f[e] + g[e] : (g[e] > 0.f ? f[e] : 0.f);
    }
    *(uint4*)(out + p * c + cc) = pack8(f);
  }
}

// ---------------------------------------------------------------------------
// features, targets, loss, output scaling
// ---------------------------------------------------------------------------

// per-block partial sums of N_pix and of the observed count over a slice
// of map blockIdx.x (gridDim.y slices per map): part[m][slice][2]
template <class T>
__global__ __launch_bounds__(256) void sigma_kernel(const T* __restrict__ npix,
                                                    const uint8_t* __restrict__ mask, int64_t hw,
                                                    double* __restrict__ part) {
  __shared__ double ss[256], sc[256];
  const int64_t base = (int64_t)blockIdx.x * hw;
  const int64_t len = hw / gridDim.y, beg = (int64_t)blockIdx.y * len;
  double s = 0.0, c = 0.0;
  for (int64_t i = beg + threadIdx.x; i < beg + len; i += blockDim.x) {
    const bool o = mask ? mask[base + i] != 0 : true;
    if (o) {
      s += (double)npix[base + i];
      c += 1.0;
    }
  }
  ss[threadIdx.x] = s;
  sc[threadIdx.x] = c;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) {
      ss[threadIdx.x] += ss[threadIdx.x + k];
      sc[threadIdx.x] += sc[threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* o = part + 2 * ((int64_t)blockIdx.x * gridDim.y + blockIdx.y);
    o[0] = ss[0];
    o[1] = sc[0];
  }
}

// sig2[m] = (sum of N_pix) / (observed count) over map m's slices, in order
__global__ void sigma_final_kernel(const double* __restrict__ part, int slices, int nb,
                                   double* __restrict__ sig2) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nb) return;
  double s = 0.0, c = 0.0;
  for (int k = 0; k < slices; ++k) {
    s += part[2 * ((int64_t)m * slices + k)];
    c += part[2 * ((int64_t)m * slices + k) + 1];
  }
  sig2[m] = c > 0 ? s / c : 1.0;
}

// rowm[r] = mean over the observed pixels of row r (of all maps) of d, or 0
template <class T>
__global__ __launch_bounds__(256) void rowmean_kernel(const T* __restrict__ d,
                                                      const uint8_t* __restrict__ mask, int w,
                                                      double* __restrict__ rowm) {
  __shared__ double ss[256], sc[256];
  const int64_t base = (int64_t)blockIdx.x * w;
  double s = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < w; i += blockDim.x) {
    if (mask ? mask[base + i] != 0 : true) {
      s += (double)d[base + i];
      c += 1.0;
    }
  }
  ss[threadIdx.x] = s;
  sc[threadIdx.x] = c;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) {
      ss[threadIdx.x] += ss[threadIdx.x + k];
      sc[threadIdx.x] += sc[threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) rowm[blockIdx.x] = sc[0] > 0 ? ss[0] / sc[0] : 0.0;
}

// x [P][32] bf16: d/sigma, log(N/sigma^2), mask, row mean of d/sigma, zeros;
// tgt[p] = s/sigma
template <class T>
__global__ void features_kernel(const T* __restrict__ d, const T* __restrict__ npix,
                                const uint8_t* __restrict__ mask, const T* __restrict__ s,
                                const double* __restrict__ sig2, const double* __restrict__ rowm,
                                int w, int64_t hw, int64_t P, uint16_t* __restrict__ x,
                                float* __restrict__ tgt) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * blockDim.x) {
    const double v2 = sig2[p / hw];
    const double sg = sqrt(v2);
    const bool o = mask ? mask[p] != 0 : true;
    float f[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    f[3] = (float)(rowm[p / w] / sg);
    if (o) {
      f[0] = (float)((double)d[p] / sg);
      f[1] = (float)log((double)npix[p] / v2);
      f[2] = 1.f;
    }
    uint4* row = (uint4*)(x + p * kPad);
    row[0] = pack8(f);
    const uint4 z = {0u, 0u, 0u, 0u};
    for (int k = 1; k < kPad / 8; ++k) row[k] = z;
    if (s && tgt) tgt[p] = (float)((double)s[p] / sg);
  }
}

// x [P][32] bf16 from caller features [P][4] float
__global__ void raw_features_kernel(const float* __restrict__ f4, int64_t P, uint16_t* __restrict__ x) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * blockDim.x) {
    float f[8] = {f4[4 * p], f4[4 * p + 1], f4[4 * p + 2], f4[4 * p + 3], 0.f, 0.f, 0.f, 0.f};
    uint4* row = (uint4*)(x + p * kPad);
    row[0] = pack8(f);
    const uint4 z = {0u, 0u, 0u, 0u};
    for (int k = 1; k < kPad / 8; ++k) row[k] = z;
  }
}

// partial sums of (y - t)^2 and the output gradient g [P][32] (channel 0)
__global__ __launch_bounds__(256) void loss_kernel(const float* __restrict__ y, const float* __restrict__ t,
                                                   int64_t P, uint16_t* __restrict__ g,
                                                   double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  const float sc = (float)(2.0 / (double)P);
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * blockDim.x) {
    const float e = y[p] - t[p];
    s += (double)e * (double)e;
    float f[8] = {sc * e, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    uint4* row = (uint4*)(g + p * kPad);
    row[0] = pack8(f);
    const uint4 z = {0u, 0u, 0u, 0u};
    for (int k = 1; k < kPad / 8; ++k) row[k] = z;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// one block of 256 threads: strided partial sums, then a fixed-order tree
__global__ __launch_bounds__(256) void loss_final_kernel(const double* __restrict__ part, int n, int64_t P,
                                                         double* out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0] / (double)P;
}

template <class T>
__global__ void scale_out_kernel(const float* __restrict__ y, const double* __restrict__ sig2,
                                 int64_t hw, int64_t P, T* __restrict__ s) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * blockDim.x)
    s[p] = (T)(sqrt(sig2[p / hw]) * (double)y[p]);
}

// ---------------------------------------------------------------------------
// optimiser and weight packing
// ---------------------------------------------------------------------------

__global__ void adam_kernel(float* __restrict__ prm, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float c1, float c2) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    prm[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  }
}

// w [9][ci][co] float -> w_orig [9][ci][co] and wt [9][co][ci] bfloat16
__global__ void pack_kernel(const float* __restrict__ w, int ci, int co, uint16_t* __restrict__ w_orig,
                            uint16_t* __restrict__ wt) {
  const int64_t n = (int64_t)9 * ci * co;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int t = (int)(i / ((int64_t)ci * co));
    const int rem = (int)(i - (int64_t)t * ci * co);
    const int a = rem / co, b = rem - (rem / co) * co;
    const uint16_t h = f2bf(w[i]);
    w_orig[i] = h;
    wt[((int64_t)t * co + b) * ci + a] = h;
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

wf_status from_hip(hipError_t e) {
  if (e == hipSuccess) return WF_OK;
  if (e == hipErrorOutOfMemory) return WF_ENOMEM;
  return WF_EDEVICE;
}

#define NN_TRY(expr)                                \
  do {                                              \
    hipError_t e_ = (expr);                         \
    if (e_ != hipSuccess) return from_hip(e_);      \
  } while (0)

int grid_for(int64_t n, int block = 256, int cap = 8192) {
  int64_t g = (n + block - 1) / block;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

hipError_t conv(const uint16_t* in, const uint16_t* wt, const float* bias, uint16_t* out, float* out_f32,
                int64_t P, int h, int w, int cin, int cout, bool flip, bool relu, hipStream_t st) {
  ConvArgs a{in, wt, bias, out, out_f32, h, w, cin, cout, flip ? 1 : 0, relu ? 1 : 0, P};
  const unsigned nb = (unsigned)((P + 127) / 128);
  if (cout % 64 == 0)
    hipLaunchKernelGGL(conv_kernel<64>, dim3(nb, cout / 64), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(conv_kernel<32>, dim3(nb, cout / 32), dim3(256), 0, st, a);
  return hipGetLastError();
}

// number of pixel chunks: the largest divisor of the 64-pixel slab count
// that is at most cap, so every chunk is a whole number of slabs
int chunks(int64_t P, int cap) {
  const int64_t slabs = P / 64;
  for (int c = cap; c > 1; --c)
    if (slabs % c == 0) return c;
  return 1;
}
// capacity of the weight-gradient partial buffer, in floats
constexpr int64_t kPartFloats = (int64_t)64 * 9 * 128 * 128;

// pixel chunks of the weight gradient: about 1024 blocks in all (more
// chunks mean more partial sums to add afterwards), within the partial buffer
int wgrad_chunks(int64_t P, int cin, int cout) {
  const int tiles = (cin / 32) * (cout / 32);
  const int64_t want = (1024 + tiles - 1) / tiles;
  const int64_t cap = kPartFloats / ((int64_t)9 * cin * cout);
  return chunks(P, (int)std::min(want, cap));
}

hipError_t wgrad(const uint16_t* in, const uint16_t* g, float* part, float* dw, int64_t P, int h, int w,
                 int cin, int cout, hipStream_t st) {
  const int nch = wgrad_chunks(P, cin, cout);
  WgradArgs a{in, g, part, h, w, cin, cout, P / nch};
  hipLaunchKernelGGL(wgrad_kernel, dim3(nch, (cin / 32) * (cout / 32)), dim3(256), 0, st, a);
  const int64_t n = (int64_t)9 * cin * cout;
  hipLaunchKernelGGL(chunk_sum_kernel, dim3((unsigned)((n + 31) / 32)), dim3(256), 0, st, part, nch, n, dw);
  return hipGetLastError();
}

hipError_t bias_grad(const uint16_t* g, float* part, float* db, int64_t P, int cout, hipStream_t st) {
  const int nch = chunks(P, 256);
  hipLaunchKernelGGL(colsum_kernel, dim3(nch), dim3(256), 0, st, g, cout, P / nch, part);
  hipLaunchKernelGGL(chunk_sum_kernel, dim3((unsigned)((cout + 31) / 32)), dim3(256), 0, st, part, nch,
                     (int64_t)cout, db);
  return hipGetLastError();
}

hipError_t ew(int op, const uint16_t* in, const uint16_t* in2, uint16_t* out, int64_t npix, int oh, int ow,
              int c, hipStream_t st) {
  hipLaunchKernelGGL(ew_kernel, dim3(grid_for(npix * (c / 8))), dim3(256), 0, st, op, in, in2, out, npix,
                     oh, ow, c);
  return hipGetLastError();
}

struct Layer {
  int ci, co;
  int64_t w_off, b_off;
  uint16_t* w_orig = nullptr;  // [9][ci][co]
  uint16_t* wt = nullptr;      // [9][co][ci]
};

std::vector<Layer> layer_table(int64_t* total) {
  std::vector<std::pair<int, int>> s;
  s.push_back({kPad, kChan[0]});
  s.push_back({kChan[0], kChan[0]});
  for (int l = 1; l < kLevels; ++l) {
    s.push_back({kChan[l - 1], kChan[l]});
    s.push_back({kChan[l], kChan[l]});
  }
  for (int l = kLevels - 2; l >= 0; --l) {
    s.push_back({kChan[l + 1], kChan[l]});
    s.push_back({kChan[l], kChan[l]});
  }
  s.push_back({kChan[0], kPad});
  std::vector<Layer> L;
  int64_t off = 0;
  for (auto& pr : s) {
    Layer ly;
    ly.ci = pr.first;
    ly.co = pr.second;
    ly.w_off = off;
    off += (int64_t)9 * ly.ci * ly.co;
    ly.b_off = off;
    off += ly.co;
    L.push_back(ly);
  }
  *total = off;
  return L;
}

struct Net {
  int h = 0, w = 0, nmax = 0, prec = 0;
  std::vector<Layer> L;
  int64_t nparam = 0;
  int adam_t = 0;
  float* prm = nullptr;
  float* grad = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  // activations per level (P_l = nmax * (h >> l) * (w >> l) pixels)
  uint16_t* x = nullptr;                 // features [P_0][32]
  uint16_t* ein[kLevels] = {};           // encoder input (l > 0: pooled)
  uint16_t* eh[kLevels] = {};
  uint16_t* ee[kLevels] = {};
  uint16_t* da[kLevels] = {};            // decoder (l < L-1)
  uint16_t* db[kLevels] = {};
  uint16_t* dc[kLevels] = {};
  uint16_t* du[kLevels] = {};
  uint16_t* gen[kLevels] = {};           // gradient with respect to e_l
  uint16_t* g1[kLevels] = {};            // gradient scratch, 128 channels
  uint16_t* g2[kLevels] = {};
  uint16_t* gy = nullptr;                // [P_0][32]
  float* yf = nullptr;                   // [P_0]
  float* tgt = nullptr;                  // [P_0]
  double* sig2 = nullptr;                // [nmax]
  double* rowm = nullptr;                // [nmax * h] row means of d
  float* part = nullptr;                 // weight-gradient chunk partials
  double* lpart = nullptr;               // loss partials
  double* loss = nullptr;
  double* h_loss = nullptr;              // pinned
  std::vector<void*> owned;
};

void free_net(Net* n) {
  for (void* p : n->owned)
    if (p) (void)hipFree(p);
  if (n->h_loss) (void)hipHostFree(n->h_loss);
  delete n;
}

template <class P>
wf_status nalloc(Net* n, P** ptr, size_t bytes) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) return from_hip(e);
  n->owned.push_back(q);
  *ptr = (P*)q;
  return WF_OK;
}

wf_status create_net(const wf_nn_shape* s, Net** out) {
  Net* n = new (std::nothrow) Net();
  if (!n) return WF_ENOMEM;
  n->h = s->h;
  n->w = s->w;
  n->nmax = s->batch_max;
  n->prec = s->precision;
  n->L = layer_table(&n->nparam);
  wf_status st = WF_OK;
#define NA(ptr, bytes)                                  \
  if ((st = nalloc(n, &(ptr), (bytes))) != WF_OK) {     \
    free_net(n);                                        \
    return st;                                          \
  }
  NA(n->prm, n->nparam * 4);
  NA(n->grad, n->nparam * 4);
  NA(n->m, n->nparam * 4);
  NA(n->v, n->nparam * 4);
  for (auto& ly : n->L) {
    NA(ly.w_orig, (size_t)9 * ly.ci * ly.co * 2);
    NA(ly.wt, (size_t)9 * ly.ci * ly.co * 2);
  }
  const int64_t P0 = (int64_t)n->nmax * n->h * n->w;
  NA(n->x, P0 * kPad * 2);
  for (int l = 0; l < kLevels; ++l) {
    const int64_t Pl = P0 >> (2 * l);
    const int c = kChan[l];
    const int cprev = l > 0 ? kChan[l - 1] : kPad;
    if (l > 0) NA(n->ein[l], Pl * cprev * 2);
    NA(n->eh[l], Pl * c * 2);
    NA(n->ee[l], Pl * c * 2);
    if (l < kLevels - 1) {
      NA(n->da[l], Pl * kChan[l + 1] * 2);
      NA(n->db[l], Pl * c * 2);
      NA(n->dc[l], Pl * c * 2);
      NA(n->du[l], Pl * c * 2);
    }
    NA(n->gen[l], Pl * c * 2);
    NA(n->g1[l], Pl * 128 * 2);
    NA(n->g2[l], Pl * 128 * 2);
  }
  n->ein[0] = n->x;
  NA(n->gy, P0 * kPad * 2);
  NA(n->yf, P0 * 4);
  NA(n->tgt, P0 * 4);
  NA(n->sig2, n->nmax * 8);
  NA(n->rowm, (size_t)n->nmax * n->h * 8);
  NA(n->part, (size_t)kPartFloats * 4);
  NA(n->lpart, 1024 * 8);
  NA(n->loss, 8);
#undef NA
  hipError_t e = hipHostMalloc((void**)&n->h_loss, 8, hipHostMallocDefault);
  if (e == hipSuccess) e = hipMemset(n->prm, 0, n->nparam * 4);
  if (e == hipSuccess) e = hipMemset(n->m, 0, n->nparam * 4);
  if (e == hipSuccess) e = hipMemset(n->v, 0, n->nparam * 4);
  if (e != hipSuccess) {
    free_net(n);
    return from_hip(e);
  }
  *out = n;
  return WF_OK;
}

hipError_t pack_all(Net* n, hipStream_t st) {
  for (auto& ly : n->L)
    hipLaunchKernelGGL(pack_kernel, dim3(grid_for((int64_t)9 * ly.ci * ly.co)), dim3(256), 0, st,
                       n->prm + ly.w_off, ly.ci, ly.co, ly.w_orig, ly.wt);
  return hipGetLastError();
}

// forward pass of nb maps from n->x into n->yf
wf_status forward(Net* n, int nb, hipStream_t st) {
  const int64_t P0 = (int64_t)nb * n->h * n->w;
  int k = 0;
  for (int l = 0; l < kLevels; ++l) {
    const int64_t Pl = P0 >> (2 * l);
    const int hl = n->h >> l, wl = n->w >> l;
    const int cin = l > 0 ? kChan[l - 1] : kPad;
    if (l > 0) NN_TRY(ew(EW_POOL, n->ee[l - 1], nullptr, n->ein[l], Pl, hl, wl, cin, st));
    const Layer& a = n->L[k];
    const Layer& b = n->L[k + 1];
    NN_TRY(conv(n->ein[l], a.wt, n->prm + a.b_off, n->eh[l], nullptr, Pl, hl, wl, a.ci, a.co, false, true, st));
    NN_TRY(conv(n->eh[l], b.wt, n->prm + b.b_off, n->ee[l], nullptr, Pl, hl, wl, b.ci, b.co, false, true, st));
    k += 2;
  }
  const uint16_t* u = n->ee[kLevels - 1];
  for (int l = kLevels - 2; l >= 0; --l) {
    const int64_t Pl = P0 >> (2 * l);
    const int hl = n->h >> l, wl = n->w >> l;
    const Layer& a = n->L[k];
    const Layer& b = n->L[k + 1];
    NN_TRY(ew(EW_UP, u, nullptr, n->da[l], Pl, hl, wl, kChan[l + 1], st));
    NN_TRY(conv(n->da[l], a.wt, n->prm + a.b_off, n->db[l], nullptr, Pl, hl, wl, a.ci, a.co, false, true, st));
    NN_TRY(ew(EW_ADD, n->db[l], n->ee[l], n->dc[l], Pl, hl, wl, kChan[l], st));
    NN_TRY(conv(n->dc[l], b.wt, n->prm + b.b_off, n->du[l], nullptr, Pl, hl, wl, b.ci, b.co, false, true, st));
    u = n->du[l];
    k += 2;
  }
  const Layer& o = n->L[k];
  NN_TRY(conv(u, o.wt, n->prm + o.b_off, nullptr, n->yf, P0, n->h, n->w, o.ci, o.co, false, false, st));
  return WF_OK;
}

// loss against n->tgt and the gradient of every parameter into n->grad
wf_status backward(Net* n, int nb, hipStream_t st) {
  const int64_t P0 = (int64_t)nb * n->h * n->w;
  const int nlp = grid_for(P0, 256, 1024);
  hipLaunchKernelGGL(loss_kernel, dim3(nlp), dim3(256), 0, st, n->yf, n->tgt, P0, n->gy, n->lpart);
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, st, n->lpart, nlp, P0, n->loss);
  NN_TRY(hipGetLastError());
  int k = kLayers - 1;
  {
    const Layer& o = n->L[k];
    NN_TRY(wgrad(n->du[0], n->gy, n->part, n->grad + o.w_off, P0, n->h, n->w, o.ci, o.co, st));
    NN_TRY(bias_grad(n->gy, n->part, n->grad + o.b_off, P0, o.co, st));
    NN_TRY(conv(n->gy, o.w_orig, nullptr, n->g1[0], nullptr, P0, n->h, n->w, o.co, o.ci, true, false, st));
  }
  // g1[0] holds the gradient with respect to u_0
  uint16_t* gu = n->g1[0];
  k -= 1;
  for (int l = 0; l < kLevels - 1; ++l) {
    const int64_t Pl = P0 >> (2 * l);
    const int hl = n->h >> l, wl = n->w >> l;
    const Layer& b = n->L[k];      // second convolution of decoder level l
    const Layer& a = n->L[k - 1];  // first one
    const int c = kChan[l];
    NN_TRY(ew(EW_RELU_BWD, gu, n->du[l], gu, Pl, hl, wl, c, st));
    NN_TRY(wgrad(n->dc[l], gu, n->part, n->grad + b.w_off, Pl, hl, wl, b.ci, b.co, st));
    NN_TRY(bias_grad(gu, n->part, n->grad + b.b_off, Pl, b.co, st));
    // gradient with respect to c_l = b_l + e_l goes to the skip and to b_l
    NN_TRY(conv(gu, b.w_orig, nullptr, n->gen[l], nullptr, Pl, hl, wl, b.co, b.ci, true, false, st));
    uint16_t* gb = (gu == n->g1[l]) ? n->g2[l] : n->g1[l];
    NN_TRY(ew(EW_RELU_BWD, n->gen[l], n->db[l], gb, Pl, hl, wl, c, st));
    NN_TRY(wgrad(n->da[l], gb, n->part, n->grad + a.w_off, Pl, hl, wl, a.ci, a.co, st));
    NN_TRY(bias_grad(gb, n->part, n->grad + a.b_off, Pl, a.co, st));
    uint16_t* ga = (gb == n->g1[l]) ? n->g2[l] : n->g1[l];
    NN_TRY(conv(gb, a.w_orig, nullptr, ga, nullptr, Pl, hl, wl, a.co, a.ci, true, false, st));
    // adjoint of the upsampling: gradient with respect to u_{l+1}
    NN_TRY(ew(EW_UP_ADJ, ga, nullptr, n->g1[l + 1], Pl >> 2, hl / 2, wl / 2, kChan[l + 1], st));
    gu = n->g1[l + 1];
    k -= 2;
  }
  // gu: gradient with respect to e_{L-1}
  NN_TRY(hipMemcpyAsync(n->gen[kLevels - 1], gu, (size_t)(P0 >> (2 * (kLevels - 1))) * kChan[kLevels - 1] * 2,
                        hipMemcpyDeviceToDevice, st));
  for (int l = kLevels - 1; l >= 0; --l) {
    const int64_t Pl = P0 >> (2 * l);
    const int hl = n->h >> l, wl = n->w >> l;
    const Layer& a = n->L[2 * l];
    const Layer& b = n->L[2 * l + 1];
    const int c = kChan[l];
    NN_TRY(ew(EW_RELU_BWD, n->gen[l], n->ee[l], n->gen[l], Pl, hl, wl, c, st));
    NN_TRY(wgrad(n->eh[l], n->gen[l], n->part, n->grad + b.w_off, Pl, hl, wl, b.ci, b.co, st));
    NN_TRY(bias_grad(n->gen[l], n->part, n->grad + b.b_off, Pl, b.co, st));
    NN_TRY(conv(n->gen[l], b.w_orig, nullptr, n->g1[l], nullptr, Pl, hl, wl, b.co, b.ci, true, false, st));
    NN_TRY(ew(EW_RELU_BWD, n->g1[l], n->eh[l], n->g1[l], Pl, hl, wl, c, st));
    NN_TRY(wgrad(n->ein[l], n->g1[l], n->part, n->grad + a.w_off, Pl, hl, wl, a.ci, a.co, st));
    NN_TRY(bias_grad(n->g1[l], n->part, n->grad + a.b_off, Pl, a.co, st));
    if (l > 0) {
      NN_TRY(conv(n->g1[l], a.w_orig, nullptr, n->g2[l], nullptr, Pl, hl, wl, a.co, a.ci, true, false, st));
      NN_TRY(ew(EW_ADD_POOL_ADJ, n->g2[l], nullptr, n->gen[l - 1], Pl << 2, hl * 2, wl * 2, kChan[l - 1], st));
    }
  }
  return WF_OK;
}

template <class T>
wf_status prepare(Net* n, int nb, const void* d, const void* npix, const uint8_t* mask, const void* s,
                  hipStream_t st) {
  const int64_t hw = (int64_t)n->h * n->w, P0 = nb * hw;
  constexpr int kSlices = 32;  // divides every supported map size
  hipLaunchKernelGGL(sigma_kernel<T>, dim3(nb, kSlices), dim3(256), 0, st, (const T*)npix, mask, hw,
                     (double*)n->part);
  hipLaunchKernelGGL(sigma_final_kernel, dim3((nb + 63) / 64), dim3(64), 0, st, (const double*)n->part,
                     kSlices, nb, n->sig2);
  hipLaunchKernelGGL(rowmean_kernel<T>, dim3(nb * n->h), dim3(256), 0, st, (const T*)d, mask, n->w, n->rowm);
  hipLaunchKernelGGL(features_kernel<T>, dim3(grid_for(P0)), dim3(256), 0, st, (const T*)d, (const T*)npix,
                     mask, (const T*)s, n->sig2, n->rowm, n->w, hw, P0, n->x, s ? n->tgt : nullptr);
  NN_TRY(hipGetLastError());
  return WF_OK;
}

wf_status adam(Net* n, float lr, hipStream_t st) {
  n->adam_t += 1;
  const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, n->adam_t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, n->adam_t)));
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n->nparam)), dim3(256), 0, st, n->prm, n->grad, n->m, n->v,
                     n->nparam, lr, c1, c2);
  NN_TRY(hipGetLastError());
  NN_TRY(pack_all(n, st));
  return WF_OK;
}

wf_status read_loss(Net* n, double* loss, hipStream_t st) {
  NN_TRY(hipMemcpyAsync(n->h_loss, n->loss, 8, hipMemcpyDeviceToHost, st));
  NN_TRY(hipStreamSynchronize(st));
  if (loss) *loss = *n->h_loss;
  return WF_OK;
}

bool shape_ok(int h, int w) {
  auto p2 = [](int v) { return v >= 64 && v <= 2048 && (v & (v - 1)) == 0; };
  return p2(h) && p2(w);
}

}  // namespace wfnn

using namespace wfnn;

extern "C" {

int64_t wf_nn_param_count(void) {
  int64_t total = 0;
  (void)layer_table(&total);
  return total;
}

wf_status wf_nn_create(const wf_nn_shape* s, void** out) {
  if (!s || !out) return WF_EINVAL;
  *out = nullptr;
  if (s->precision != WF_F32 && s->precision != WF_F64) return WF_EINVAL;
  if (s->batch_max < 1 || s->batch_max > 4096) return WF_EINVAL;
  if (!shape_ok(s->h, s->w)) return WF_EUNSUPPORTED;
  Net* n = nullptr;
  wf_status st = create_net(s, &n);
  if (st == WF_OK) *out = n;
  return st;
}

void wf_nn_destroy(void* net) {
  if (net) free_net((Net*)net);
}

wf_status wf_nn_set_params(void* net, const float* params, hipStream_t stream) {
  Net* n = (Net*)net;
  if (!n || !params) return WF_EINVAL;
  NN_TRY(hipMemcpyAsync(n->prm, params, n->nparam * 4, hipMemcpyDeviceToDevice, stream));
  NN_TRY(hipMemsetAsync(n->m, 0, n->nparam * 4, stream));
  NN_TRY(hipMemsetAsync(n->v, 0, n->nparam * 4, stream));
  n->adam_t = 0;
  NN_TRY(pack_all(n, stream));
  NN_TRY(hipStreamSynchronize(stream));
  return WF_OK;
}

wf_status wf_nn_get_params(void* net, float* params, hipStream_t stream) {
  Net* n = (Net*)net;
  if (!n || !params) return WF_EINVAL;
  NN_TRY(hipMemcpyAsync(params, n->prm, n->nparam * 4, hipMemcpyDeviceToDevice, stream));
  NN_TRY(hipStreamSynchronize(stream));
  return WF_OK;
}

wf_status wf_nn_predict(void* net, int32_t nb, const void* d, const void* n_pix, const uint8_t* mask,
                        void* s_out, hipStream_t stream) {
  Net* n = (Net*)net;
  if (!n || !d || !n_pix || !s_out || nb < 1 || nb > n->nmax) return WF_EINVAL;
  const int64_t hw = (int64_t)n->h * n->w, P0 = nb * hw;
  wf_status st = n->prec == WF_F64 ? prepare<double>(n, nb, d, n_pix, mask, nullptr, stream)
                                   : prepare<float>(n, nb, d, n_pix, mask, nullptr, stream);
  if (st != WF_OK) return st;
  st = forward(n, nb, stream);
  if (st != WF_OK) return st;
  if (n->prec == WF_F64)
    hipLaunchKernelGGL(scale_out_kernel<double>, dim3(grid_for(P0)), dim3(256), 0, stream, n->yf, n->sig2, hw,
                       P0, (double*)s_out);
  else
    hipLaunchKernelGGL(scale_out_kernel<float>, dim3(grid_for(P0)), dim3(256), 0, stream, n->yf, n->sig2, hw,
                       P0, (float*)s_out);
  NN_TRY(hipGetLastError());
  NN_TRY(hipStreamSynchronize(stream));
  return WF_OK;
}

wf_status wf_nn_train_step(void* net, int32_t nb, const void* d, const void* n_pix, const uint8_t* mask,
                           const void* s_target, float lr, double* loss, hipStream_t stream) {
  Net* n = (Net*)net;
  if (!n || !d || !n_pix || !s_target || nb < 1 || nb > n->nmax) return WF_EINVAL;
  if (!(lr > 0.f) || !std::isfinite(lr)) return WF_EINVAL;
  wf_status st = n->prec == WF_F64 ? prepare<double>(n, nb, d, n_pix, mask, s_target, stream)
                                   : prepare<float>(n, nb, d, n_pix, mask, s_target, stream);
  if (st != WF_OK) return st;
  if ((st = forward(n, nb, stream)) != WF_OK) return st;
  if ((st = backward(n, nb, stream)) != WF_OK) return st;
  if ((st = adam(n, lr, stream)) != WF_OK) return st;
  return read_loss(n, loss, stream);
}

wf_status wf_nn_forward_features(void* net, int32_t nb, const float* x, float* y, hipStream_t stream) {
  Net* n = (Net*)net;
  if (!n || !x || !y || nb < 1 || nb > n->nmax) return WF_EINVAL;
  const int64_t P0 = (int64_t)nb * n->h * n->w;
  hipLaunchKernelGGL(raw_features_kernel, dim3(grid_for(P0)), dim3(256), 0, stream, x, P0, n->x);
  NN_TRY(hipGetLastError());
  wf_status st = forward(n, nb, stream);
  if (st != WF_OK) return st;
  NN_TRY(hipMemcpyAsync(y, n->yf, P0 * 4, hipMemcpyDeviceToDevice, stream));
  NN_TRY(hipStreamSynchronize(stream));
  return WF_OK;
}

wf_status wf_nn_gradient_features(void* net, int32_t nb, const float* x, const float* target, float* grad,
                                  double* loss, hipStream_t stream) {
  Net* n = (Net*)net;
  if (!n || !x || !target || !grad || nb < 1 || nb > n->nmax) return WF_EINVAL;
  const int64_t P0 = (int64_t)nb * n->h * n->w;
  hipLaunchKernelGGL(raw_features_kernel, dim3(grid_for(P0)), dim3(256), 0, stream, x, P0, n->x);
  NN_TRY(hipGetLastError());
  NN_TRY(hipMemcpyAsync(n->tgt, target, P0 * 4, hipMemcpyDeviceToDevice, stream));
  wf_status st = forward(n, nb, stream);
  if (st != WF_OK) return st;
  if ((st = backward(n, nb, stream)) != WF_OK) return st;
  NN_TRY(hipMemcpyAsync(grad, n->grad, n->nparam * 4, hipMemcpyDeviceToDevice, stream));
  return read_loss(n, loss, stream);
}

wf_status wf_nn_conv3x3(int32_t mode, int32_t nb, int32_t h, int32_t w, int32_t ci, int32_t co,
                        const uint16_t* in, const uint16_t* wt, const float* b, const uint16_t* g, void* out,
                        hipStream_t stream) {
  if (mode < 0 || mode > 3 || nb < 1 || !in || !out) return WF_EINVAL;
  if (ci < 32 || co < 32 || ci % 32 || co % 32 || ci > 128 || co > 128) return WF_EINVAL;
  if (h < 8 || w < 8 || (h & (h - 1)) || (w & (w - 1))) return WF_EINVAL;
  const int64_t P = (int64_t)nb * h * w;
  if (P % 64) return WF_EINVAL;
  if (mode == 3) {
    if (!g) return WF_EINVAL;
    float* part = nullptr;
    NN_TRY(hipMalloc((void**)&part, (size_t)wgrad_chunks(P, ci, co) * 9 * ci * co * 4));
    hipError_t e = wgrad(in, g, part, (float*)out, P, h, w, ci, co, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    (void)hipFree(part);
    return from_hip(e);
  }
  if (!wt) return WF_EINVAL;
  if (mode == 2) {
    // input adjoint: the [9][ci][co] weights are already [tap][out = ci][reduction = co]
    NN_TRY(conv(in, wt, nullptr, (uint16_t*)out, nullptr, P, h, w, co, ci, true, false, stream));
    NN_TRY(hipStreamSynchronize(stream));
    return WF_OK;
  }
  // forward needs [9][co][ci]
  uint16_t* tmp = nullptr;
  NN_TRY(hipMalloc((void**)&tmp, (size_t)9 * ci * co * 2));
  std::vector<uint16_t> hw_((size_t)9 * ci * co), ht((size_t)9 * ci * co);
  hipError_t e = hipMemcpyAsync(hw_.data(), wt, hw_.size() * 2, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e == hipSuccess) {
    for (int t = 0; t < 9; ++t)
      for (int a = 0; a < ci; ++a)
        for (int c = 0; c < co; ++c) ht[((size_t)t * co + c) * ci + a] = hw_[((size_t)t * ci + a) * co + c];
    e = hipMemcpyAsync(tmp, ht.data(), ht.size() * 2, hipMemcpyHostToDevice, stream);
  }
  if (e == hipSuccess) e = conv(in, tmp, b, (uint16_t*)out, nullptr, P, h, w, ci, co, false, mode == 1, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  (void)hipFree(tmp);
  return from_hip(e);
}

}  // extern "C"
