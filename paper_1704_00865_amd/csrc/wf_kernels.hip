// Device code of the multi-messenger Wiener filter (gfx950).
//
// One sweep of the iteration (Section 2 equations, data side first) is two
// launches over a transit buffer B that holds a field transformed along x
// only (a "row spectrum", half spectrum in k_x):
//
//   row kernel    per band of kTR rows: inverse row FFT of d_1's row spectrum
//                 -> pixel update t_2 = [T_2 d + Nbar_2 d_1] / (Nbar_2 + T_2)
//                 (eqn 2mess_t1 form, white level) -> forward row FFT of t_2.
//   column kernel per group of kTC half-spectrum columns: forward column FFT
//                 -> the Fourier-side chain per mode (eqns 2mess_d0, 2mess_t0,
//                 2mess_s and their stripe-level analogues) -> inverse
//                 column FFT of d_1.
//
// B is tiled [y/kTR][kx/kTC][kTR][kTC] so that both kernels read and write it
// in contiguous runs (a row band is one contiguous block; a column group is
// kTR*kTC*sizeof(complex) contiguous per tile).  Fourier-side state and
// per-mode coefficients are stored column-major [kx][ky] so the column kernel
// streams them with consecutive threads on consecutive ky.
//
// Fields are stored unnormalised in Fourier space (forward transforms carry
// no factor); the inverse's 1/(nx ny) is applied once in the row kernel.  All
// messenger covariances are multiples of the identity, so the update
// coefficients do not depend on that scale.
//
// The residual monitor starts from the stored state: x = S^-1 s =
// t_A / (S_chain + T_A) and y = (S + N_Fourier) x are formed per mode in
// float64, rounded once to the path's precision and taken to pixel space by
// inverse transforms of that precision; Delta d = y + N_white x - d
// (Section 2) is then summed in float64 over observed pixels, and x^2 over
// masked ones.  During a solve the column transforms of x and y run at the
// end of each chunk's last column sweep (the J variant) and only the row pass
// is a launch of its own; the monitor's column kernel serves the output and
// the refinement.  A one-block controller applies the cooling schedule on
// the device.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "wf_fft.hpp"
#include "wf_kernels.hpp"

// The build compiles this file three times, with WF_PART = 1 (float32
// kernels in the default tiling and the precision-free ones), 2 (float64
// kernels) and 4 (float32 kernels in the other tilings), so that the parts
// compile in parallel; without a definition everything is built.
#ifndef WF_PART
#define WF_PART 7
#endif

namespace wf {

template <int N, int TC>
struct KP {
  static constexpr int value = ((N / 2 + 1 + TC - 1) / TC) * TC;
};

// 1/x: the hardware reciprocal (within 1 ulp) in float32, where an IEEE
// division costs about ten instructions and the sweep's updates are about a
// quarter of the column kernel's arithmetic; a correctly rounded division in
// float64
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }

template <class T>
__device__ __forceinline__ T white_update(T d, T nb, T d1, T lt) {
  // masked pixel (Nbar = inf, stored as a negative sentinel): t_2 = d_1
  if (nb < (T)0) return d1;
  return d1 + (lt * rcp(nb + lt)) * (d - d1);
}

// The joint objective J_lambda (eqn 2mess_prob, the quadratic form that the
// sweep minimises one field at a time) of the state after a sweep, summed in
// float64 from the values the sweep computed:
//   |t_0|^2 / (S_chain + T_0)           (the s terms, s = S_c (S_c + T_0)^-1 t_0)
//   + sum over links of |difference|^2 / covariance,
// the Fourier-diagonal links per mode in the column kernel, the white level's
// link to the data per pixel in the row kernel.  A masked pixel (infinite
// Nbar) adds nothing, nor does one with Nbar_2 = 0, whose exact update puts
// t_2 on the data.
template <class T>
__device__ __forceinline__ double white_term(T d, T nb, T t2) {
  if (!(nb > (T)0)) return 0.0;
  const double r = (double)d - (double)t2;
  return r * r / (double)nb;
}

// wave sum; lane 0 leaves it in sh[wave]
__device__ __forceinline__ void wave_partial(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
}

// the block's wave partials in a fixed order (after a barrier)
__device__ __forceinline__ double sum_partials(const double* sh, int nthreads) {
  double r = 0.0;
  for (int w = 0; w < (nthreads + 63) >> 6; ++w) r += sh[w];
  return r;
}

// ---------------------------------------------------------------------------
// block reductions (wave64 shuffles, then one LDS round)
// ---------------------------------------------------------------------------
enum RedOp { RED_SUM = 0, RED_MIN = 1, RED_MAX = 2 };

template <int OP>
__device__ __forceinline__ double red2(double a, double b) {
  if constexpr (OP == RED_SUM) return a + b;
  if constexpr (OP == RED_MIN) return fmin(a, b);
  return fmax(a, b);
}

template <int OP>
__device__ double block_reduce(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = red2<OP>(v, __shfl_xor(v, off, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = sh[0];
  for (int w = 1; w < nw; ++w) r = red2<OP>(r, sh[w]);
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// setup: validation statistics
// ---------------------------------------------------------------------------
// Four consecutive pixels 4 i4 .. 4 i4 + 3 (n is a multiple of 4: every
// side is at least 64), in one vector access when VEC (the caller's arrays
// are aligned to it), else element by element; the values and their order
// are the same either way.
template <class T>
using vec4 = T __attribute__((ext_vector_type(4)));
typedef unsigned char u8x4 __attribute__((ext_vector_type(4)));
template <bool VEC, class T>
__device__ __forceinline__ vec4<T> load4(const T* __restrict__ p, int64_t i4) {
  if constexpr (VEC) return reinterpret_cast<const vec4<T>*>(p)[i4];
  else return vec4<T>{p[4 * i4], p[4 * i4 + 1], p[4 * i4 + 2], p[4 * i4 + 3]};
}
template <bool VEC, class T>
__device__ __forceinline__ void store4(T* __restrict__ p, int64_t i4, vec4<T> v) {
  if constexpr (VEC) {
    reinterpret_cast<vec4<T>*>(p)[i4] = v;
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u) p[4 * i4 + u] = v[u];
  }
}

// per block: n_obs, min N_pix(obs), max N_pix(obs), sum d^2 (obs),
//            #non-finite (d or N_pix on observed), #N_pix <= 0 (observed)
template <class T, bool VEC>
__global__ __launch_bounds__(256) void stats_pixels_kernel(const T* __restrict__ d,
                                                           const T* __restrict__ npix,
                                                           const uint8_t* __restrict__ mask,
                                                           int64_t n, double* __restrict__ part) {
  __shared__ double sh[16];
  double cnt = 0, mn = INFINITY, mx = -INFINITY, s2 = 0, bad = 0, badn = 0;
  for (int64_t i4 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i4 < n / 4;
       i4 += (int64_t)gridDim.x * blockDim.x) {
    const vec4<T> dq = load4<VEC>(d, i4), nq = load4<VEC>(npix, i4);
    const u8x4 mq = mask ? load4<VEC>(mask, i4) : u8x4{1, 1, 1, 1};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (mq[u] == 0) continue;
      const double dv = (double)dq[u], nv = (double)nq[u];
      cnt += 1;
      if (!isfinite(dv) || !isfinite(nv)) {
        bad += 1;
        continue;
      }
      if (!(nv > 0)) badn += 1;
      mn = fmin(mn, nv);
      mx = fmax(mx, nv);
      s2 += dv * dv;
    }
  }
  cnt = block_reduce<RED_SUM>(cnt, sh);
  mn = block_reduce<RED_MIN>(mn, sh);
  mx = block_reduce<RED_MAX>(mx, sh);
  s2 = block_reduce<RED_SUM>(s2, sh);
  bad = block_reduce<RED_SUM>(bad, sh);
  badn = block_reduce<RED_SUM>(badn, sh);
  if (threadIdx.x == 0) {
    double* o = part + 8 * blockIdx.x;
    o[0] = cnt; o[1] = mn; o[2] = mx; o[3] = s2; o[4] = bad; o[5] = badn; o[6] = 0; o[7] = 0;
  }
}

// per block: min S, min P_1/f, min over modes of (P_1/f + nx P_st on k_x = 0),
//            #bad S, #bad P_1/f, #bad P_st (non-finite or negative),
//            #values that break the evenness of the real columns
template <class T>
__global__ __launch_bounds__(256) void stats_spectra_kernel(const T* __restrict__ sk,
                                                            const T* __restrict__ poof,
                                                            const T* __restrict__ pst,
                                                            int ny, int nx, double* __restrict__ part) {
  __shared__ double sh[16];
  const int nh = nx / 2 + 1;
  double ms = INFINITY, mo = INFINITY, mf = INFINITY, bs = 0, bo = 0, bp = 0, asym = 0;
  // block b takes rows b, b + gridDim.x, ...; its threads stride along a row
  for (int ky = blockIdx.x; ky < ny; ky += gridDim.x)
  for (int kx = threadIdx.x; kx < nh; kx += blockDim.x) {
    const int64_t i = (int64_t)ky * nh + kx;
    const double s = (double)sk[i];
    if (!isfinite(s) || s < 0) bs += 1;
    ms = fmin(ms, s);
    double f = 0;
    if (poof) {
      const double o = (double)poof[i];
      if (isnan(o) || o < 0) bo += 1;  // +inf is allowed: a projected mode
      mo = fmin(mo, o);
      f = o;
    }
    if (pst && kx == 0) {
      const double p = (double)pst[ky];
      if (!isfinite(p) || p < 0) bp += 1;
      f += (double)nx * p;
    }
    mf = fmin(mf, f);
    // spectra of a real field are even in k: on the real columns k_x = 0 and
    // nx/2 the value at -k_y must equal the one at k_y (and P_st is even)
    if ((kx == 0 || kx == nx / 2) && ky > 0 && ky < ny / 2) {
      const int64_t im = (int64_t)(ny - ky) * nh + kx;
      if (!(sk[im] == sk[i])) asym += 1;
      if (poof && !(poof[im] == poof[i])) asym += 1;
      if (pst && kx == 0 && !(pst[ny - ky] == pst[ky])) asym += 1;
    }
  }
  ms = block_reduce<RED_MIN>(ms, sh);
  mo = block_reduce<RED_MIN>(mo, sh);
  mf = block_reduce<RED_MIN>(mf, sh);
  bs = block_reduce<RED_SUM>(bs, sh);
  bo = block_reduce<RED_SUM>(bo, sh);
  bp = block_reduce<RED_SUM>(bp, sh);
  asym = block_reduce<RED_SUM>(asym, sh);
  if (threadIdx.x == 0) {
    double* o = part + 8 * blockIdx.x;
    o[0] = ms; o[1] = mo; o[2] = mf; o[3] = bs; o[4] = bo; o[5] = bp; o[6] = asym; o[7] = 0;
  }
}

// reduce per-block statistics in a fixed order; ops[j] says how column j
// combines (sum / min / max).  Wave j reduces column j: lane l takes blocks
// l, l + 64, ..., then the lanes combine in a fixed butterfly.
#if WF_PART & 1
__global__ __launch_bounds__(512) void stats_finalize_kernel(const double* __restrict__ part, int nblk,
                                                             int4 ops_lo, int4 ops_hi,
                                                             double* __restrict__ out) {
  const int j = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ops[8] = {ops_lo.x, ops_lo.y, ops_lo.z, ops_lo.w, ops_hi.x, ops_hi.y, ops_hi.z, ops_hi.w};
  const int op = ops[j];
  auto comb = [op](double a, double b) {
    return op == RED_SUM ? a + b : (op == RED_MIN ? fmin(a, b) : fmax(a, b));
  };
  double r = op == RED_SUM ? 0.0 : (op == RED_MIN ? INFINITY : -INFINITY);
  for (int b = lane; b < nblk; b += 64) r = comb(r, part[8 * b + j]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) r = comb(r, __shfl_xor(r, off, 64));
  if (lane == 0) out[j] = r;
}
#else
__global__ __launch_bounds__(512) void stats_finalize_kernel(const double* __restrict__ part, int nblk,
                                                             int4 ops_lo, int4 ops_hi,
                                                             double* __restrict__ out);
#endif

// ---------------------------------------------------------------------------
// setup: per-pixel and per-mode coefficients
// ---------------------------------------------------------------------------
// Also zeroes zb (n values: the transit buffer, whose nx/2 complex columns
// per row hold as many values as the map has pixels) for the zero start.
template <class T, bool VEC>
__global__ __launch_bounds__(256) void prep_pixels_kernel(const T* __restrict__ npix,
                                                          const uint8_t* __restrict__ mask, int64_t n,
                                                          double sub, T* __restrict__ nbar2,
                                                          T* __restrict__ zb) {
  for (int64_t i4 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i4 < n / 4;
       i4 += (int64_t)gridDim.x * blockDim.x) {
    const vec4<T> nq = load4<VEC>(npix, i4);
    const u8x4 mq = mask ? load4<VEC>(mask, i4) : u8x4{1, 1, 1, 1};
    vec4<T> o;
#pragma unroll
    for (int u = 0; u < 4; ++u) o[u] = mq[u] != 0 ? (T)((double)nq[u] - sub) : (T)(-1);
    store4<true>(nbar2, i4, o);  // the context's own arrays: aligned
    store4<true>(zb, i4, vec4<T>{(T)0, (T)0, (T)0, (T)0});
  }
}

// column-major [kx][ky] per-mode arrays:
//   sc  = covariance at the signal end of the chain (S, or S + N_F for the
//         augmented chain, plus the lent floor when it sits in N_F)
//   nbA = Nbar of the array level = N_A - tau_A
//   sy  = S + N_1/f + N_stripe (true Fourier noise; the white level is added
//         in pixel space by the monitor)
//   sig = S


// One block per 32 x 32 tile of modes: the caller's row-major [ky][kx]
// spectra are read along k_x and staged in LDS, and the outputs are written
// along k_y, so that both sides are coalesced.
constexpr int kPrepTile = 32;

// Also zeroes the three per-mode state arrays z0, z1, z2 (complex, same
// layout) for the zero start.
template <class T>
__global__ __launch_bounds__(256) void prep_spectra_kernel(const T* __restrict__ sk,
                                                           const T* __restrict__ poof,
                                                           const T* __restrict__ pst, PrepSpecArgs a,
                                                           T* __restrict__ sc, T* __restrict__ nbA,
                                                           T* __restrict__ sy, T* __restrict__ sig,
                                                           cx<T>* __restrict__ z0,
                                                           cx<T>* __restrict__ z1,
                                                           cx<T>* __restrict__ z2) {
  constexpr int TT = kPrepTile;
  __shared__ T ls[TT][TT + 1], lo[TT][TT + 1];  // [ky][kx] within the tile
  const int nh = a.nx / 2 + 1;
  const int kx0 = blockIdx.x * TT, ky0 = blockIdx.y * TT;
  const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;
  constexpr int RS = 256 / TT;  // rows per step
#pragma unroll
  for (int r = ty; r < TT; r += RS) {
    const int ky = ky0 + r, kx = kx0 + tx;
    if (ky < a.ny && kx < nh) {
      const int64_t i = (int64_t)ky * nh + kx;
      ls[r][tx] = sk[i];
      lo[r][tx] = a.has_oof ? poof[i] : (T)0;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = ty; r < TT; r += RS) {
    const int kx = kx0 + r, ky = ky0 + tx;
    if (ky >= a.ny || kx >= nh) continue;
    const int64_t j = (int64_t)kx * a.ny + ky;  // column-major output index
    const double s = (double)ls[tx][r];
    double o = (double)lo[tx][r];
    if (isinf(o)) o = kInfiniteCov;  // projected mode (see kInfiniteCov)
    const double st = (a.has_st && kx == 0) ? (double)a.nx * (double)pst[ky] : 0.0;
    const double nf = o + st;
    sc[j] = (T)(a.sc_adds_nf ? s + nf + a.phi_nf : s);
    if (a.nbA_kind == 1) nbA[j] = (T)(o - a.tauA);
    else if (a.nbA_kind == 2) nbA[j] = (T)(nf + a.phi_nf - a.tauA);
    sy[j] = (T)(s + nf);
    sig[j] = (T)s;
    const cx<T> zero = {(T)0, (T)0};
    z0[j] = zero;
    z1[j] = zero;
    z2[j] = zero;
  }
}

// ---------------------------------------------------------------------------
// transit-buffer tiling
// ---------------------------------------------------------------------------
// B holds nx/2 complex columns per row: column 0 packs the two real-valued
// columns k_x = 0 (re) and k_x = nx/2 (im) of the row spectrum, so the
// column pass works on exactly nx/2 complex columns.  Layout:
// [y / TR][kx / TC][TR][TC].  A row workgroup takes RW consecutive rows
// (RW divides TR), a column workgroup one tile column of TC columns.

// map a block index to a work index so that the `per` work items whose data
// share HBM lines run on the same XCD (blocks go round-robin to the 8 XCDs)
__device__ __forceinline__ int xcd_remap(int b, int n, int per) {
  const int span = 8 * per;
  if (per <= 1 || b >= (n / span) * span) return b;  // a remainder keeps its order
  const int x = b & 7, s = b >> 3;
  return (s / per) * span + x * per + (s % per);
}

template <class T>
constexpr int lines_share(int elems) {
  const int bytes = elems * 2 * (int)sizeof(T);
  return bytes >= 128 ? 1 : 128 / bytes;
}

// copy `n` complex values in 16-byte units (n and both offsets even for float)
template <class T>
__device__ __forceinline__ void copy16(cx<T>* dst, const cx<T>* src) {
  *reinterpret_cast<uint4*>(dst) = *reinterpret_cast<const uint4*>(src);
}
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <class T>
__device__ __forceinline__ void copy16(cx<T>* dst, const WF_GLOBAL cx<T>* src) {
  *reinterpret_cast<u32x4*>(dst) = *reinterpret_cast<const WF_GLOBAL u32x4*>(src);
}
template <class T>
__device__ __forceinline__ void copy16(WF_GLOBAL cx<T>* dst, const cx<T>* src) {
  *reinterpret_cast<WF_GLOBAL u32x4*>(dst) = *reinterpret_cast<const u32x4*>(src);
}

// ---------------------------------------------------------------------------
// row kernel: inverse row FFT -> white-level update -> forward row FFT
// ---------------------------------------------------------------------------
// twiddle table staged in LDS, in the pass-major order of the kernel's radix
// plan, when it is small (float32 up to 2048 points); larger tables are read
// in natural order through the L1/L2 caches
template <class T, int N>
constexpr bool lds_twiddles() {
  return N * 2 * (int)sizeof(T) <= 16384;
}

// values per thread of the row kernel's transforms: 8 for the float32
// lengths 1024 and 2048 (twice the threads of 16 values, so twice the waves
// to hide the row kernel's memory latency; measured 6% faster at 2048), else
// the default (at 4096, 8 values would make 1024-thread blocks that spill)
template <class T, int N>
constexpr int row_elems() {
  return (sizeof(T) == 4 && (N == 1024 || N == 2048)) ? 8 : elems<N>::value;
}

// values per thread of the column kernel's transforms: 8 for the float32
// lengths 1024 and 2048, with four waves per SIMD and the per-mode state
// loaded two modes at a time (every wave of a 2048^2 sweep is then resident
// at once: 27.3 instead of 31.1 us per launch), else the default
template <class T, int N>
constexpr int col_elems() {
  return (sizeof(T) == 4 && (N == 1024 || N == 2048)) ? 8 : elems<N>::value;
}

// values per thread of the monitor's transforms (path precision): 8 at
// 1024-4096 (measured 12% faster than 16 at 2048 when the monitor ran its
// transforms in float64: 99 vs 113 us per check; with float32 transforms,
// 16 values in the row pass took a check from 27.0 to 29.1 us, and to 28.2
// with its twiddles read through the caches instead of staged in LDS)
template <int N>
constexpr int mon_elems() {
  return (N == 1024 || N == 2048 || N == 4096) ? 8 : elems<N>::value;
}

// at least 2 waves per SIMD so that two blocks share a CU and one
// block's memory phase overlaps another's FFT; 3 for the float32 lengths with
// a factor 3 (12 values per thread)
template <class T, int N>
constexpr int min_waves() {
  return (sizeof(T) == 4 && N % 3 == 0) ? 3 : 2;
}
// waves per SIMD the column kernel is built for: four with 8 values per
// thread, else as above
template <class T, int N>
constexpr int col_min_waves() {
  return col_elems<T, N>() == 8 ? 4 : min_waves<T, N>();
}
// the chunk's last sweep (joint objective and the monitor's column
// transforms) runs once per chunk: one wave per SIMD fewer, so that its
// longer body does not spill
template <class T, int N, int MODE>
constexpr int col_waves() {
  return (MODE == COL_SWEEP_J && col_min_waves<T, N>() > 2) ? col_min_waves<T, N>() - 1
                                                              : col_min_waves<T, N>();
}

template <class T, int NX, int TR, int TC, int RW, int MODE>
__global__ __launch_bounds__((RW / 2) * (NX / row_elems<T, NX>()), (min_waves<T, NX>())) void row_kernel(const SweepArgs<T>* __restrict__ argv, int k_local,
    const T* __restrict__ xin, T* __restrict__ xout) {
  const SweepArgs<T>& a = argv[blockIdx.y];  // one map per grid row
  constexpr int E = row_elems<T, NX>();
  constexpr int NT = NX / E;
  constexpr int RP = RW / 2;
  constexpr int KPC = NX / 2;                 // packed half width
  constexpr int SUB = RW * KPC;               // complex values of this block's rows
  using LM = ldsmap<T, NX, E>;  // exchange-buffer index map
  constexpr int XS = LM::size;
  // the band is staged row-major with a padded row stride (rows 16 banks
  // apart), so that reading one row's consecutive k_x and writing a tile's
  // rows are free of LDS bank conflicts (the tile order of the transit buffer
  // is not)
  constexpr int RS = KPC + 8;
  constexpr int LDSN = (RW * RS > RP * XS) ? RW * RS : RP * XS;
  constexpr int EPC = 16 / (2 * (int)sizeof(T));  // complex values per 16 bytes
  __shared__ __align__(16) cx<T> lds[LDSN];
  constexpr bool LTW = lds_twiddles<T, NX>();
  __shared__ cx<T> twl[LTW ? NX : 1];

  constexpr bool SW = MODE == ROW_SWEEP || MODE == ROW_SWEEP_J;
  constexpr bool JV = MODE == ROW_SWEEP_J;
  T lt = (T)0;  // lambda * tau of the white level
  bool jdo = false;  // this sweep closes its chunk: sum the pixel term of J
  if constexpr (SW) {
    const WF_GLOBAL DevSched* s = gmem(a.sch);
    if (s->done) return;
    const int kk = s->base + k_local;
    if (kk >= s->max_sweeps) return;
    lt = (T)(gmem(a.lam)[kk] * a.tauW);
    if constexpr (JV) jdo = kk == min(s->base + s->K, s->max_sweeps) - 1;
  }
  __shared__ double jsh[JV ? 16 : 1];
  double jacc = 0.0;
  const int tid = threadIdx.x;
  const int blk = xcd_remap(blockIdx.x, gridDim.x, min(TR / RW, lines_share<T>(RW * TC)));
  const int y0 = blk * RW;
  const int r0 = y0 % TR;
  WF_GLOBAL cx<T>* gband = gmem((cx<T>*)a.B) + (size_t)(y0 / TR) * (TR * KPC) + r0 * TC;
  const WF_GLOBAL cx<T>* twg = gmem((const cx<T>*)a.twx);
  const int p = tid / NT, t = tid - p * NT;
  const int ya = y0 + 2 * p;
  constexpr int NTHR = RP * NT;  // threads of the block
  cx<T> reg[E];

  if constexpr (SW || MODE == ROW_C2R) {
    // every load of the band and of the twiddle table is issued before the
    // first LDS write, so their latencies overlap
    constexpr int NIT = SUB / (NTHR * EPC);
    static_assert(NIT * NTHR * EPC == SUB, "the band splits evenly over the threads");
    cx<T> bv[NIT][EPC];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int e = (tid + it * NTHR) * EPC;
      const int g = e / (RW * TC), w = e - g * (RW * TC);
      copy16(bv[it], &gband[g * (TR * TC) + w]);
    }
    TwiddleStage<T, NX, E, NTHR> tws;
    if constexpr (LTW) tws.load(twg, tid);
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int e = (tid + it * NTHR) * EPC;
      const int g = e / (RW * TC), w = e - g * (RW * TC);
      const int rr = w / TC, cc = w - rr * TC;
      copy16(&lds[rr * RS + g * TC + cc], bv[it]);
    }
    if constexpr (LTW) tws.store(twl, tid);
    __syncthreads();
    // Z = A + i B for the row pair; A, B Hermitian in k_x; slot 0 packs
    // (re of k_x = 0, re of k_x = nx/2)
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int k = t + NT * q;
      const bool hi = k > NX / 2;
      const int kx = hi ? NX - k : k;
      const int ks = (kx == NX / 2) ? 0 : kx;
      const int li = (2 * p) * RS + ks;
      cx<T> A = lds[li], Bv = lds[li + RS];
      if (kx == 0) {
        A.im = (T)0;
        Bv.im = (T)0;
      } else if (kx == NX / 2) {
        A = cx<T>{A.im, (T)0};
        Bv = cx<T>{Bv.im, (T)0};
      }
      if (hi) {
        A.im = -A.im;
        Bv.im = -Bv.im;
      }
      reg[q] = cx<T>{A.re - Bv.im, A.im + Bv.re};
    }
    __syncthreads();
    if constexpr (LTW) fft<T, NX, true, E, true>(reg, lds + p * XS, t, (const cx<T>*)twl);
    else fft<T, NX, true, E, false>(reg, lds + p * XS, t, twg);
    const T sc = (T)a.scale;
    if constexpr (MODE == ROW_C2R) {
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const size_t i0 = (size_t)ya * NX + t + NT * q;
        xout[i0] = reg[q].re * sc;
        xout[i0 + NX] = reg[q].im * sc;
      }
      return;
    } else {
      // white-level update, data and coefficients loaded in batches of 8
      // (float32) or 4 (float64, or 12 values per thread) values, to stay
      // within the register budget
      constexpr int QB = (sizeof(T) == 8 || E % 8 != 0) ? 4 : 8;
      static_assert(E % QB == 0, "batches split the thread's values evenly");
      const WF_GLOBAL T* gd = gmem(a.d);
      const WF_GLOBAL T* gn2 = gmem(a.nbar2);
#pragma unroll
      for (int h = 0; h < E; h += QB) {
        T dv0[QB], dv1[QB], nb0[QB], nb1[QB];
#pragma unroll
        for (int q = 0; q < QB; ++q) {
          const size_t i0 = (size_t)ya * NX + t + NT * (h + q);
          dv0[q] = gd[i0];
          dv1[q] = gd[i0 + NX];
          nb0[q] = gn2[i0];
          nb1[q] = gn2[i0 + NX];
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
          const T d1a = reg[h + q].re * sc, d1b = reg[h + q].im * sc;
          const T t2a = white_update<T>(dv0[q], nb0[q], d1a, lt);
          const T t2b = white_update<T>(dv1[q], nb1[q], d1b, lt);
          if constexpr (JV) {
            if (jdo) jacc += white_term<T>(dv0[q], nb0[q], t2a) + white_term<T>(dv1[q], nb1[q], t2b);
          }
          reg[h + q] = cx<T>{t2a, t2b};
        }
      }
      if constexpr (JV) {
        if (jdo) wave_partial(jacc, jsh);
      }
    }
  } else {  // ROW_R2C
    if constexpr (LTW) stage_twiddles<T, NX, E, NTHR>(twl, twg, tid);
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const size_t i0 = (size_t)ya * NX + t + NT * q;
      reg[q] = cx<T>{xin[i0], xin[i0 + NX]};
    }
    if constexpr (LTW) __syncthreads();
  }
  if constexpr (LTW) fft<T, NX, false, E, true>(reg, lds + p * XS, t, (const cx<T>*)twl);
  else fft<T, NX, false, E, false>(reg, lds + p * XS, t, twg);
#pragma unroll
  for (int q = 0; q < E; ++q) lds[p * XS + LM::at_tq(t, q)] = reg[q];
  __syncthreads();
  if constexpr (JV) {
    if (jdo && tid == 0) gmem(a.jpart)[blk] = sum_partials(jsh, blockDim.x);
  }
  // split Z into the two rows' spectra; write this block's rows, tile order
  for (int e = tid * EPC; e < SUB; e += blockDim.x * EPC) {
    cx<T> v[EPC];
#pragma unroll
    for (int u = 0; u < EPC; ++u) {
      const int eu = e + u;
      const int g = eu / (RW * TC), w = eu - g * (RW * TC);
      const int rr = w / TC, c = w - rr * TC;
      const int kx = g * TC + c;
      const cx<T>* Z = lds + (rr >> 1) * XS;
      if (kx == 0) {
        const cx<T> z0 = Z[LM::at(0)], zn = Z[LM::at(NX / 2)];
        v[u] = (rr & 1) ? cx<T>{z0.im, zn.im} : cx<T>{z0.re, zn.re};
      } else {
        const cx<T> zk = Z[LM::at(kx)], zm = Z[LM::at(NX - kx)];
        v[u] = (rr & 1) ? cx<T>{(zk.im + zm.im) * (T)0.5, (zm.re - zk.re) * (T)0.5}
                        : cx<T>{(zk.re + zm.re) * (T)0.5, (zk.im - zm.im) * (T)0.5};
      }
    }
    const int g = e / (RW * TC), w = e - g * (RW * TC);
    copy16(&gband[g * (TR * TC) + w], v);
  }
}

// ---------------------------------------------------------------------------
// column kernel: forward column FFT -> Fourier-side chain -> inverse FFT
// ---------------------------------------------------------------------------
// [wa a + wb b] / (wa + wb) with inv = 1 / (wa + wb).  The weights are
// normalised before they touch the fields: a projected mode's covariance
// (kInfiniteCov) times an unnormalised Fourier coefficient would overflow
// float32, while wa * inv stays in [0, 1].
template <class T>
__device__ __forceinline__ cx<T> wavg(T wa, cx<T> a, T wb, cx<T> b, T inv) {
  const T ua = wa * inv, ub = wb * inv;
  return cx<T>{ua * a.re + ub * b.re, ua * a.im + ub * b.im};
}

// Per-mode coefficients of the chain at one sweep.
template <class T>
struct ChainCoef {
  T TW, TA, TB, SA, cB, nxr;
  int fk;
  bool store_first;
  double jTW, jTA, jTB;  // lambda tau in float64, for the joint objective
};

template <class T>
__device__ __forceinline__ double cnorm2(cx<T> a) {
  const double r = a.re, i = a.im;
  return r * r + i * i;
}
template <class T>
__device__ __forceinline__ double cdist2(cx<T> a, cx<T> b) {
  const double r = (double)a.re - (double)b.re, i = (double)a.im - (double)b.im;
  return r * r + i * i;
}

// One mode: t_2 (white messenger, Fourier) in, field for the white level out.
// Reads and writes the stored Fourier-side fields of this mode.  With JV, adds
// jw times this mode's terms of the joint objective (unnormalised
// coefficients; the caller applies 1/(nx ny)) to jacc.
template <class T, int FK, bool JV>
__device__ __forceinline__ cx<T> chain_mode(WF_GLOBAL cx<T>* tA, WF_GLOBAL cx<T>* dA,
                                            WF_GLOBAL cx<T>* tB, const ChainCoef<T>& k, int kx,
                                            int ky, size_t idx, cx<T> t2, T s, T nbA, T pst,
                                            cx<T> tAo, cx<T> dAo, cx<T> tBo, double& jacc,
                                            double jw) {
  if constexpr (FK == FK_NONE) {
    if (k.store_first) stc(tA + idx, t2);
    if constexpr (JV) jacc += jw * cnorm2(t2) / ((double)s + k.jTW);
    return cscale(t2, s * rcp(s + k.TW));
  } else if constexpr (FK == FK_ARRAY_STRIPE) {
    const T nbB = (kx == 0 ? k.nxr * pst : (T)0) + k.cB;
    const cx<T> dBn = wavg(nbB, t2, k.TW, tBo, rcp(nbB + k.TW));
    const cx<T> tBn = wavg(k.TB, dBn, nbB, dAo, rcp(nbB + k.TB));
    const cx<T> dAn = wavg(nbA, tBn, k.TB, tAo, rcp(nbA + k.TB));
    const cx<T> so = cscale(tAo, s * rcp(s + k.SA));
    const cx<T> tAn = wavg(k.TA, dAn, nbA, so, rcp(nbA + k.TA));
    stc(tB + idx, tBn);
    stc(dA + idx, dAn);
    stc(tA + idx, tAn);
    if constexpr (JV)
      jacc += jw * (cnorm2(tAn) / ((double)s + k.jTA) + cdist2(dAn, tAn) / (double)nbA +
                     cdist2(tBn, dAn) / k.jTB + cdist2(dBn, tBn) / (double)nbB +
                     cdist2(t2, dBn) / k.jTW);
    return dBn;
  } else {
    // one Fourier level: an array level or the stripe level
    T nb;
    if constexpr (FK == FK_ARRAY) nb = nbA;
    else nb = (kx == 0 ? k.nxr * pst : (T)0) + k.cB;
    const cx<T> dAn = wavg(nb, t2, k.TW, tAo, rcp(nb + k.TW));
    const cx<T> so = cscale(tAo, s * rcp(s + k.SA));
    const cx<T> tAn = wavg(k.TA, dAn, nb, so, rcp(nb + k.TA));
    stc(tA + idx, tAn);
    if constexpr (JV)
      jacc += jw * (cnorm2(tAn) / ((double)s + k.jTA) + cdist2(dAn, tAn) / (double)nb +
                     cdist2(t2, dAn) / k.jTW);
    return dAn;
  }
}

template <class T>
__device__ __forceinline__ cx<T> cconj(cx<T> v) { return cx<T>{v.re, -v.im}; }

template <class T, int NY, int TR, int TC, int MODE, int FK>
__global__ __launch_bounds__(TC * (NY / col_elems<T, NY>()), (col_waves<T, NY, MODE>())) void col_kernel(const SweepArgs<T>* __restrict__ argv, int k_local,
    cx<T>* __restrict__ spec, double lam_init) {
  const SweepArgs<T>& a = argv[blockIdx.y];  // one map per grid row
  constexpr int E = col_elems<T, NY>();
  constexpr int NT = NY / E;
  using LM = ldsmap<T, NY, E>;  // exchange-buffer index map
  constexpr int YS = LM::size;
  constexpr int TRTC = TR * TC;
  constexpr int EPC = 16 / (2 * (int)sizeof(T));
  __shared__ __align__(16) cx<T> lds[TC * YS];
  constexpr bool LTW = lds_twiddles<T, NY>();
  __shared__ cx<T> twl[LTW ? NY : 1];

  constexpr bool SW = MODE == COL_SWEEP || MODE == COL_SWEEP_J;
  constexpr bool JV = MODE == COL_SWEEP_J;
  __shared__ double jsh[JV ? 16 : 1];
  double jacc = 0.0;
  double lam = 0.0, lamp = 0.0;
  bool store_first = false;  // the chunk's last sweep (also: sum J there)
  if constexpr (SW) {
    const WF_GLOBAL DevSched* s = gmem(a.sch);
    if (s->done) return;
    const int base = s->base;
    const int kk = base + k_local;
    if (kk >= s->max_sweeps) return;
    const WF_GLOBAL double* glam = gmem(a.lam);
    lam = glam[kk];
    lamp = glam[kk > 0 ? kk - 1 : 0];
    const int klast = min(base + s->K, s->max_sweeps) - 1;
    store_first = (kk == klast);
  }
  const int tid = threadIdx.x;
  const int G = a.nx / 2 / TC;
  const int g = xcd_remap(blockIdx.x, G, lines_share<T>(TRTC));
  const int c = tid / NT, t = tid - c * NT;
  const int kxc = g * TC + c;          // column of B (0 packs k_x = 0 and nx/2)
  const bool packed = (kxc == 0);
  const int nh = a.nx / 2 + 1;
  const int kxn = a.nx / 2;
  WF_GLOBAL cx<T>* gB = gmem((cx<T>*)a.B);
  const WF_GLOBAL cx<T>* twg = gmem((const cx<T>*)a.twy);
  // per-mode coefficients and stored fields
  const WF_GLOBAL T* gsc = gmem(a.sc);
  const WF_GLOBAL T* gnb = gmem(a.nbA);
  const WF_GLOBAL T* gps = gmem(a.pst);
  WF_GLOBAL cx<T>* gtA = gmem((cx<T>*)a.tA);
  WF_GLOBAL cx<T>* gdA = gmem((cx<T>*)a.dA);
  WF_GLOBAL cx<T>* gtB = gmem((cx<T>*)a.tB);
  cx<T> reg[E];
  constexpr int NTHR = TC * NT;  // threads of the block

  // per-mode state and coefficients of this column, loaded in batches of 8
  // modes, or 4 where the registers are scarce (float64, or 4096 points; 8
  // spilled there), or 2 with 8 values per thread (four waves per SIMD leave
  // 128 registers) and with 12 float32 values (three waves, 168 registers)
  constexpr int HB = (E == 8 || (E == 12 && sizeof(T) == 4))
                         ? 2
                         : ((sizeof(T) == 8 || E % 8 != 0 || NY >= 4096) ? 4 : 8);
  static_assert(E % HB == 0, "batches split the thread's values evenly");
  constexpr bool hasA = FK != FK_NONE;
  constexpr bool hasB = FK == FK_ARRAY_STRIPE;
  constexpr bool needNb = FK == FK_ARRAY || FK == FK_ARRAY_STRIPE;
  constexpr bool needP = FK == FK_STRIPE || FK == FK_ARRAY_STRIPE;
  const cx<T> z0 = {(T)0, (T)0};
  T sv[HB], nv[HB], pv[HB];
  cx<T> ta[HB], da[HB], tb[HB];
  auto load_half = [&](int h) {
#pragma unroll
    for (int q = 0; q < HB; ++q) {
      const int ky = t + NT * (h + q);
      const size_t idx = (size_t)kxc * NY + ky;
      sv[q] = gsc[idx];
      nv[q] = needNb ? gnb[idx] : (T)0;
      pv[q] = needP ? gps[ky] : (T)0;
      ta[q] = hasA ? ldc(gtA + idx) : z0;
      da[q] = hasB ? ldc(gdA + idx) : z0;
      tb[q] = hasB ? ldc(gtB + idx) : z0;
    }
  };

  if constexpr (MODE == COL_INV_IN) {
    if constexpr (LTW) stage_twiddles<T, NY, E, NTHR>(twl, twg, tid);
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int ky = t + NT * q;
      if (packed) {
        // Hermitian parts of the k_x = 0 and nx/2 columns (irfft2 semantics)
        const int km = ky == 0 ? 0 : NY - ky;
        const cx<T> a0 = spec[(size_t)ky * nh], b0 = spec[(size_t)km * nh];
        const cx<T> an = spec[(size_t)ky * nh + kxn], bn = spec[(size_t)km * nh + kxn];
        const cx<T> h0 = cscale(a0 + cconj(b0), (T)0.5), hn = cscale(an + cconj(bn), (T)0.5);
        reg[q] = cx<T>{h0.re - hn.im, h0.im + hn.re};
      } else {
        reg[q] = spec[(size_t)ky * nh + kxc];
      }
    }
    if constexpr (LTW) __syncthreads();
  } else {
    // every 16-byte load of this block's columns, then the twiddle table's,
    // is issued before the first LDS store (0.7 us faster at 2048^2 than
    // load-store pairs)
    constexpr int NIT = E / EPC;
    static_assert(NIT * NTHR * EPC == TC * NY, "the columns split evenly over the threads");
    cx<T> bv[NIT][EPC];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int e = (tid + it * NTHR) * EPC;
      const int yb = e / TRTC, w = e - yb * TRTC;
      copy16(bv[it], &gB[((size_t)yb * G + g) * TRTC + w]);
    }
    TwiddleStage<T, NY, E, NTHR> tws;
    if constexpr (LTW) tws.load(twg, tid);
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int e = (tid + it * NTHR) * EPC;
      const int yb = e / TRTC, w = e - yb * TRTC;
#pragma unroll
      for (int u = 0; u < EPC; ++u) {
        const int r = (w + u) / TC, cc = (w + u) - r * TC;
        lds[cc * YS + LM::at(yb * TR + r)] = bv[it][u];
      }
    }
    if constexpr (LTW) tws.store(twl, tid);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < E; ++q) reg[q] = lds[c * YS + LM::at_tq(t, q)];
    __syncthreads();
    if constexpr (LTW) fft<T, NY, false, E, true>(reg, lds + c * YS, t, (const cx<T>*)twl);
    else fft<T, NY, false, E, false>(reg, lds + c * YS, t, twg);
  }

  // packed column (block 0, column 0): split Z = C0 + i CN into the k_x = 0
  // and k_x = nx/2 spectra; C0 stays in registers, CN goes to this column's
  // LDS slots (only this column's threads touch them until the inverse FFT)
  cx<T>* cnl = lds;  // column 0's region
  if constexpr (MODE != COL_INV_IN) {
    if (g == 0) {
      if (packed) {
#pragma unroll
        for (int q = 0; q < E; ++q) lds[LM::at_tq(t, q)] = reg[q];
      }
      __syncthreads();
      cx<T> cnv[E];
      if (packed) {
#pragma unroll
        for (int q = 0; q < E; ++q) {
          const int ky = t + NT * q;
          const cx<T> zk = reg[q], zm = lds[LM::at(ky == 0 ? 0 : NY - ky)];
          reg[q] = cx<T>{(zk.re + zm.re) * (T)0.5, (zk.im - zm.im) * (T)0.5};
          cnv[q] = cx<T>{(zk.im + zm.im) * (T)0.5, (zm.re - zk.re) * (T)0.5};
        }
      }
      __syncthreads();
      if (packed) {
#pragma unroll
        for (int q = 0; q < E; ++q) cnl[LM::at_tq(t, q)] = cnv[q];
      }
    }
  }

  if constexpr (MODE == COL_FWD_OUT) {
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const size_t row = (size_t)(t + NT * q) * nh;
      spec[row + kxc] = reg[q];
      if (packed) spec[row + kxn] = cnl[LM::at_tq(t, q)];
    }
    return;
  }


  if constexpr (SW) {
    ChainCoef<T> k;
    k.TW = (T)(lam * a.tauW);
    k.TA = (T)(lam * a.tauA);
    k.TB = (T)(lam * a.tauB);
    k.SA = (T)(lamp * a.tauA);
    k.cB = (T)a.cB;
    k.nxr = (T)a.nx;
    k.fk = a.fk;
    k.store_first = store_first;
    k.jTW = lam * a.tauW;
    k.jTA = lam * a.tauA;
    k.jTB = lam * a.tauB;
    // J only on the chunk's last sweep (block-uniform)
    const bool jdo = JV && store_first;
    const cx<T> z = {(T)0, (T)0};
    if (!packed) {
      // this column, in batches of loads
#pragma unroll
      for (int h = 0; h < E; h += HB) {
        load_half(h);
#pragma unroll
        for (int q = 0; q < HB; ++q) {
          const int ky = t + NT * (h + q);
          const size_t idx = (size_t)kxc * NY + ky;
          if (jdo)
            reg[h + q] = chain_mode<T, FK, JV>(gtA, gdA, gtB, k, kxc, ky, idx, reg[h + q], sv[q],
                                               nv[q], pv[q], ta[q], da[q], tb[q], jacc, 2.0);
          else
            reg[h + q] = chain_mode<T, FK, false>(gtA, gdA, gtB, k, kxc, ky, idx, reg[h + q],
                                                  sv[q], nv[q], pv[q], ta[q], da[q], tb[q], jacc,
                                                  0.0);
        }
      }
    }
    if (g == 0) {
      // the packed column: the real-valued columns k_x = 0 (C0, in registers)
      // and k_x = nx/2 (CN, in this column's LDS slots) are Hermitian in k_y,
      // so the chain runs on k_y <= NY/2 only -- as many modes per thread as
      // any other column, so this block is no straggler -- and the rest
      // follows by conjugation.  The stored fields of k_y > NY/2 in these two
      // columns are not updated (readers take the mirrored mode).
      constexpr int EH = E / 2;  // registers q < EH hold k_y < NY/2
      if (packed) {
#pragma unroll
        for (int q = 0; q <= EH; ++q) {
          if (q == EH && t != 0) break;  // k_y = NY/2 on thread 0 only
          const int ky = t + NT * q;
          const int li = LM::at_tq(t, q);
          const T ps = needP ? gps[ky] : (T)0;
          const size_t i0 = (size_t)ky, iN = (size_t)kxn * NY + ky;
          // k_y and NY - k_y of a real column are one conjugate pair; the
          // terms are summed (weight > 0) on the chunk's last sweep only
          const double jw = !jdo ? 0.0 : ((ky == 0 || ky == NY / 2) ? 1.0 : 2.0);
          reg[q] = chain_mode<T, FK, JV>(gtA, gdA, gtB, k, 0, ky, i0, reg[q], gsc[i0],
                                         needNb ? gnb[i0] : (T)0, ps, hasA ? ldc(gtA + i0) : z,
                                         hasB ? ldc(gdA + i0) : z, hasB ? ldc(gtB + i0) : z,
                                         jacc, jw);
          cnl[li] = chain_mode<T, FK, JV>(gtA, gdA, gtB, k, kxn, ky, iN, cnl[li], gsc[iN],
                                          needNb ? gnb[iN] : (T)0, ps, hasA ? ldc(gtA + iN) : z,
                                          hasB ? ldc(gdA + iN) : z, hasB ? ldc(gtB + iN) : z,
                                          jacc, jw);
          // C0 of k_y in (0, NY/2) waits in the unused CN slot of NY - k_y
          if (q < EH && ky > 0) cnl[LM::at(NY - ky)] = reg[q];
        }
      }
      __syncthreads();
      if (packed) {
#pragma unroll
        for (int q = 0; q < E; ++q) {
          const int ky = t + NT * q;
          cx<T> c0, cn;
          if (ky <= NY / 2) {
            c0 = reg[q];
            cn = cnl[LM::at_tq(t, q)];
          } else {
            c0 = cconj(cnl[LM::at_tq(t, q)]);
            cn = cconj(cnl[LM::at(NY - ky)]);
          }
          reg[q] = cx<T>{c0.re - cn.im, c0.im + cn.re};
        }
      }
    }
  }

  if constexpr (MODE == COL_INIT) {
    // warm start: every stored field = s_init; the field handed to the white
    // level is s_init too, except for a chain without Fourier level, where it
    // is the signal-end field S_c (S_c + lambda_0 tau)^-1 s_init (or s_init
    // itself when s_init is that field)
    WF_GLOBAL cx<T>* tA = gtA;
    WF_GLOBAL cx<T>* dA = gdA;
    WF_GLOBAL cx<T>* tB = gtB;
    const T TW0 = (T)(lam_init * a.tauW);
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int ky = t + NT * q;
      cx<T> out[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (h == 1 && !packed) break;
        const int kx = h == 0 ? kxc : kxn;
        const size_t idx = (size_t)kx * NY + ky;
        cx<T> v = h == 0 ? reg[q] : cnl[LM::at_tq(t, q)];
        if (a.fk == FK_NONE) {
          if (!a.warm_chain) {
            const T s = gsc[idx];
            v = cscale(v, s * rcp(s + TW0));
          }
        } else {
          stc(tA + idx, v);
          if (a.fk == FK_ARRAY_STRIPE) {
            stc(dA + idx, v);
            stc(tB + idx, v);
          }
        }
        out[h] = v;
      }
      reg[q] = packed ? cx<T>{out[0].re - out[1].im, out[0].im + out[1].re} : out[0];
    }
  }

  if constexpr (JV) {
    if (store_first) wave_partial(jacc, jsh);
  }
  // the inverse transform reuses column 0's LDS region
  __syncthreads();
  if constexpr (JV) {
    // this block's share of the Fourier-side terms, unitary normalisation
    if (store_first && tid == 0)
      gmem(a.jpart)[a.jrow + g] = sum_partials(jsh, blockDim.x) * a.scale;
  }
  if constexpr (LTW) fft<T, NY, true, E, true>(reg, lds + c * YS, t, (const cx<T>*)twl);
  else fft<T, NY, true, E, false>(reg, lds + c * YS, t, twg);
#pragma unroll
  for (int q = 0; q < E; ++q) lds[c * YS + LM::at_tq(t, q)] = reg[q];
  __syncthreads();
  for (int e = tid * EPC; e < TC * NY; e += blockDim.x * EPC) {
    const int yb = e / TRTC, w = e - yb * TRTC;
    cx<T> v[EPC];
#pragma unroll
    for (int u = 0; u < EPC; ++u) {
      const int r = (w + u) / TC, cc = (w + u) - r * TC;
      v[u] = lds[cc * YS + LM::at(yb * TR + r)];
    }
    copy16(&gB[((size_t)yb * G + g) * TRTC + w], v);
  }
  if constexpr (JV) {
    if (store_first) {
      // The monitor's column pass for this block's columns, from the state
      // this sweep left (the chunk's last): x = t_A / (S_c + lambda tau) and
      // y = (S + N_F) x per mode in float64, rounded once, inverse column
      // transforms, written to the monitor transit in its own tiling.  The
      // real columns k_x = 0 and nx/2 go through one transform as
      // x_0 + i x_nx/2 (both transforms are real).  Fields of this block
      // that other threads stored are read after the barrier.
      __syncthreads();
      const double Tf = lam * (FK == FK_NONE ? a.tauW : a.tauA);
      const WF_GLOBAL T* gsy = gmem(a.sy);
      auto xy = [&](int kx, int ky, cx<double>& xo, cx<double>& yo) {
        const bool mir = (kx == 0 || kx == kxn) && ky > NY / 2;
        const size_t idx = (size_t)kx * NY + (mir ? NY - ky : ky);
        cx<T> v = ldc(gtA + idx);
        if (mir) v.im = -v.im;
        if ((kx == 0 || kx == kxn) && (ky == 0 || ky == NY / 2)) v.im = (T)0;
        const double inv = 1.0 / ((double)gsc[idx] + Tf), f = (double)gsy[idx];
        xo = cx<double>{(double)v.re * inv, (double)v.im * inv};
        yo = cx<double>{xo.re * f, xo.im * f};
      };
      cx<T> rx[E], ry[E];
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const int ky = t + NT * q;
        cx<double> x0, y0;
        xy(kxc, ky, x0, y0);
        if (packed) {
          cx<double> xn, yn;
          xy(kxn, ky, xn, yn);
          x0 = cx<double>{x0.re - xn.im, x0.im + xn.re};
          y0 = cx<double>{y0.re - yn.im, y0.im + yn.re};
        }
        rx[q] = cx<T>{(T)x0.re, (T)x0.im};
        ry[q] = cx<T>{(T)y0.re, (T)y0.im};
      }
      const int GM = a.kpm / kTCM;  // monitor tiles per tile row
#pragma unroll
      for (int field = 0; field < 2; ++field) {
        cx<T>* reg2 = field == 0 ? rx : ry;
        WF_GLOBAL cx<T>* dst = gmem((cx<T>*)(field == 0 ? a.Mx : a.My));
        if constexpr (LTW) fft<T, NY, true, E, true>(reg2, lds + c * YS, t, (const cx<T>*)twl);
        else fft<T, NY, true, E, false>(reg2, lds + c * YS, t, twg);
#pragma unroll
        for (int q = 0; q < E; ++q) lds[c * YS + LM::at_tq(t, q)] = reg2[q];
        __syncthreads();
        // element e of this block: row y = e / TC, column g TC + e % TC; EPC
        // consecutive values share a monitor tile row (TC and kTCM even)
        for (int e = tid * EPC; e < TC * NY; e += blockDim.x * EPC) {
          const int y = e / TC, cc0 = e - y * TC;
          const int kx0 = g * TC + cc0;
          cx<T> v[EPC];
#pragma unroll
          for (int u = 0; u < EPC; ++u) v[u] = lds[(cc0 + u) * YS + LM::at(y)];
          const size_t tile = ((size_t)(y / kTRM) * GM + kx0 / kTCM) * (kTRM * kTCM);
          const size_t off = tile + (y % kTRM) * kTCM + kx0 % kTCM;
          if (g == 0 && cc0 == 0) {
            // block 0's column 0 holds x_0 + i x_nx/2 (whichever thread
            // writes it): split into the two real columns
            const cx<T> z = v[0];
            v[0] = cx<T>{z.re, (T)0};
            const size_t tn = ((size_t)(y / kTRM) * GM + kxn / kTCM) * (kTRM * kTCM) +
                              (y % kTRM) * kTCM + kxn % kTCM;
            stc(dst + tn, cx<T>{z.im, (T)0});
          }
          copy16(dst + off, v);
        }
        __syncthreads();
      }
    }
  }
}

// ---------------------------------------------------------------------------
// float64 residual monitor and output
// ---------------------------------------------------------------------------


__device__ __forceinline__ bool monitor_active(const WF_GLOBAL DevSched* s, double* lam_last,
                                               const WF_GLOBAL double* lam) {
  if (s->done) return false;
  const int klast = min(s->base + s->K, s->max_sweeps) - 1;
  *lam_last = lam[klast];
  return true;
}

template <class T, int NY>
__global__ __launch_bounds__(kTCM * (NY / mon_elems<NY>())) void mon_col_kernel(const MonArgs<T>* __restrict__ argv, int mode) {
  const MonArgs<T>& m = argv[blockIdx.y];
  constexpr int E = mon_elems<NY>();
  constexpr int NT = NY / E;
  using LM = ldsmap<T, NY, E>;  // exchange-buffer index map
  constexpr int YS = LM::size;
  constexpr int TRTC = kTRM * kTCM;
  constexpr int EPC = 16 / (2 * (int)sizeof(T));  // complex values per 16 bytes
  static_assert(TRTC % EPC == 0, "16-byte runs stay within a tile");
  __shared__ __align__(16) cx<T> lds[kTCM * YS];
  constexpr bool LTW = lds_twiddles<T, NY>();
  __shared__ cx<T> twl[LTW ? NY : 1];
  // residual: lambda of the chunk's last sweep; output: of the last sweep run
  double lamv = gmem(m.sch)->lam_last;
  if (mode == MON_RESIDUAL && !monitor_active(gmem(m.sch), &lamv, gmem(m.lam))) return;
  const int tid = threadIdx.x, G = m.kpm / kTCM;
  // the transit tiles of neighbouring blocks share HBM lines: keep them on one XCD
  const int g = xcd_remap(blockIdx.x, G, lines_share<T>(TRTC));
  const int c = tid / NT, t = tid - c * NT;
  const int kx = g * kTCM + c;
  const bool valid = kx < m.nx / 2 + 1;
  const double Tf = lamv * m.tau_first;
  const WF_GLOBAL cx<T>* tf = gmem((const cx<T>*)m.tfirst);
  const WF_GLOBAL T* msc = gmem(m.sc);
  const WF_GLOBAL T* msy = gmem(m.sy);
  const WF_GLOBAL T* msig = gmem(m.sig);
  const WF_GLOBAL cx<T>* twg = gmem((const cx<T>*)m.twy);
  TwiddleStage<T, NY, E, kTCM * NT> tws;
  if constexpr (LTW) tws.load(twg, tid);
  // x = t / (S_c + lambda tau) and the Fourier-diagonal products are formed
  // in float64 and rounded once to the transform precision
  cx<T> rx[E], ry[E];
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int ky = t + NT * q;
    // the sweep keeps the real columns k_x = 0 and nx/2 for k_y <= NY/2 only:
    // the other half is the conjugate of the mirrored mode
    const bool mir = (kx == 0 || kx == m.nx / 2) && ky > NY / 2;
    const size_t idx = (size_t)kx * NY + (mir ? NY - ky : ky);
    if (valid) {
      cx<T> v = ldc(tf + idx);
      if (mir) v.im = -v.im;
      const double inv = m.x_direct ? 1.0 : 1.0 / ((double)msc[idx] + Tf);
      const double xr = (double)v.re * inv, xi = (double)v.im * inv;
      const double f = (mode == MON_OUTPUT) ? (m.out_chain ? (double)msc[idx] : (double)msig[idx])
                                            : (double)msy[idx];
      rx[q] = cx<T>{(T)xr, (T)xi};
      ry[q] = cx<T>{(T)(xr * f), (T)(xi * f)};
    } else {
      rx[q] = cx<T>{(T)0, (T)0};
      ry[q] = cx<T>{(T)0, (T)0};
    }
  }
  if constexpr (LTW) {
    tws.store(twl, tid);
    __syncthreads();
  }
#pragma unroll
  for (int field = 0; field < 2; ++field) {
    cx<T>* reg = field == 0 ? rx : ry;
    WF_GLOBAL cx<T>* dst = gmem((cx<T>*)(field == 0 ? m.Mx : m.My));
    if constexpr (LTW) fft<T, NY, true, E, true>(reg, lds + c * YS, t, (const cx<T>*)twl);
    else fft<T, NY, true, E, false>(reg, lds + c * YS, t, twg);
#pragma unroll
    for (int q = 0; q < E; ++q) lds[c * YS + LM::at_tq(t, q)] = reg[q];
    __syncthreads();
    // 16-byte stores: EPC consecutive values of a tile
    for (int e = tid * EPC; e < kTCM * NY; e += blockDim.x * EPC) {
      const int yb = e / TRTC, w = e - yb * TRTC;
      cx<T> v[EPC];
#pragma unroll
      for (int u = 0; u < EPC; ++u) {
        const int r = (w + u) / kTCM, cc = (w + u) - r * kTCM;
        v[u] = lds[cc * YS + LM::at(yb * kTRM + r)];
      }
      copy16(dst + ((size_t)yb * G + g) * TRTC + w, v);
    }
    __syncthreads();
  }
}

template <class T, int NX>
__global__ __launch_bounds__(kRWM * (NX / mon_elems<NX>())) void mon_row_kernel(const MonArgs<T>* __restrict__ argv, int mode) {
  const MonArgs<T>& m = argv[blockIdx.y];
  WF_GLOBAL T* s_out = gmem((T*)m.s_out);
  constexpr int E = mon_elems<NX>();
  constexpr int NT = NX / E;
  constexpr int KPm = KP<NX, kTCM>::value;
  constexpr int GM = KPm / kTCM;          // tiles per tile row
  constexpr int TRTC = kTRM * kTCM;
  constexpr int BANDm = kRWM * KPm;      // values of this block's rows, per field
  // the two bands are staged row-major, X rows then Y rows, with a row stride
  // of 8 mod 16 values (rows 32 banks apart for 16-byte values, 16 for 8-byte
  // ones): reading a row's consecutive k_x and writing a tile's rows are then
  // free of bank conflicts
  constexpr int RSm = KPm + ((8 - KPm % 16) + 16) % 16;
  using LM = ldsmap<T, NX, E>;  // exchange-buffer index map
  constexpr int XS = LM::size;
  constexpr int LDSN = (2 * kRWM * RSm > kRWM * XS) ? 2 * kRWM * RSm : kRWM * XS;
  __shared__ __align__(16) cx<T> lds[LDSN];
  constexpr bool LTW = lds_twiddles<T, NX>();
  __shared__ cx<T> twl[LTW ? NX : 1];
  __shared__ double sh[32];
  double lamv = 0.0;
  if (mode == MON_RESIDUAL && !monitor_active(gmem(m.sch), &lamv, gmem(m.lam))) return;
  // a block takes kRWM rows of a kTRM-row tile row; the kTRM / kRWM
  // blocks of one tile row share its HBM lines, so they run on one XCD
  const int tid = threadIdx.x;
  const int band = xcd_remap(blockIdx.x, gridDim.x, kTRM / kRWM);
  const int y0 = band * kRWM;
  const size_t tile_row = (size_t)(y0 / kTRM) * GM * TRTC + (y0 % kTRM) * kTCM;
  const WF_GLOBAL cx<T>* gx = gmem((const cx<T>*)m.Mx) + tile_row;
  const WF_GLOBAL cx<T>* gy = gmem((const cx<T>*)m.My) + tile_row;
  const WF_GLOBAL cx<T>* twg = gmem((const cx<T>*)m.twx);
  // the two bands' loads and the twiddle table's, all issued before the
  // first LDS write; value e of the band is row rr, column g kTCM + cc with
  // g = e / (kRWM kTCM): each tile holds kRWM kTCM consecutive values of it
  constexpr int NTHR = kRWM * NT;
  constexpr int EPC = 16 / (2 * (int)sizeof(T));  // complex values per 16-byte load
  static_assert(BANDm % EPC == 0 && (kRWM * kTCM) % EPC == 0, "16-byte runs stay in a tile");
  constexpr int NB = (BANDm + NTHR * EPC - 1) / (NTHR * EPC);
  cx<T> bx[NB][EPC], by[NB][EPC];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int e = (tid + i * NTHR) * EPC;
    if (e < BANDm) {
      const int g = e / (kRWM * kTCM), w = e - g * (kRWM * kTCM);
      const size_t off = (size_t)g * TRTC + w;
      copy16(bx[i], gx + off);
      copy16(by[i], gy + off);
    }
  }
  TwiddleStage<T, NX, E, NTHR> tws;
  if constexpr (LTW) tws.load(twg, tid);
  // the residual's inputs for this thread's pixels, loaded with the bands
  // (before the transform; 56 -> 51 us per check at 2048^2: this kernel has
  // the registers and the band is not delayed, unlike in the sweep's row
  // kernel, where the same prefetch made it slower)
  const int r = tid / NT, t = tid - r * NT;
  const int y = y0 + r;
  // (the white variance is Nbar_2 + nw_off on observed pixels: no read of
  // the caller's N_pix, a quarter of this pass's bytes)
  const WF_GLOBAL T* mn2 = gmem(m.nbar2);
  const WF_GLOBAL T* md = gmem(m.d);
  T pn2[E], pdd[E];
  if (mode != MON_OUTPUT) {
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const size_t i = (size_t)y * NX + t + NT * q;
      pn2[q] = mn2[i];
      pdd[q] = md[i];
    }
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int e = (tid + i * NTHR) * EPC;
    if (e < BANDm) {
      const int g = e / (kRWM * kTCM), w0 = e - g * (kRWM * kTCM);
#pragma unroll
      for (int u = 0; u < EPC; ++u) {
        const int w = w0 + u;
        const int rr = w / kTCM, kx = g * kTCM + (w - rr * kTCM);
        lds[rr * RSm + kx] = bx[i][u];
        lds[(kRWM + rr) * RSm + kx] = by[i][u];
      }
    }
  }
  if constexpr (LTW) tws.store(twl, tid);
  __syncthreads();
  cx<T> reg[E];
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int k = t + NT * q;
    const bool hi = k > NX / 2;
    const int kx = hi ? NX - k : k;
    const int li = r * RSm + kx;
    cx<T> X = lds[li], Y = lds[kRWM * RSm + li];
    if (kx == 0 || kx == NX / 2) {
      X.im = (T)0;
      Y.im = (T)0;
    }
    if (hi) {
      X.im = -X.im;
      Y.im = -Y.im;
    }
    reg[q] = cx<T>{X.re - Y.im, X.im + Y.re};
  }
  __syncthreads();
  if constexpr (LTW) fft<T, NX, true, E, true>(reg, lds + r * XS, t, (const cx<T>*)twl);
  else fft<T, NX, true, E, false>(reg, lds + r * XS, t, twg);
  double a_dd = 0.0, a_mx = 0.0;
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const size_t i = (size_t)y * NX + t + NT * q;
    const double xv = (double)reg[q].re * m.scale, yv = (double)reg[q].im * m.scale;
    if (mode == MON_OUTPUT) {
      s_out[i] = (T)yv;
    } else if (pn2[q] >= (T)0) {
      const double dd = yv + ((double)pn2[q] + m.nw_off) * xv - (double)pdd[q];
      a_dd += dd * dd;
      if (mode == MON_REFINE) gmem(m.rout)[i] = (float)(-dd);
    } else {
      a_mx += xv * xv;
      if (mode == MON_REFINE) gmem(m.rout)[i] = 0.0f;
    }
  }
  if (mode == MON_OUTPUT) return;
  a_dd = block_reduce<RED_SUM>(a_dd, sh);
  a_mx = block_reduce<RED_SUM>(a_mx, sh);
  if (tid == 0) {
    WF_GLOBAL double* part = gmem(m.part);
    part[2 * band] = a_dd;
    part[2 * band + 1] = a_mx;
  }
}

// Refinement: x = S_chain^-1 u of a finished solve, t / (S_chain + T) per mode
// in float64 from the solve's stored messenger t (state layout [kx][ky]; the
// real columns k_x = 0 and nx/2 hold k_y <= ny/2 only, the rest is the
// conjugate of the mirrored mode), added to (or, first, stored in) xacc.
template <class S>
__global__ __launch_bounds__(256) void accum_x_kernel(const cx<S>* __restrict__ tA,
                                                      const S* __restrict__ sc, double Tf,
                                                      int ny, int nx, int first,
                                                      cx<double>* __restrict__ xacc) {
  const int nh = nx / 2 + 1;
  const int64_t n = (int64_t)nh * ny;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int kx = (int)(j / ny), ky = (int)(j - (int64_t)kx * ny);
    const bool mir = (kx == 0 || kx == nx / 2) && ky > ny / 2;
    const int64_t src = mir ? (int64_t)kx * ny + (ny - ky) : j;
    const cx<S> t = tA[src];
    const double inv = 1.0 / ((double)sc[src] + Tf);
    const double xr = (double)t.re * inv, xi = (mir ? -(double)t.im : (double)t.im) * inv;
    if (first) {
      xacc[j] = cx<double>{xr, xi};
    } else {
      const cx<double> o = xacc[j];
      xacc[j] = cx<double>{o.re + xr, o.im + xi};
    }
  }
}

// precision conversion of an input array (refinement: float32 copies)
template <class S, class D>
__global__ __launch_bounds__(256) void convert_kernel(const S* __restrict__ src, int64_t n,
                                                      D* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (D)src[i];
}

// fixed-order sum of the monitor's (dd^2, masked x^2) block pairs
__global__ __launch_bounds__(256) void pair_sum_kernel(const double* __restrict__ part, int nblk,
                                                       double* __restrict__ out);

// fill / scale helpers for the inverse-noise weighting (S = alpha I)
template <class T>
__global__ __launch_bounds__(256) void fill_kernel(T* __restrict__ x, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = (T)v;
}

template <class T>
__global__ __launch_bounds__(256) void scale_kernel(T* __restrict__ x, int64_t n, double f) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = (T)((double)x[i] * f);
}

#if WF_PART & 1
// Thread t's share of a fixed-order sum over n partials: elements t, t + B,
// t + 2B, ... (B = blockDim.x) added in that order, their loads issued U at a
// time before the adds (a loop of load-wait-add pairs waited on memory once
// per element).  Pairs when PAIR (two sums over interleaved values).
template <bool PAIR>
__device__ __forceinline__ void thread_sums(const WF_GLOBAL double* v, int n, double& a,
                                            double& b) {
  constexpr int U = 8;
  const int B = blockDim.x;
  for (int i0 = threadIdx.x; i0 < n; i0 += U * B) {
    double x[U], y[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * B;
      x[u] = i < n ? v[PAIR ? 2 * i : i] : 0.0;
      y[u] = (PAIR && i < n) ? v[2 * i + 1] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (i0 + u * B < n) {
        a += x[u];
        if (PAIR) b += y[u];
      }
    }
  }
}

__global__ __launch_bounds__(256) void pair_sum_kernel(const double* __restrict__ part, int nblk,
                                                       double* __restrict__ out) {
  __shared__ double sh[16];
  double a = 0.0, b = 0.0;
  thread_sums<true>(gmem(part), nblk, a, b);
  a = block_reduce<RED_SUM>(a, sh);
  b = block_reduce<RED_SUM>(b, sh);
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = b;
  }
}

// One block: fixed-order reduction of the monitor partials, then the cooling
// schedule (fixed array, or the plateau rule of Section 3.3) and the stop test.
__global__ __launch_bounds__(256) void controller_kernel(const CtrlArgs* __restrict__ argv) {
  // one block per map
  const CtrlArgs& ca = argv[blockIdx.x];
  DevSched* s = ca.sch;
  double* lam = ca.lam;
  const double* __restrict__ part = ca.part;
  const int nblk = ca.nblk;
  double* __restrict__ trace = ca.trace;
  __shared__ double sh[16];
  if (s->done) return;
  double a = 0.0, b = 0.0, jv = 0.0, unused = 0.0;
  thread_sums<true>(gmem(part), nblk, a, b);
  thread_sums<false>(gmem(ca.jpart), ca.njblk, jv, unused);
  a = block_reduce<RED_SUM>(a, sh);
  b = block_reduce<RED_SUM>(b, sh);
  jv = block_reduce<RED_SUM>(jv, sh);
  if (threadIdx.x != 0) return;
  const int klast = min(s->base + s->K, s->max_sweeps) - 1;
  const double l = lam[klast];
  const double rho = sqrt(a / s->d2);
  const double rho_mask = s->nu * sqrt(b) / sqrt(s->d2);
  if (s->n_rec < s->max_rec) {
    double* r = trace + kTraceCols * s->n_rec;
    r[0] = (double)klast;
    r[1] = l;
    r[2] = rho;
    r[3] = a;
    r[4] = rho_mask;
    r[5] = jv;
    s->n_rec = s->n_rec + 1;
  }
  s->rho = rho;
  s->rho_mask = rho_mask;
  s->dd2 = a;
  s->masked_x = sqrt(b);
  s->J = jv;
  s->lam_last = l;
  s->sweeps_done = klast + 1;
  const double test = s->stop_full ? hypot(rho, rho_mask) : rho;
  if (!isfinite(a) || !isfinite(b)) {
    s->status = -3;  // WF_ENONFINITE
    s->done = 1;
  } else if (l == 1.0 && test <= s->rtol) {
    s->status = 0;
    s->done = 1;
  } else if (klast + 1 >= s->max_sweeps) {
    s->status = 1;  // WF_NOT_CONVERGED
    s->done = 1;
  } else if (s->adaptive) {
    double ln = l;
    if (s->have_prev && fabs(a - s->dd2_prev) < s->plateau * (double)(klast - s->k_prev) * a) {
      ln = pow(l, s->shrink);
      if (ln - 1.0 < s->snap) ln = 1.0;
    }
    const int end = min(klast + s->K, s->max_sweeps - 1);
    for (int k = klast + 1; k <= end; ++k) lam[k] = ln;
    s->dd2_prev = a;
    s->k_prev = klast;
    s->have_prev = 1;
  }
  s->base = klast + 1;
}
#endif

// ---------------------------------------------------------------------------
// explicit instantiations and launch helpers (host-callable, C++ linkage)
// ---------------------------------------------------------------------------
}  // namespace wf

#include "wf_launch.inc"
