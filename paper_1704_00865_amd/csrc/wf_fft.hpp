// Workgroup FFTs for gfx950: radix-16/12/8/4/2 Stockham passes with the data in
// registers and one LDS exchange between passes.
//
// A transform of length N (a power of two from 64 to 4096, or 3 times one:
// 384, 768, 1536) is spread over NT = N/E threads that each hold E complex
// values (E = 16, or 12 when N has a factor 3).  Register q of thread t holds
// element t + NT*q both before the first pass and after the last one (natural
// order), so a transform can be followed by per-element work and by another
// transform without any reshuffle, and its first loads and last stores are
// coalesced.  Pass j with radix R and span p (product of the earlier radices)
// computes, for butterfly i in [0, N/R):
//     u_m = x[i + m N/R] * w_{pR}^{m (i mod p)},  U = DFT_R(u),
//     y[(i - i mod p) R + (i mod p) + m p] = U_m,
// the autosorting Stockham form (radix 16, 12, 8, 4, 2).  Twiddles w_N^j come from a table built in
// double precision on the host and rounded once (no device sin/cos).
#pragma once

#include <hip/hip_runtime.h>

namespace wf {

template <class T>
struct cx {
  T re, im;
};

// Buffers reached through pointers stored in argument blocks in device memory
// are generic to the compiler, which then emits flat loads and stores: their
// completion is counted with the LDS operations, so every wait for an LDS
// exchange also waits for outstanding memory traffic.  Kernels address such
// buffers through global-memory pointers (gmem) instead.
#define WF_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ WF_GLOBAL T* gmem(T* p) {
  return (WF_GLOBAL T*)p;
}
// complex loads and stores through either kind of pointer (a class object in
// global memory is copied field by field)
template <class T>
__device__ __forceinline__ cx<T> ldc(const cx<T>* p) {
  return *p;
}
template <class T>
__device__ __forceinline__ cx<T> ldc(const WF_GLOBAL cx<T>* p) {
  return cx<T>{p->re, p->im};
}
template <class T>
__device__ __forceinline__ void stc(WF_GLOBAL cx<T>* p, cx<T> v) {
  p->re = v.re;
  p->im = v.im;
}

template <class T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.re * s, a.im * s}; }

// multiply by w_4 = -i (forward) or +i (inverse)
template <class T, bool INV>
__device__ __forceinline__ cx<T> mul_w4(cx<T> a) {
  return INV ? cx<T>{-a.im, a.re} : cx<T>{a.im, -a.re};
}

// cos and sin of j*pi/8, j = 0..15
__device__ constexpr double kC16[16] = {
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
__device__ constexpr double kS16[16] = {
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173};

// w_16^j = exp(-+ 2 pi i j / 16) (minus for the forward transform)
template <class T, bool INV>
__device__ __forceinline__ cx<T> w16(int j) {
  const T c = (T)kC16[j & 15];
  const T s = (T)kS16[j & 15];
  return INV ? cx<T>{c, s} : cx<T>{c, -s};
}

template <class T, bool INV>
__device__ __forceinline__ void dft2(cx<T>* u) {
  const cx<T> a = u[0], b = u[1];
  u[0] = a + b;
  u[1] = a - b;
}

template <class T, bool INV>
__device__ __forceinline__ void dft4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
  const cx<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3;
  const cx<T> t3 = mul_w4<T, INV>(a1 - a3);
  a0 = t0 + t2;
  a2 = t0 - t2;
  a1 = t1 + t3;
  a3 = t1 - t3;
}

template <class T, bool INV>
__device__ __forceinline__ void dft4(cx<T>* u) { dft4<T, INV>(u[0], u[1], u[2], u[3]); }

// 8 = 4 (n1) x 2 (n2): n = 2 n1 + n2, k = k1 + 4 k2
template <class T, bool INV>
__device__ __forceinline__ void dft8(cx<T>* u) {
  cx<T> y0[4] = {u[0], u[2], u[4], u[6]};
  cx<T> y1[4] = {u[1], u[3], u[5], u[7]};
  dft4<T, INV>(y0);
  dft4<T, INV>(y1);
#pragma unroll
  for (int k1 = 1; k1 < 4; ++k1) y1[k1] = cmul(y1[k1], w16<T, INV>(2 * k1));
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    u[k1] = y0[k1] + y1[k1];
    u[k1 + 4] = y0[k1] - y1[k1];
  }
}

// 16 = 4 (n1) x 4 (n2): n = 4 n1 + n2, k = k1 + 4 k2
template <class T, bool INV>
__device__ __forceinline__ void dft16(cx<T>* u) {
  cx<T> y[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    y[n2][0] = u[n2];
    y[n2][1] = u[4 + n2];
    y[n2][2] = u[8 + n2];
    y[n2][3] = u[12 + n2];
    dft4<T, INV>(y[n2]);
  }
#pragma unroll
  for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1) y[n2][k1] = cmul(y[n2][k1], w16<T, INV>(n2 * k1));
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cx<T> a0 = y[0][k1], a1 = y[1][k1], a2 = y[2][k1], a3 = y[3][k1];
    dft4<T, INV>(a0, a1, a2, a3);
    u[k1] = a0;
    u[k1 + 4] = a1;
    u[k1 + 8] = a2;
    u[k1 + 12] = a3;
  }
}

// 3-point DFT: w_3 = -1/2 -+ i sqrt(3)/2 (minus for the forward transform)
template <class T, bool INV>
__device__ __forceinline__ void dft3(cx<T>* u) {
  const T c = (T)-0.5, s = (T)(INV ? 0.86602540378443864676 : -0.86602540378443864676);
  const cx<T> a0 = u[0], a1 = u[1], a2 = u[2];
  const cx<T> sm = a1 + a2, df = a1 - a2;
  const cx<T> m = {a0.re + c * sm.re, a0.im + c * sm.im};
  const cx<T> r = {-s * df.im, s * df.re};  // i s (a1 - a2)
  u[0] = a0 + sm;
  u[1] = m + r;
  u[2] = m - r;
}

// 12 = 3 (n1) x 4 (n2): n = 4 n1 + n2, k = k1 + 3 k2.  Three-point DFTs over
// n1, twiddles w_12^(n2 k1), four-point DFTs over n2.
template <class T, bool INV>
__device__ __forceinline__ void dft12(cx<T>* u) {
  const T h = (T)0.5, r3 = (T)0.86602540378443864676;  // cos 60, sin 60 degrees
  cx<T> y[4][3];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    y[n2][0] = u[n2];
    y[n2][1] = u[4 + n2];
    y[n2][2] = u[8 + n2];
    dft3<T, INV>(y[n2]);
  }
  // w_12^j for j = 1, 2, 4 (forward: exp(-i pi j / 6)); j = 3 is -+i, j = 6 is -1
  const T sg = INV ? (T)1 : (T)-1;
  const cx<T> w1 = {r3, sg * h}, w2 = {h, sg * r3}, w4 = {-h, sg * r3};
  y[1][1] = cmul(y[1][1], w1);
  y[1][2] = cmul(y[1][2], w2);
  y[2][1] = cmul(y[2][1], w2);
  y[2][2] = cmul(y[2][2], w4);
  y[3][1] = mul_w4<T, INV>(y[3][1]);
  y[3][2] = cx<T>{-y[3][2].re, -y[3][2].im};
#pragma unroll
  for (int k1 = 0; k1 < 3; ++k1) {
    cx<T> a0 = y[0][k1], a1 = y[1][k1], a2 = y[2][k1], a3 = y[3][k1];
    dft4<T, INV>(a0, a1, a2, a3);
    u[k1] = a0;
    u[k1 + 3] = a1;
    u[k1 + 6] = a2;
    u[k1 + 9] = a3;
  }
}

template <class T, int R, bool INV>
__device__ __forceinline__ void dft(cx<T>* u) {
  if constexpr (R == 2) dft2<T, INV>(u);
  else if constexpr (R == 3) dft3<T, INV>(u);
  else if constexpr (R == 4) dft4<T, INV>(u);
  else if constexpr (R == 8) dft8<T, INV>(u);
  else if constexpr (R == 12) dft12<T, INV>(u);
  else if constexpr (R == 16) dft16<T, INV>(u);
}

// complex values held by each thread: 16 for powers of two, 12 for lengths
// with a factor 3 (radices 4, 2 and 12 divide it; with 24 values and radix 8
// a 1536-point transform filled one wave, whose 12 KB exchange buffer held
// the kernels to 1.5-2 waves per SIMD)
template <int N>
struct elems {
  static constexpr int value = (N % 3 == 0) ? 12 : 16;
};

// Index map of one transform's LDS exchange buffer (N complex values, E per
// thread, NT = N/E threads).  With 8-byte values and at least one wave per
// transform, the low five bits of the index are XORed with those of
// 5 (j >> 5): each aligned run of 32 values is permuted within itself, so
// natural-order accesses stay free of bank conflicts, while the strided stores
// of the passes spread over the 64 banks.  When NT is a multiple of 256 only
// bits 5-7 enter the XOR (as few conflicts in the passes of those plans), so
// that element t + NT q of thread t (t < NT) sits at at(t) + NT q: the natural
// order accesses of a thread need one address computation instead of E.
// Buffers of one block are N + 16 values apart (32 banks), so a wave that
// touches two of them does not collide with itself.  Otherwise (16-byte
// values, or several transforms per wave) one pad value per 16, and buffers
// N + N/16 + 8 values apart, so that neighbouring buffers start on different
// banks; at(t + NT q) = at(t) + q (NT + NT/16) there when 16 divides NT.
template <class T, int N, int E>
struct ldsmap {
  static constexpr int NT = N / E;
  static constexpr bool swz = sizeof(T) == 4 && NT >= 64;
  static constexpr bool swz3 = swz && NT % 256 == 0;
  static_assert(!swz || N % 32 == 0, "the swizzle permutes aligned runs of 32");
  static constexpr int size = swz ? N + 16 : N + N / 16 + 8;
  __device__ __forceinline__ static int at(int j) {
    if constexpr (swz3) return j ^ ((5 * ((j >> 5) & 7)) & 31);
    else if constexpr (swz) return j ^ ((5 * (j >> 5)) & 31);
    else return j + (j >> 4);
  }
  // at(t + NT q) for 0 <= t < NT
  __device__ __forceinline__ static int at_tq(int t, int q) {
    if constexpr (swz3) return at(t) + NT * q;
    else if constexpr (!swz && NT % 16 == 0) return at(t) + q * (NT + NT / 16);
    else return at(t + NT * q);
  }
};

// radix plan R0 * R1 * R2 * R3 * R4 = N (1 = no pass); the radix-12 pass of
// the lengths with a factor 3 comes last, so every earlier span is a power of two
template <int N>
struct plan;
template <> struct plan<64> { static constexpr int r[5] = {16, 4, 1, 1, 1}; };
template <> struct plan<128> { static constexpr int r[5] = {16, 8, 1, 1, 1}; };
template <> struct plan<256> { static constexpr int r[5] = {16, 16, 1, 1, 1}; };
template <> struct plan<512> { static constexpr int r[5] = {16, 8, 4, 1, 1}; };
template <> struct plan<1024> { static constexpr int r[5] = {16, 16, 4, 1, 1}; };
template <> struct plan<2048> { static constexpr int r[5] = {16, 16, 8, 1, 1}; };
template <> struct plan<4096> { static constexpr int r[5] = {16, 16, 16, 1, 1}; };
template <> struct plan<384> { static constexpr int r[5] = {4, 4, 2, 12, 1}; };
template <> struct plan<768> { static constexpr int r[5] = {4, 4, 4, 12, 1}; };
template <> struct plan<1536> { static constexpr int r[5] = {4, 4, 4, 2, 12}; };

constexpr int kE = 16;  // values per thread for power-of-two lengths

// radix plan for a transform spread over E values per thread: the default
// plan, or (E = 8) radices of at most 8
template <int N, int E>
struct plan_for {
  static constexpr int r0 = plan<N>::r[0], r1 = plan<N>::r[1], r2 = plan<N>::r[2], r3 = plan<N>::r[3],
                       r4 = plan<N>::r[4];
};
template <> struct plan_for<1024, 8> { static constexpr int r0 = 8, r1 = 8, r2 = 4, r3 = 4, r4 = 1; };
template <> struct plan_for<2048, 8> { static constexpr int r0 = 8, r1 = 8, r2 = 8, r3 = 4, r4 = 1; };
template <> struct plan_for<4096, 8> { static constexpr int r0 = 8, r1 = 8, r2 = 8, r3 = 8, r4 = 1; };

// Twiddle tables.  The natural table holds w_N^j (forward sign) at j; pass
// (span P, radix R) reads it at j = m k N/(P R), so that the lanes of one read
// fall on a few LDS banks.  The pass-major table of a radix plan holds, for
// every pass after the first in order, w_N^{m k N/(P R)} at
// off + (m - 1) P + k (m = 1..R-1, k = 0..P-1): lanes with consecutive k read
// consecutive entries.  It has N - R0 entries (the spans grow by the factor R,
// so the passes' counts (R - 1) P add up to N - R0).
template <int N, int E>
struct twp_offsets {
  using PL = plan_for<N, E>;
  static constexpr int p1 = PL::r0, p2 = p1 * PL::r1, p3 = p2 * PL::r2, p4 = p3 * PL::r3;
  static constexpr int o2 = 0;                             // pass 2 (span p1)
  static constexpr int o3 = o2 + (PL::r1 - 1) * p1;        // pass 3 (span p2)
  static constexpr int o4 = o3 + (PL::r2 - 1) * p2;        // pass 4 (span p3)
  static constexpr int o5 = o4 + (PL::r3 - 1) * p3;        // pass 5 (span p4)
  static constexpr int size = N - p1;
};

// Natural-table index of entry e of the pass-major table of plan_for<N, E>.
template <int N, int E>
__device__ __forceinline__ int twp_source(int e) {
  using PL = plan_for<N, E>;
  using O = twp_offsets<N, E>;
  if (e < O::o3) {
    const int o = e - O::o2, m = 1 + o / O::p1, k = o - (m - 1) * O::p1;
    return m * k * (N / (O::p1 * PL::r1));
  } else if (e < O::o4) {
    const int o = e - O::o3, m = 1 + o / O::p2, k = o - (m - 1) * O::p2;
    return m * k * (N / (O::p2 * PL::r2));
  }
  if (e < O::o5) {
    const int o = e - O::o4, m = 1 + o / O::p3, k = o - (m - 1) * O::p3;
    return m * k * (N / (O::p3 * PL::r3));
  }
  const int o = e - O::o5, m = 1 + o / O::p4, k = o - (m - 1) * O::p4;
  return m * k * (N / (O::p4 * PL::r4));
}

// Staging of the pass-major table into LDS by NTHR threads, in two steps so
// that a kernel can issue every global load it needs (its own data and the
// table) before the first wait: load() fetches this thread's share into
// registers, store() writes it to the LDS table.
template <class T, int N, int E, int NTHR>
struct TwiddleStage {
  using O = twp_offsets<N, E>;
  static constexpr int PER = (O::size + NTHR - 1) / NTHR;
  cx<T> v[PER];
  template <class TW>
  __device__ __forceinline__ void load(TW tw, int tid) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = tid + i * NTHR;
      if (e < O::size) v[i] = ldc(tw + twp_source<N, E>(e));
    }
  }
  __device__ __forceinline__ void store(cx<T>* twp, int tid) const {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = tid + i * NTHR;
      if (e < O::size) twp[e] = v[i];
    }
  }
};

// Fill the pass-major table twp (LDS, twp_offsets::size entries) from the
// natural table tw with NTHR threads (loads first, then the LDS writes).
template <class T, int N, int E, int NTHR, class TW>
__device__ __forceinline__ void stage_twiddles(cx<T>* twp, TW tw, int tid) {
  TwiddleStage<T, N, E, NTHR> s;
  s.load(tw, tid);
  s.store(twp, tid);
}

// One Stockham pass.  reg: the thread's E values; lds: this transform's
// padded exchange buffer; tw: the natural twiddle table (OFF < 0) or the
// pass-major one, whose entries for this pass start at OFF.
template <class T, int N, int R, int P, bool INV, bool LAST, int E = elems<N>::value, int OFF = -1,
          class TW = const cx<T>*>
__device__ __forceinline__ void stockham_pass(cx<T>* reg, cx<T>* lds, int t, TW tw) {
  constexpr int NT = N / E;
  constexpr int NB = E / R;
  using LM = ldsmap<T, N, E>;
  static_assert(E % R == 0, "radix must divide the values per thread");
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int i = t + b * NT;
    const int k = i & (P - 1);
    cx<T> u[R];
#pragma unroll
    for (int m = 0; m < R; ++m) u[m] = reg[b + m * NB];
    if constexpr (P > 1) {
      constexpr int STEP = N / (P * R);
#pragma unroll
      for (int m = 1; m < R; ++m) {
        cx<T> w = ldc(OFF >= 0 ? tw + (OFF + (m - 1) * P + k) : tw + m * k * STEP);
        if (INV) w.im = -w.im;
        u[m] = cmul(u[m], w);
      }
    }
    dft<T, R, INV>(u);
    if constexpr (LAST) {
#pragma unroll
      for (int m = 0; m < R; ++m) reg[b + m * NB] = u[m];
    } else {
      const int j = (i - k) * R + k;
#pragma unroll
      for (int m = 0; m < R; ++m) lds[LM::at(j + m * P)] = u[m];
    }
  }
  if constexpr (!LAST) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < E; ++q) reg[q] = lds[LM::at_tq(t, q)];
    __syncthreads();
  }
}

// Full transform of length N.  Every thread of the workgroup must call it
// (it contains barriers); lds must hold ldsmap<T, N, E>::size elements per
// transform and must not be in use by the caller.  tw is the natural
// twiddle table, or the pass-major one of plan_for<N, E> when TWP.
template <class T, int N, bool INV, int E = elems<N>::value, bool TWP = false,
          class TW = const cx<T>*>
__device__ __forceinline__ void fft(cx<T>* reg, cx<T>* lds, int t, TW tw) {
  using PL = plan_for<N, E>;
  using O = twp_offsets<N, E>;
  constexpr int R0 = PL::r0, R1 = PL::r1, R2 = PL::r2, R3 = PL::r3, R4 = PL::r4;
  static_assert(R0 * R1 * R2 * R3 * R4 == N, "radix plan must multiply to N");
  constexpr int F2 = TWP ? O::o2 : -1, F3 = TWP ? O::o3 : -1, F4 = TWP ? O::o4 : -1,
                F5 = TWP ? O::o5 : -1;
  constexpr int P2 = R0 * R1, P3 = P2 * R2, P4 = P3 * R3;
  if constexpr (R2 == 1) {
    stockham_pass<T, N, R0, 1, INV, false, E, -1, TW>(reg, lds, t, tw);
    stockham_pass<T, N, R1, R0, INV, true, E, F2, TW>(reg, lds, t, tw);
  } else if constexpr (R3 == 1) {
    stockham_pass<T, N, R0, 1, INV, false, E, -1, TW>(reg, lds, t, tw);
    stockham_pass<T, N, R1, R0, INV, false, E, F2, TW>(reg, lds, t, tw);
    stockham_pass<T, N, R2, P2, INV, true, E, F3, TW>(reg, lds, t, tw);
  } else if constexpr (R4 == 1) {
    stockham_pass<T, N, R0, 1, INV, false, E, -1, TW>(reg, lds, t, tw);
    stockham_pass<T, N, R1, R0, INV, false, E, F2, TW>(reg, lds, t, tw);
    stockham_pass<T, N, R2, P2, INV, false, E, F3, TW>(reg, lds, t, tw);
    stockham_pass<T, N, R3, P3, INV, true, E, F4, TW>(reg, lds, t, tw);
  } else {
    stockham_pass<T, N, R0, 1, INV, false, E, -1, TW>(reg, lds, t, tw);
    stockham_pass<T, N, R1, R0, INV, false, E, F2, TW>(reg, lds, t, tw);
    stockham_pass<T, N, R2, P2, INV, false, E, F3, TW>(reg, lds, t, tw);
    stockham_pass<T, N, R3, P3, INV, false, E, F4, TW>(reg, lds, t, tw);
    stockham_pass<T, N, R4, P4, INV, true, E, F5, TW>(reg, lds, t, tw);
  }
}

}  // namespace wf
