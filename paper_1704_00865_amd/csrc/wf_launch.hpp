// Host-callable launch helpers for the kernels in wf_kernels.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "wf_kernels.hpp"

namespace wf {

// transit-buffer tile: TR rows x TC columns per tile, RW rows per row block
struct TileCfg {
  int TR, TC, RW;
};
constexpr int kNumTiles = 7;
constexpr int kTileDefault = 1;
extern const TileCfg kTiles[kNumTiles];

// Every launch covers nmaps maps of one shape and chain kind: argv is a
// DEVICE array of nmaps argument blocks (blockIdx.y selects one); a / m is a
// host copy of one of them, for the sizes.
// e0, e1 (optional, sweep modes): events the dispatch itself records at the
// kernel's start and end.
template <class T>
hipError_t launch_row(int cfg, int mode, const SweepArgs<T>& a, const SweepArgs<T>* argv,
                      int nmaps, int k_local, const T* xin, T* xout, hipStream_t st,
                      hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
template <class T>
hipError_t launch_col(int cfg, int mode, const SweepArgs<T>& a, const SweepArgs<T>* argv,
                      int nmaps, int k_local, void* spec, double lam_init, hipStream_t st,
                      hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
template <class T>
hipError_t launch_mon_col(const MonArgs<T>& m, const MonArgs<T>* argv, int nmaps, int mode,
                          hipStream_t st);
template <class T>
hipError_t launch_mon_row(const MonArgs<T>& m, const MonArgs<T>* argv, int nmaps, int mode,
                          hipStream_t st);
hipError_t launch_controller(const CtrlArgs* argv, int nmaps, hipStream_t st);
// refinement helpers: x of a float32 solve added to a float64 accumulator,
// float64 -> float32 input copies, and the monitor's pair sums
hipError_t launch_accum_x(const void* tA, const float* sc, double Tf, int ny, int nx, int first,
                          void* xacc, hipStream_t st);
hipError_t launch_to_float(const double* src, int64_t n, float* dst, hipStream_t st);
hipError_t launch_pair_sum(const double* part, int nblk, double* out, hipStream_t st);
template <class T>
hipError_t launch_stats(const T* d, const T* npix, const uint8_t* mask, const T* sk, const T* poof,
                        const T* pst, int ny, int nx, double* part, int nblk, double* out_pix,
                        double* out_spec, hipStream_t st);
template <class T>
// per-pixel and per-mode coefficients; also zeroes the transit buffer zB and
// the three per-mode state arrays zA, zD, zT (the zero start)
hipError_t launch_prep(const T* npix, const uint8_t* mask, int ny, int nx, double sub, T* nbar2,
                       const T* sk, const T* poof, const T* pst, const PrepSpecArgs& pa, T* sc, T* nbA,
                       T* sy, T* sig, void* zB, void* zA, void* zD, void* zT, hipStream_t st);

template <class T>
hipError_t launch_fill(T* x, int64_t n, double v, hipStream_t st);
template <class T>
hipError_t launch_scale(T* x, int64_t n, double f, hipStream_t st);

}  // namespace wf
