// Kernel-side data structures shared by wf_kernels.hip and the host runtime.
#pragma once

#include <stdint.h>

#include "wf_fft.hpp"

namespace wf {

// tile of the monitor's transit buffers (kTRM rows x kTCM columns: 128
// contiguous bytes in float32), and the rows one monitor row block takes
constexpr int kTRM = 8;
constexpr int kTCM = 2;
constexpr int kRWM = 2;

// Fourier side of the messenger chain (levels between the signal and the
// pixel-space white level)
enum FourierKind : int32_t {
  FK_NONE = 0,          // no Fourier level: augmented chain or white noise only
  FK_ARRAY = 1,         // one level, Nbar from an array (1/f alone, or merged)
  FK_STRIPE = 2,        // one level, the stripe level (no 1/f term)
  FK_ARRAY_STRIPE = 3,  // 1/f level (signal side) then the stripe level
};

// ROW_SWEEP_J / COL_SWEEP_J: a sweep that also sums the joint objective's
// terms (eqn 2mess_prob) when it is the last sweep of its chunk; the column
// variant then also runs the monitor's column transforms into Mx, My
enum RowMode : int32_t { ROW_SWEEP = 0, ROW_R2C = 1, ROW_C2R = 2, ROW_SWEEP_J = 3 };
enum ColMode : int32_t { COL_SWEEP = 0, COL_FWD_OUT = 1, COL_INV_IN = 2, COL_INIT = 3,
                         COL_SWEEP_J = 4 };
// MON_RESIDUAL: residual sums of the state after a chunk (during a solve the
// column pass of this mode runs inside the chunk's last column sweep, and
// only the row kernel is launched).  MON_OUTPUT: the output field.
// MON_REFINE: the residual sums of MON_RESIDUAL and the float32 right-hand
// side d - d_rec (zero on masked pixels) to rout.
enum MonMode : int32_t { MON_RESIDUAL = 0, MON_OUTPUT = 1, MON_REFINE = 3 };

// Schedule state resident on the device.  Sweep kernels read it; only the
// controller kernel (after each monitor) writes it.
struct DevSched {
  int32_t base;        // first sweep of the current chunk
  int32_t done;        // 1: converged / failed / budget spent -> kernels skip
  int32_t status;      // wf_status once done
  int32_t max_sweeps;
  int32_t K;           // sweeps per chunk (monitor interval)
  int32_t adaptive;
  int32_t n_rec;       // trace records written
  int32_t max_rec;
  int32_t have_prev;
  int32_t k_prev;
  int32_t stop_full;
  int32_t sweeps_done;
  double shrink, plateau, snap, rtol;
  double d2;           // sum of d^2 over observed pixels
  double nu;           // largest observed white variance
  double dd2_prev;
  double rho, rho_mask, dd2, lam_last;
  double masked_x;     // |(1 - m) x| at the last check
  double J;            // joint objective J_lambda at the last check
};

template <class T>
struct SweepArgs {
  void* B;                // transit buffer, cx<T>, nx/2 packed columns, tiled [y/TR][kx/TC][TR][TC]
  void* tA;               // state: t of the signal-side Fourier level (or t_white copy)
  void* dA;               // state: d of that level (FK_ARRAY_STRIPE only)
  void* tB;               // state: t of the stripe level (FK_ARRAY_STRIPE only)
  const T* sc;            // [kx][ky] covariance of the chain's signal end
  const T* nbA;           // [kx][ky] Nbar of the array level
  const T* pst;           // [ny] stripe mode variance (caller's array)
  const T* d;             // [ny][nx] data (caller's array)
  const T* nbar2;         // [ny][nx] Nbar of the white level, < 0 where masked
  const void* twx;        // w_nx^j table, cx<T>
  const void* twy;        // w_ny^j table, cx<T>
  const DevSched* sch;
  const double* lam;      // lambda per sweep index
  int32_t nx, ny;
  int32_t fk;             // FourierKind
  double tauA, tauB, tauW;  // messenger variances (A: signal-side level)
  double cB;              // Nbar offset of a stripe level (phi - tau)
  double scale;           // 1 / (nx ny)
  int32_t warm_chain;     // warm start gives the chain's signal-end field itself
  int32_t jrow;           // row-kernel blocks: column partials of J start there
  double* jpart;          // per-block partial sums of the joint objective
  // the monitor's column pass, run by the chunk's last column sweep
  const T* sy;            // [kx][ky] factor of y = (S + N_F) x for the residual
  void* Mx;               // monitor transit, tiled [y/kTRM][kx/kTCM][kTRM][kTCM]
  void* My;
  int32_t kpm;            // monitor transit columns (nx/2 + 1, padded to kTCM)
};

// per-mode coefficient preparation (see prep_spectra_kernel)
// An infinite noise variance on a Fourier mode (a 1/f spectrum entry of
// +inf) projects that mode out of the data (Section 4).  It is carried as
// this finite value: every update of the multiplied form then takes its
// limit up to a relative 1e-30 * (largest other covariance).  The sweep
// normalises each pair of weights before multiplying a field by it, so no
// product of this value with a field is formed.
constexpr double kInfiniteCov = 1.0e30;

struct PrepSpecArgs {
  int ny, nx;
  int has_oof, has_st;
  int sc_adds_nf;      // augmented chain: sc = S + N_F (+ phi_nf)
  int nbA_kind;        // 0 none, 1: P_1/f - tau, 2: N_F (+phi_nf) - tau
  double phi_nf;       // floor added to N_F when the stripes have no 1/f partner
  double tauA;
};

template <class T>
struct MonArgs {
  const void* tfirst;   // cx<T> [kx][ky]: t of the chain's signal-end level
  const T* sc;          // [kx][ky] S_chain
  const T* sy;          // [kx][ky] S + N_Fourier
  const T* sig;         // [kx][ky] S
  const T* d;           // [ny][nx]
  const T* nbar2;       // [ny][nx] sign marks the mask
  double nw_off;        // white variance = nbar2 + nw_off on observed pixels
  void* Mx;             // cx<T> monitor transit, tiled [y/kTRM][kx/kTCM][kTRM][kTCM]
  void* My;
  const void* twx;      // cx<T> twiddle tables (natural order)
  const void* twy;
  const DevSched* sch;
  const double* lam;
  double* part;         // per-block (sum dd^2, sum masked x^2)
  void* s_out;          // T [ny][nx]: output of the final (output-mode) pass
  int nx, ny, kpm;      // kpm: padded half width (multiple of kTCM)
  double tau_first;
  double scale;
  int32_t out_chain;    // output u = S_chain x instead of s = S x
  int32_t x_direct;     // tfirst holds x itself (refinement), not a messenger
  float* rout;          // MON_REFINE: [ny][nx] right-hand side of the next solve
};

// per-map arguments of the controller (one block per map)
struct CtrlArgs {
  DevSched* sch;
  double* lam;
  const double* part;
  int nblk;
  double* trace;       // kTraceCols values per monitor record
  const double* jpart; // joint-objective partials of the chunk's last sweep
  int njblk;
};

// columns of a trace record: sweep, lambda, rho, dd2, rho_mask, J
constexpr int kTraceCols = 6;

}  // namespace wf
