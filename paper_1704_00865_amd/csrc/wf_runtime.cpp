// Host runtime of the Wiener-filter library: context, validation, messenger
// set-up, the sweep loop with a device-resident cooling schedule, and the
// C ABI declared in include/wf.h.
//
// The loop enqueues chunks of K sweeps (2 launches each), then the float64
// monitor (2 launches) and the one-block controller that evaluates the
// schedule on the device.  The host never waits inside a chunk: it copies the
// controller's state to pinned memory after each chunk and checks it two
// chunks later, so the GPU keeps a queue of work; sweeps enqueued after
// convergence see the device's done flag and return at once, which keeps the
// result identical whatever the run-ahead.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "wf.h"
#include "wf_launch.hpp"

using namespace wf;

namespace {

constexpr int kStatBlocks = 1024;  // blocks of the validation statistics (partials in c->part)
constexpr int kRing = 4;   // pinned readback slots
constexpr int kLag = 2;    // chunks between enqueue and the host's check
constexpr int kProfSlots = 512;
constexpr int kStaticCheck = 4;  // chunks between host checks without events

struct Ctx {
  int ny = 0, nx = 0, prec = 0;
  int nh = 0, kpm = 0;
  int tile = kTileDefault;
  size_t esz = 0;
  int device = 0;
  void* B = nullptr;
  void* tA = nullptr;
  void* dA = nullptr;
  void* tB = nullptr;
  void* sc = nullptr;
  void* nbA = nullptr;
  void* sy = nullptr;
  void* sig = nullptr;
  void* nbar2 = nullptr;
  void* twx = nullptr;
  void* twy = nullptr;
  void* Mx = nullptr;  // monitor transit, context precision
  void* My = nullptr;
  double* part = nullptr;
  double* jpart = nullptr;   // joint-objective partials (row blocks, then column blocks)
  double* stats = nullptr;
  DevSched* sch = nullptr;
  double* lam = nullptr;
  int lam_cap = 0;
  double* trace = nullptr;
  int trace_cap = 0;
  void* alpha_sk = nullptr;  // flat signal spectrum for the inverse-noise weighting
  void* d_args = nullptr;    // device argument blocks of the single-map launches
  void* d_margs = nullptr;
  void* d_ctrl = nullptr;
  void* h_args = nullptr;    // pinned staging of the same
  void* h_margs = nullptr;
  void* h_ctrl = nullptr;
  DevSched* h_ring = nullptr;  // pinned
  double* h_stats = nullptr;   // pinned
  hipEvent_t ev_ring[kRing] = {};
  int profiling = 0;
  std::vector<hipEvent_t> prof_ev;
  // workspace carved from the library's static scratch (wf_solve_noalloc):
  // no events, no pinned memory, nothing to free
  bool no_alloc = false;
  // iterative refinement (wf_solve_refined), allocated on first use: on the
  // float32 context the float32 copies of the inputs (the data copy then
  // holds each round's right-hand side) and a dummy output; on the float64
  // context the monitor argument blocks of its three passes
  void* ref_d = nullptr;
  void* ref_npix = nullptr;
  void* ref_sk = nullptr;
  void* ref_poof = nullptr;
  void* ref_pst = nullptr;
  void* ref_out = nullptr;
  void* ref_init = nullptr;  // float32 copy of a warm start of round 0
  void* ref_margs = nullptr;
  // wf_solve_batch's per-call arrays when this context is a batch's first:
  // per-map device schedules, argument blocks and controller arguments
  // (device), and the ring the host reads the schedules back into (pinned);
  // kept between calls and grown when a larger batch comes
  void* batch_dev = nullptr;
  size_t batch_dev_bytes = 0;
  void* batch_host = nullptr;
  size_t batch_host_bytes = 0;
  // one chunk of the single-map solve recorded as a HIP graph on cap_stream,
  // replayed for every chunk; valid for the (K, last sweep of the budget
  // within a chunk, tiling, chain kind) it was recorded with
  hipStream_t cap_stream = nullptr;
  hipGraph_t chunk_graph = nullptr;
  hipGraphExec_t chunk_exec = nullptr;
  int chunk_key[4] = {-1, -1, -1, -1};
};

// Every device buffer of a context with its size: take(&pointer, bytes) is
// called once per buffer in a fixed order.
template <class F>
void for_each_buffer(Ctx* c, F take) {
  const size_t ny = c->ny, nx = c->nx, nh = c->nh, esz = c->esz;
  const size_t modes = nh * ny;
  take((void**)&c->B, ny * (nx / 2) * 2 * esz);
  take((void**)&c->tA, modes * 2 * esz);
  take((void**)&c->dA, modes * 2 * esz);
  take((void**)&c->tB, modes * 2 * esz);
  take((void**)&c->sc, modes * esz);
  take((void**)&c->nbA, modes * esz);
  take((void**)&c->sy, modes * esz);
  take((void**)&c->sig, modes * esz);
  take((void**)&c->nbar2, ny * nx * esz);
  take((void**)&c->twx, nx * 2 * esz);
  take((void**)&c->twy, ny * 2 * esz);
  take((void**)&c->Mx, ny * c->kpm * 2 * esz);
  take((void**)&c->My, ny * c->kpm * 2 * esz);
  take((void**)&c->part, std::max<size_t>(2 * ny / kRWM, 16 * kStatBlocks) * sizeof(double));
  // at most ny/2 row blocks and nx/4 column blocks (every tiling has at
  // least 2 rows per row block and 2 columns per tile)
  take((void**)&c->jpart, (ny / 2 + nx / 4) * sizeof(double));
  take((void**)&c->stats, 16 * sizeof(double));
  take((void**)&c->sch, sizeof(DevSched));
  take((void**)&c->d_args, sizeof(SweepArgs<double>));
  take((void**)&c->d_margs, sizeof(MonArgs<double>));
  take((void**)&c->d_ctrl, sizeof(CtrlArgs));
}

wf_status from_hip(hipError_t e) {
  if (e == hipSuccess) return WF_OK;
  if (e == hipErrorOutOfMemory) return WF_ENOMEM;
  return WF_EDEVICE;
}

#define WF_TRY(expr)                      \
  do {                                    \
    hipError_t e_ = (expr);               \
    if (e_ != hipSuccess) return from_hip(e_); \
  } while (0)

// transform lengths with a built radix plan: powers of two 64..4096 (float64
// up to 2048) and 3 x 128, 3 x 256, 3 x 512
bool length_ok(int n, int prec) {
  if (n == 384 || n == 768 || n == 1536) return true;
  const int hi = prec == WF_F64 ? 2048 : 4096;
  return n >= 64 && n <= hi && (n & (n - 1)) == 0;
}

// lengths whose float32 kernels are built in every tiling (the others have
// the default tiling only)
bool tuned_length(int n) { return n == 256 || n == 768 || n == 1536 || n == 2048; }

int supported(int ny, int nx, int prec) {
  if (prec != WF_F32 && prec != WF_F64) return 0;
  return length_ok(ny, prec) && length_ok(nx, prec);
}

template <class T>
void make_table(std::vector<T>& out, int n) {
  out.resize(2 * (size_t)n);
  for (int j = 0; j < n; ++j) {
    const double ang = 2.0 * M_PI * (double)j / (double)n;
    out[2 * j] = (T)std::cos(ang);
    out[2 * j + 1] = (T)(-std::sin(ang));
  }
}

void free_ctx(Ctx* c) {
  void* bufs[] = {c->B, c->tA, c->dA, c->tB, c->sc, c->nbA, c->sy, c->sig, c->nbar2, c->twx, c->twy,
                  c->Mx, c->My, c->part, c->jpart, c->stats, c->sch, c->lam, c->trace,
                  c->alpha_sk, c->d_args, c->d_margs, c->d_ctrl, c->ref_d, c->ref_npix,
                  c->ref_sk, c->ref_poof, c->ref_pst, c->ref_out, c->ref_init, c->ref_margs};
  for (void* p : bufs)
    if (p) (void)hipFree(p);
  if (c->batch_dev) (void)hipFree(c->batch_dev);
  if (c->batch_host) (void)hipHostFree(c->batch_host);
  if (c->h_ring) (void)hipHostFree(c->h_ring);
  if (c->h_stats) (void)hipHostFree(c->h_stats);
  if (c->h_args) (void)hipHostFree(c->h_args);
  if (c->h_margs) (void)hipHostFree(c->h_margs);
  if (c->h_ctrl) (void)hipHostFree(c->h_ctrl);
  for (auto& e : c->ev_ring)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : c->prof_ev)
    if (e) (void)hipEventDestroy(e);
  if (c->chunk_exec) (void)hipGraphExecDestroy(c->chunk_exec);
  if (c->chunk_graph) (void)hipGraphDestroy(c->chunk_graph);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

wf_status alloc(void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return from_hip(e);
  }
  return WF_OK;
}

wf_status create(const wf_shape* sh, Ctx** out) {
  Ctx* c = new (std::nothrow) Ctx();
  if (!c) return WF_ENOMEM;
  c->ny = sh->ny;
  c->nx = sh->nx;
  c->prec = sh->precision;
  c->esz = c->prec == WF_F64 ? 8 : 4;
  c->nh = c->nx / 2 + 1;
  c->kpm = ((c->nh + kTCM - 1) / kTCM) * kTCM;
  (void)hipGetDevice(&c->device);
  wf_status st = WF_OK;
  for_each_buffer(c, [&](void** p, size_t bytes) {
    if (st == WF_OK) st = alloc(p, bytes);
  });
  if (st != WF_OK) {
    free_ctx(c);
    return st;
  }
  hipError_t e = hipHostMalloc((void**)&c->h_ring, kRing * sizeof(DevSched), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->h_stats, 16 * sizeof(double), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc(&c->h_args, sizeof(SweepArgs<double>), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc(&c->h_margs, sizeof(MonArgs<double>), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc(&c->h_ctrl, sizeof(CtrlArgs), hipHostMallocDefault);
  for (int i = 0; i < kRing && e == hipSuccess; ++i)
    e = hipEventCreateWithFlags(&c->ev_ring[i], hipEventDisableTiming);
  if (e != hipSuccess) {
    free_ctx(c);
    return from_hip(e);
  }
  // twiddle tables, computed in double and rounded once
  if (c->prec == WF_F64) {
    std::vector<double> tdx, tdy;
    make_table(tdx, c->nx);
    make_table(tdy, c->ny);
    e = hipMemcpy(c->twx, tdx.data(), tdx.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->twy, tdy.data(), tdy.size() * 8, hipMemcpyHostToDevice);
  } else {
    std::vector<float> fx, fy;
    make_table(fx, c->nx);
    make_table(fy, c->ny);
    e = hipMemcpy(c->twx, fx.data(), fx.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->twy, fy.data(), fy.size() * 4, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    free_ctx(c);
    return from_hip(e);
  }
  *out = c;
  return WF_OK;
}

// ----- solve ---------------------------------------------------------------

struct Chain {
  int fk = FK_NONE;
  double tauA = 0, tauB = 0, tauW = 0, cB = 0, phi = 0, tau_first = 0;
  int n_levels = 1;
  double tau_report[3] = {0, 0, 0};
  PrepSpecArgs pa{};
};

wf_status plan_chain(const Ctx* c, const wf_schedule* s, bool has_oof, bool has_st,
                     const double* pix, const double* spec, Chain* ch) {
  const double min_npix = pix[1];
  const double min_oof = spec[1];
  if (has_oof && !std::isfinite(min_oof)) return WF_EINVAL;  // every mode projected out
  const double min_nf = spec[2];  // min over modes of (P_1/f or 0) + nx P_st delta_kx0
  const double b0 = s->beta[0], b1 = s->beta[1], b2 = s->beta[2];
  const double alpha = s->floor_frac;
  PrepSpecArgs& pa = ch->pa;
  pa.ny = c->ny;
  pa.nx = c->nx;
  pa.has_oof = has_oof;
  pa.has_st = has_st;
  pa.sc_adds_nf = 0;
  pa.nbA_kind = 0;
  pa.phi_nf = 0.0;
  pa.tauA = 0.0;
  if (s->chain == WF_CHAIN_THREE) {
    ch->phi = has_st ? alpha * min_npix : 0.0;
    const double tau0 = has_oof ? b0 * min_oof : 0.0;
    const double tau1 = has_st ? b1 * ch->phi : 0.0;
    if (has_oof && !(tau0 > 0)) return WF_ENOTPD;
    if (has_st && !(tau1 > 0)) return WF_ENOTPD;
    ch->tau_report[0] = tau0;
    ch->tau_report[1] = tau1;
    if (has_oof && has_st) {
      ch->fk = FK_ARRAY_STRIPE;
      ch->tauA = tau0;
      ch->tauB = tau1;
      ch->n_levels = 3;
    } else if (has_oof) {
      ch->fk = FK_ARRAY;
      ch->tauA = tau0;
      ch->n_levels = 2;
    } else if (has_st) {
      ch->fk = FK_STRIPE;
      ch->tauA = tau1;
      ch->n_levels = 2;
    }
    ch->cB = ch->phi - tau1;
    pa.nbA_kind = has_oof ? 1 : 0;
    pa.tauA = tau0;
  } else {
    const bool any = has_oof || has_st;
    ch->phi = (has_st && !has_oof) ? alpha * min_npix : 0.0;
    pa.phi_nf = ch->phi;
    if (s->chain == WF_CHAIN_MERGED && any) {
      const double tauF = b0 * (min_nf + ch->phi);
      if (!(tauF > 0)) return WF_ENOTPD;
      ch->fk = FK_ARRAY;
      ch->tauA = tauF;
      ch->n_levels = 2;
      ch->tau_report[0] = tauF;
      pa.nbA_kind = 2;
      pa.tauA = tauF;
    } else if (s->chain == WF_CHAIN_AUGMENTED && any) {
      pa.sc_adds_nf = 1;
    }
  }
  ch->tauW = b2 * (min_npix - ch->phi);
  if (!(ch->tauW > 0)) return WF_ENOTPD;
  ch->tau_report[2] = ch->tauW;
  ch->tau_first = ch->fk == FK_NONE ? ch->tauW : ch->tauA;
  return WF_OK;
}

template <class T>
SweepArgs<T> sweep_args(Ctx* c, const wf_inputs* in, const Chain& ch) {
  SweepArgs<T> a{};
  a.B = c->B;
  a.tA = c->tA;
  a.dA = c->dA;
  a.tB = c->tB;
  a.sc = (const T*)c->sc;
  a.nbA = (const T*)c->nbA;
  a.pst = in ? (const T*)in->p_stripe : nullptr;
  a.d = in ? (const T*)in->d : nullptr;
  a.nbar2 = (const T*)c->nbar2;
  a.twx = c->twx;
  a.twy = c->twy;
  a.sch = c->sch;
  a.lam = c->lam;
  a.nx = c->nx;
  a.ny = c->ny;
  a.fk = ch.fk;
  a.tauA = ch.tauA;
  a.tauB = ch.tauB;
  a.tauW = ch.tauW;
  a.cB = ch.cB;
  a.scale = 1.0 / ((double)c->nx * (double)c->ny);
  a.jrow = c->ny / kTiles[c->tile].RW;
  a.jpart = c->jpart;
  a.sy = (const T*)c->sy;
  a.Mx = c->Mx;
  a.My = c->My;
  a.kpm = c->kpm;
  return a;
}

// joint-objective partials of one sweep: row blocks, then column blocks
int j_blocks(const Ctx* c) {
  const TileCfg& t = kTiles[c->tile];
  return c->ny / t.RW + (c->nx / 2) / t.TC;
}

// Sweeps launched with the joint-objective variants: those that can close a
// chunk (the last of a full chunk, and the last of the budget when the
// budget is not a multiple of K).  They sum J only when they do.
bool j_sweep(int k, int K, int max_sweeps) {
  return k == K - 1 || k == (max_sweeps - 1) % K;
}

template <class T>
MonArgs<T> mon_args(Ctx* c, const wf_inputs* in, const Chain& ch) {
  MonArgs<T> m{};
  m.tfirst = c->tA;
  m.sc = (const T*)c->sc;
  m.sy = (const T*)c->sy;
  m.sig = (const T*)c->sig;
  m.d = (const T*)in->d;
  m.nw_off = ch.phi + ch.tauW;  // the offset the set-up subtracted from N_pix
  m.nbar2 = (const T*)c->nbar2;
  m.Mx = c->Mx;
  m.My = c->My;
  m.twx = c->twx;
  m.twy = c->twy;
  m.sch = c->sch;
  m.lam = c->lam;
  m.part = c->part;
  m.nx = c->nx;
  m.ny = c->ny;
  m.kpm = c->kpm;
  m.tau_first = ch.tau_first;
  m.scale = 1.0 / ((double)c->nx * (double)c->ny);
  return m;
}

wf_status check_schedule(const wf_schedule* s) {
  if (s->max_sweeps < 1 || s->monitor_every < 1) return WF_EINVAL;
  if (s->field_mode != 0 && s->field_mode != 1) return WF_EINVAL;
  if (s->kind == WF_SCHED_FIXED) {
    if (!s->lambda || s->n_lambda < 1) return WF_EINVAL;
    for (int i = 0; i < s->n_lambda; ++i)
      if (!(s->lambda[i] > 0) || !std::isfinite(s->lambda[i])) return WF_EINVAL;
  } else if (s->kind == WF_SCHED_ADAPTIVE) {
    if (!(s->lambda0 >= 1.0) || !std::isfinite(s->lambda0)) return WF_EINVAL;
    if (!(s->shrink_exp > 0 && s->shrink_exp < 1)) return WF_EINVAL;
    if (!(s->plateau_rtol >= 0) || !(s->snap_eps >= 0)) return WF_EINVAL;
  } else {
    return WF_EINVAL;
  }
  if (!(s->rtol >= 0)) return WF_EINVAL;
  for (int i = 0; i < 3; ++i)
    if (!(s->beta[i] > 0 && s->beta[i] <= 1)) return WF_EINVAL;
  if (!(s->floor_frac >= 0 && s->floor_frac < 1)) return WF_EINVAL;
  if (s->chain < WF_CHAIN_THREE || s->chain > WF_CHAIN_AUGMENTED) return WF_EINVAL;
  return WF_OK;
}

// Per-map state of one solve: the chain plan, host copies of the kernel
// argument blocks, the schedule, and where its device schedule lives.
template <class T>
struct MapRun {
  Ctx* c = nullptr;
  const wf_inputs* in = nullptr;
  Chain ch;
  double pix[8] = {0}, spec[8] = {0};
  SweepArgs<T> a{};
  MonArgs<T> m{};
  CtrlArgs ctrl{};
  DevSched h{};
  std::vector<double> lam;
  int n_chunks = 0;
};

// a group of maps of one shape and chain kind: one launch per kernel
template <class T>
struct ShapeClass {
  std::vector<int> maps;
  SweepArgs<T>* argv = nullptr;  // device arrays, one entry per map
  MonArgs<T>* margv = nullptr;
  int tile = kTileDefault;
};

// Validation statistics of one map's inputs, copied to the context's pinned
// slot (stream-ordered; the caller waits).
template <class T>
hipError_t enqueue_stats(Ctx* c, const wf_inputs* in, hipStream_t st) {
  hipError_t e = launch_stats<T>((const T*)in->d, (const T*)in->n_pix, in->mask, (const T*)in->s_k,
                                 (const T*)in->p_oof, (const T*)in->p_stripe, c->ny, c->nx,
                                 c->part, kStatBlocks, c->stats, c->stats + 8, st);
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(c->h_stats, c->stats, 16 * sizeof(double), hipMemcpyDeviceToHost, st);
}

// Validation, tau_i, coefficients, schedule and zero/warm start of one map.
// dsched: where this map's device schedule lives.  stats_ready: the map's
// statistics are already in c->h_stats (a batch enqueues every map's
// statistics and waits once).
template <class T>
wf_status map_setup(Ctx* c, const wf_inputs* in, const wf_schedule* s, const void* s_init,
                    void* s_out, DevSched* dsched, MapRun<T>& r, hipStream_t st,
                    bool stats_ready = false) {
  r.c = c;
  r.in = in;
  const bool has_oof = in->p_oof != nullptr, has_st = in->p_stripe != nullptr;
  if (!stats_ready) {
    WF_TRY(enqueue_stats<T>(c, in, st));
    WF_TRY(hipStreamSynchronize(st));
  }
  std::memcpy(r.pix, c->h_stats, sizeof(r.pix));
  std::memcpy(r.spec, c->h_stats + 8, sizeof(r.spec));
  if (r.pix[0] < 1) return WF_EINVAL;                             // no observed pixel
  if (r.pix[4] > 0) return WF_ENONFINITE;                         // NaN/Inf on observed pixels
  if (r.spec[3] > 0 || r.spec[4] > 0 || r.spec[5] > 0) return WF_EINVAL;  // bad spectra
  if (r.spec[6] > 0) return WF_EINVAL;  // not even in k_y on the real columns
  if (r.pix[5] > 0) return WF_ENOTPD;                             // N_pix <= 0 observed
  wf_status ps = plan_chain(c, s, has_oof, has_st, r.pix, r.spec, &r.ch);
  if (ps != WF_OK) return ps;
  WF_TRY(launch_prep<T>((const T*)in->n_pix, in->mask, c->ny, c->nx, r.ch.phi + r.ch.tauW,
                        (T*)c->nbar2, (const T*)in->s_k, (const T*)in->p_oof,
                        (const T*)in->p_stripe, r.ch.pa, (T*)c->sc, (T*)c->nbA, (T*)c->sy,
                        (T*)c->sig, c->B, c->tA, c->dA, c->tB, st));
  // schedule: lambda per sweep and the device-side controller state
  const int K = s->monitor_every, maxs = s->max_sweeps;
  r.n_chunks = (maxs + K - 1) / K;
  if (c->no_alloc && (c->lam_cap < maxs + 1 || c->trace_cap < r.n_chunks)) return WF_ESCRATCH;
  if (c->lam_cap < maxs + 1) {
    if (c->lam) (void)hipFree(c->lam);
    c->lam = nullptr;
    c->lam_cap = 0;
    wf_status as = alloc((void**)&c->lam, (size_t)(maxs + 1) * sizeof(double));
    if (as != WF_OK) return as;
    c->lam_cap = maxs + 1;
  }
  if (c->trace_cap < r.n_chunks) {
    if (c->trace) (void)hipFree(c->trace);
    c->trace = nullptr;
    c->trace_cap = 0;
    wf_status as = alloc((void**)&c->trace, (size_t)r.n_chunks * kTraceCols * sizeof(double));
    if (as != WF_OK) return as;
    c->trace_cap = r.n_chunks;
  }
  r.lam.assign(maxs + 1, 0.0);
  for (int k = 0; k <= maxs; ++k)
    r.lam[k] = s->kind == WF_SCHED_FIXED ? s->lambda[std::min(k, s->n_lambda - 1)] : s->lambda0;
  DevSched& h = r.h;
  h = DevSched{};
  h.status = WF_NOT_CONVERGED;
  h.max_sweeps = maxs;
  h.K = K;
  h.adaptive = s->kind == WF_SCHED_ADAPTIVE;
  h.max_rec = r.n_chunks;
  h.stop_full = s->stop_full ? 1 : 0;
  h.shrink = s->shrink_exp;
  h.plateau = s->plateau_rtol;
  h.snap = s->snap_eps;
  h.rtol = s->rtol;
  h.d2 = r.pix[3];
  h.nu = r.pix[2];
  h.lam_last = r.lam[0];
  WF_TRY(hipMemcpyAsync(c->lam, r.lam.data(), r.lam.size() * sizeof(double),
                        hipMemcpyHostToDevice, st));
  WF_TRY(hipMemcpyAsync(dsched, &h, sizeof(h), hipMemcpyHostToDevice, st));
  r.a = sweep_args<T>(c, in, r.ch);
  r.a.sch = dsched;
  r.a.warm_chain = s->field_mode;
  r.m = mon_args<T>(c, in, r.ch);
  r.m.sch = dsched;
  r.m.s_out = s_out;
  r.m.out_chain = s->field_mode;
  r.ctrl = CtrlArgs{dsched, c->lam, c->part, c->ny / kRWM, c->trace, c->jpart, j_blocks(c)};
  // initial state (the single-map argument block is used for the warm start)
  if (s_init) {
    std::memcpy(c->h_args, &r.a, sizeof(r.a));
    WF_TRY(hipMemcpyAsync(c->d_args, c->h_args, sizeof(r.a), hipMemcpyHostToDevice, st));
    WF_TRY(launch_row<T>(c->tile, ROW_R2C, r.a, (const SweepArgs<T>*)c->d_args, 1, 0,
                         (const T*)s_init, nullptr, st));
    WF_TRY(launch_col<T>(c->tile, COL_INIT, r.a, (const SweepArgs<T>*)c->d_args, 1, 0, nullptr,
                         r.lam[0], st));
    WF_TRY(hipStreamSynchronize(st));
  }
  // (the zero start: the set-up's coefficient passes zeroed B and the state)
  return WF_OK;
}

// One chunk: K sweeps of every class, then the monitor of every class and
// the controller of every map.  ev (optional): 6 timing events, recorded by
// the first sweep's row and column launches of class 0 themselves (start,
// end) and around the monitor.
template <class T>
wf_status enqueue_chunk(std::vector<ShapeClass<T>>& cls, const std::vector<MapRun<T>>& runs,
                        const CtrlArgs* ctrl_argv, int nmaps, int K, hipEvent_t* ev,
                        hipStream_t st) {
  for (int k = 0; k < K; ++k) {
    for (size_t i = 0; i < cls.size(); ++i) {
      const SweepArgs<T>& a0 = runs[cls[i].maps[0]].a;
      const int n = (int)cls[i].maps.size();
      const bool timed = ev && k == 0 && i == 0;
      const bool jv = j_sweep(k, K, runs[cls[i].maps[0]].h.max_sweeps);
      WF_TRY(launch_row<T>(cls[i].tile, jv ? ROW_SWEEP_J : ROW_SWEEP, a0, cls[i].argv, n, k,
                           nullptr, nullptr, st, timed ? ev[0] : nullptr, timed ? ev[1] : nullptr));
      WF_TRY(launch_col<T>(cls[i].tile, jv ? COL_SWEEP_J : COL_SWEEP, a0, cls[i].argv, n, k,
                           nullptr, 0.0, st, timed ? ev[2] : nullptr, timed ? ev[3] : nullptr));
    }
  }
  if (ev) WF_TRY(hipEventRecord(ev[4], st));
  // the monitor's column pass ran in the chunk's last column sweep
  for (auto& cl : cls) {
    const MonArgs<T>& m0 = runs[cl.maps[0]].m;
    WF_TRY(launch_mon_row<T>(m0, cl.margv, (int)cl.maps.size(), MON_RESIDUAL, st));
  }
  WF_TRY(launch_controller(ctrl_argv, nmaps, st));
  if (ev) WF_TRY(hipEventRecord(ev[5], st));
  return WF_OK;
}

// One class's K sweeps and its monitor, on one stream (a branch of the batch
// graph: the classes of a batch are independent until the controller).
template <class T>
wf_status enqueue_class(ShapeClass<T>& cl, const std::vector<MapRun<T>>& runs, int K, hipStream_t st) {
  const SweepArgs<T>& a0 = runs[cl.maps[0]].a;
  const MonArgs<T>& m0 = runs[cl.maps[0]].m;
  const int n = (int)cl.maps.size();
  const int maxs = runs[cl.maps[0]].h.max_sweeps;
  for (int k = 0; k < K; ++k) {
    const bool jv = j_sweep(k, K, maxs);
    WF_TRY(launch_row<T>(cl.tile, jv ? ROW_SWEEP_J : ROW_SWEEP, a0, cl.argv, n, k, nullptr,
                         nullptr, st));
    WF_TRY(launch_col<T>(cl.tile, jv ? COL_SWEEP_J : COL_SWEEP, a0, cl.argv, n, k, nullptr, 0.0,
                         st));
  }
  // the monitor's column pass ran in the chunk's last column sweep
  WF_TRY(launch_mon_row<T>(m0, cl.margv, n, MON_RESIDUAL, st));
  return WF_OK;
}

void fill_report(wf_report* rep, const DevSched& fin, const Chain& ch, const double* pix) {
  std::memset(rep, 0, sizeof(*rep));
  rep->status = fin.status;
  rep->sweeps = fin.sweeps_done;
  rep->n_records = fin.n_rec;
  rep->n_levels = ch.n_levels;
  rep->lambda = fin.lam_last;
  rep->rho = fin.rho;
  rep->rho_mask = fin.rho_mask;
  rep->dd2 = fin.dd2;
  rep->d2 = pix[3];
  rep->chi2_joint = fin.J;
  rep->masked_x_norm = fin.masked_x;
  for (int i = 0; i < 3; ++i) rep->tau[i] = ch.tau_report[i];
  rep->phi = ch.phi;
}

// The chunk graph of a context for this solve: recorded on the context's
// capture stream the first time (or when the key changed), then reused.  The
// launches read everything that changes between solves from the device
// argument blocks and schedule, so one recording serves every solve with
// the same key.
template <class T>
wf_status chunk_graph(Ctx* c, std::vector<ShapeClass<T>>& cls, const std::vector<MapRun<T>>& runs,
                      int K, hipGraphExec_t* out) {
  const int key[4] = {K, (runs[0].h.max_sweeps - 1) % K, c->tile, runs[0].a.fk};
  if (c->chunk_exec && std::memcmp(key, c->chunk_key, sizeof(key)) == 0) {
    *out = c->chunk_exec;
    return WF_OK;
  }
  if (c->chunk_exec) (void)hipGraphExecDestroy(c->chunk_exec);
  if (c->chunk_graph) (void)hipGraphDestroy(c->chunk_graph);
  c->chunk_exec = nullptr;
  c->chunk_graph = nullptr;
  if (!c->cap_stream) WF_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  WF_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  const wf_status es = enqueue_chunk<T>(cls, runs, (const CtrlArgs*)c->d_ctrl, 1, K, nullptr,
                                        c->cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t ce = hipStreamEndCapture(c->cap_stream, &g);
  if (es != WF_OK) {
    if (g) (void)hipGraphDestroy(g);
    return es;
  }
  WF_TRY(ce);
  c->chunk_graph = g;
  WF_TRY(hipGraphInstantiate(&c->chunk_exec, g, nullptr, nullptr, 0));
  std::memcpy(c->chunk_key, key, sizeof(key));
  *out = c->chunk_exec;
  return WF_OK;
}

template <class T>
wf_status solve_t(Ctx* c, const wf_inputs* in, const wf_schedule* s, const void* s_init,
                  void* s_out, wf_report* rep, double* trace, hipStream_t st,
                  Chain* chain_out = nullptr) {
  std::vector<MapRun<T>> runs(1);
  MapRun<T>& r = runs[0];
  wf_status ss = map_setup<T>(c, in, s, s_init, s_out, c->sch, r, st);
  if (ss != WF_OK) return ss;
  if (chain_out) *chain_out = r.ch;
  // argument blocks for the single-map launches
  std::memcpy(c->h_args, &r.a, sizeof(r.a));
  std::memcpy(c->h_margs, &r.m, sizeof(r.m));
  std::memcpy(c->h_ctrl, &r.ctrl, sizeof(r.ctrl));
  WF_TRY(hipMemcpyAsync(c->d_args, c->h_args, sizeof(r.a), hipMemcpyHostToDevice, st));
  WF_TRY(hipMemcpyAsync(c->d_margs, c->h_margs, sizeof(r.m), hipMemcpyHostToDevice, st));
  WF_TRY(hipMemcpyAsync(c->d_ctrl, c->h_ctrl, sizeof(r.ctrl), hipMemcpyHostToDevice, st));
  std::vector<ShapeClass<T>> cls(1);
  cls[0].maps = {0};
  cls[0].argv = (SweepArgs<T>*)c->d_args;
  cls[0].margv = (MonArgs<T>*)c->d_margs;
  cls[0].tile = c->tile;

  const int K = s->monitor_every;
  const bool prof = c->profiling != 0;
  if (prof && (int)c->prof_ev.size() < kProfSlots) {
    for (int i = (int)c->prof_ev.size(); i < kProfSlots; ++i) {
      // timing-only events: no system-scope fence, which would flush caches
      // and lengthen the measured kernel
      hipEvent_t e;
      WF_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
      c->prof_ev.push_back(e);
    }
  }
  const int prof_chunks = kProfSlots / 6;
  int launched = 0;
  // without profiling (whose events are recorded by the dispatches of the
  // first sweeps) every chunk is the replayed graph
  hipGraphExec_t exec = nullptr;
  if (!prof && !c->no_alloc) {
    wf_status gs = chunk_graph<T>(c, cls, runs, K, &exec);
    if (gs != WF_OK) return gs;
  }
  for (int ci = 0; ci < r.n_chunks; ++ci) {
    if (exec) {
      WF_TRY(hipGraphLaunch(exec, st));
    } else {
      hipEvent_t* ev = (prof && ci < prof_chunks) ? &c->prof_ev[6 * ci] : nullptr;
      wf_status es = enqueue_chunk<T>(cls, runs, (const CtrlArgs*)c->d_ctrl, 1, K, ev, st);
      if (es != WF_OK) return es;
    }
    launched = ci + 1;
    if (c->no_alloc) {
      // no events: every kStaticCheck chunks the host waits for the stream
      // and reads the device schedule (plain host memory)
      if ((ci + 1) % kStaticCheck == 0 && ci + 1 < r.n_chunks) {
        WF_TRY(hipMemcpyAsync(c->h_ring, c->sch, sizeof(DevSched), hipMemcpyDeviceToHost, st));
        WF_TRY(hipStreamSynchronize(st));
        if (c->h_ring[0].done) break;
      }
      continue;
    }
    const int slot = ci % kRing;
    WF_TRY(hipMemcpyAsync(&c->h_ring[slot], c->sch, sizeof(DevSched), hipMemcpyDeviceToHost, st));
    WF_TRY(hipEventRecord(c->ev_ring[slot], st));
    if (ci >= kLag) {
      const int chk = (ci - kLag) % kRing;
      WF_TRY(hipEventSynchronize(c->ev_ring[chk]));
      if (c->h_ring[chk].done) break;
    }
  }
  WF_TRY(hipStreamSynchronize(st));
  DevSched fin;
  WF_TRY(hipMemcpy(&fin, c->sch, sizeof(fin), hipMemcpyDeviceToHost));

  // output s = S x, x = t_A / (S_chain + T_A) at the last lambda
  WF_TRY(launch_mon_col<T>(r.m, cls[0].margv, 1, MON_OUTPUT, st));
  WF_TRY(launch_mon_row<T>(r.m, cls[0].margv, 1, MON_OUTPUT, st));
  if (trace && fin.n_rec > 0)
    WF_TRY(hipMemcpyAsync(trace, c->trace, (size_t)fin.n_rec * kTraceCols * sizeof(double),
                          hipMemcpyDeviceToHost, st));
  WF_TRY(hipStreamSynchronize(st));

  if (rep) {
    fill_report(rep, fin, r.ch, r.pix);
    if (prof) {
      const int last_chunk = fin.sweeps_done > 0 ? (fin.sweeps_done - 1) / K : 0;
      const int nsamp = std::min(std::min(launched, prof_chunks), last_chunk + 1);
      for (int ci = 0; ci < nsamp; ++ci) {
        hipEvent_t* ev = &c->prof_ev[6 * ci];
        float t01 = 0, t12 = 0, t34 = 0;
        WF_TRY(hipEventElapsedTime(&t01, ev[0], ev[1]));
        WF_TRY(hipEventElapsedTime(&t12, ev[2], ev[3]));
        WF_TRY(hipEventElapsedTime(&t34, ev[4], ev[5]));
        rep->kernel_ms[0] += t01;
        rep->kernel_ms[1] += t12;
        rep->kernel_ms[2] += t34;
        rep->kernel_launches[0] += 1;
        rep->kernel_launches[1] += 1;
        rep->kernel_launches[2] += 1;
      }
    }
  }
  return (wf_status)fin.status;
}

// Batched solve: maps of equal shape and chain kind share every launch; a
// chunk of sweeps is captured once in a HIP graph and replayed.
template <class T>
wf_status solve_batch_t(Ctx** ctxs, int n, const wf_inputs* ins, const wf_schedule* s,
                        const void* const* s_init, void* const* s_out, wf_report* reps,
                        hipStream_t user_st) {
  std::vector<MapRun<T>> runs(n);
  // this call's schedules, argument blocks and controller arguments, in the
  // first context's batch workspace
  DevSched* dsch = nullptr;
  SweepArgs<T>* dargs = nullptr;
  MonArgs<T>* dmargs = nullptr;
  CtrlArgs* dctrl = nullptr;
  DevSched* hring = nullptr;
  hipStream_t cs = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev_in = nullptr, ev_ring[kRing] = {};
  std::vector<hipStream_t> bs;     // one capture branch per shape class
  std::vector<hipEvent_t> bev;     // fork event + one join event per class
  wf_status ret = WF_OK;
  auto cleanup = [&]() {
    for (auto& e : bev)
      if (e) (void)hipEventDestroy(e);
    for (auto& b : bs)
      if (b) (void)hipStreamDestroy(b);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cs) (void)hipStreamDestroy(cs);
    if (ev_in) (void)hipEventDestroy(ev_in);
    for (auto& e : ev_ring)
      if (e) (void)hipEventDestroy(e);
  };
#define BT(expr)                          \
  do {                                    \
    hipError_t e_ = (expr);               \
    if (e_ != hipSuccess) {               \
      cleanup();                          \
      return from_hip(e_);                \
    }                                     \
  } while (0)
  {
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t o1 = al((size_t)n * sizeof(DevSched));
    const size_t o2 = o1 + al((size_t)n * sizeof(SweepArgs<T>));
    const size_t o3 = o2 + al((size_t)n * sizeof(MonArgs<T>));
    const size_t need = o3 + al((size_t)n * sizeof(CtrlArgs));
    const size_t need_h = (size_t)kRing * n * sizeof(DevSched);
    Ctx* w = ctxs[0];
    if (w->batch_dev_bytes < need) {
      if (w->batch_dev) (void)hipFree(w->batch_dev);
      w->batch_dev = nullptr;
      w->batch_dev_bytes = 0;
      BT(hipMalloc(&w->batch_dev, need));
      w->batch_dev_bytes = need;
    }
    if (w->batch_host_bytes < need_h) {
      if (w->batch_host) (void)hipHostFree(w->batch_host);
      w->batch_host = nullptr;
      w->batch_host_bytes = 0;
      BT(hipHostMalloc(&w->batch_host, need_h, hipHostMallocDefault));
      w->batch_host_bytes = need_h;
    }
    char* base = (char*)w->batch_dev;
    dsch = (DevSched*)base;
    dargs = (SweepArgs<T>*)(base + o1);
    dmargs = (MonArgs<T>*)(base + o2);
    dctrl = (CtrlArgs*)(base + o3);
    hring = (DevSched*)w->batch_host;
  }
  for (int i = 0; i < n; ++i) BT(enqueue_stats<T>(ctxs[i], &ins[i], user_st));
  BT(hipStreamSynchronize(user_st));
  for (int i = 0; i < n; ++i) {
    wf_status ms = map_setup<T>(ctxs[i], &ins[i], s, s_init ? s_init[i] : nullptr, s_out[i],
                                dsch + i, runs[i], user_st, true);
    if (ms != WF_OK) {
      (void)hipStreamSynchronize(user_st);
      cleanup();
      return ms;
    }
  }
  // classes of (shape, chain kind); argument blocks laid out class by class
  std::vector<ShapeClass<T>> cls;
  std::vector<int> order;
  for (int i = 0; i < n; ++i) {
    bool placed = false;
    for (auto& cl : cls) {
      const MapRun<T>& r0 = runs[cl.maps[0]];
      if (r0.c->ny == runs[i].c->ny && r0.c->nx == runs[i].c->nx && r0.a.fk == runs[i].a.fk &&
          r0.c->tile == runs[i].c->tile) {
        cl.maps.push_back(i);
        placed = true;
        break;
      }
    }
    if (!placed) {
      ShapeClass<T> cl;
      cl.maps = {i};
      cl.tile = runs[i].c->tile;
      cls.push_back(cl);
    }
  }
  std::vector<SweepArgs<T>> ha;
  std::vector<MonArgs<T>> hm;
  std::vector<CtrlArgs> hc;
  for (auto& cl : cls) {
    cl.argv = dargs + ha.size();
    cl.margv = dmargs + hm.size();
    for (int i : cl.maps) {
      ha.push_back(runs[i].a);
      hm.push_back(runs[i].m);
    }
  }
  for (int i = 0; i < n; ++i) hc.push_back(runs[i].ctrl);
  BT(hipMemcpyAsync(dargs, ha.data(), ha.size() * sizeof(SweepArgs<T>), hipMemcpyHostToDevice, user_st));
  BT(hipMemcpyAsync(dmargs, hm.data(), hm.size() * sizeof(MonArgs<T>), hipMemcpyHostToDevice, user_st));
  BT(hipMemcpyAsync(dctrl, hc.data(), hc.size() * sizeof(CtrlArgs), hipMemcpyHostToDevice, user_st));
  // the sweeps run on a stream of this call (a captured stream cannot be the
  // legacy default stream); it starts after the set-up on the caller's stream
  BT(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  BT(hipEventCreateWithFlags(&ev_in, hipEventDisableTiming));
  for (int i = 0; i < kRing; ++i) BT(hipEventCreateWithFlags(&ev_ring[i], hipEventDisableTiming));
  BT(hipEventRecord(ev_in, user_st));
  BT(hipStreamWaitEvent(cs, ev_in, 0));
  const int K = s->monitor_every;
  int n_chunks = 0;
  for (auto& r : runs) n_chunks = std::max(n_chunks, r.n_chunks);
  // the chunk's classes run as parallel branches of the graph (small maps
  // fill the GPU beside large ones), joined before the controller
  const int nc = (int)cls.size();
  bs.assign(nc, nullptr);
  bev.assign(nc + 1, nullptr);
  for (int c = 0; c < nc; ++c) BT(hipStreamCreateWithFlags(&bs[c], hipStreamNonBlocking));
  for (int c = 0; c <= nc; ++c) BT(hipEventCreateWithFlags(&bev[c], hipEventDisableTiming));
  BT(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  wf_status es = WF_OK;
  hipError_t fe = hipEventRecord(bev[nc], cs);
  for (int c = 0; c < nc && fe == hipSuccess && es == WF_OK; ++c) {
    fe = hipStreamWaitEvent(bs[c], bev[nc], 0);
    if (fe == hipSuccess) es = enqueue_class<T>(cls[c], runs, K, bs[c]);
    if (fe == hipSuccess && es == WF_OK) fe = hipEventRecord(bev[c], bs[c]);
    if (fe == hipSuccess && es == WF_OK) fe = hipStreamWaitEvent(cs, bev[c], 0);
  }
  if (fe == hipSuccess && es == WF_OK) fe = launch_controller(dctrl, n, cs);
  if (fe != hipSuccess && es == WF_OK) es = from_hip(fe);
  hipError_t ce = hipStreamEndCapture(cs, &graph);
  if (es != WF_OK) {
    cleanup();
    return es;
  }
  BT(ce);
  BT(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  for (int ci = 0; ci < n_chunks; ++ci) {
    BT(hipGraphLaunch(exec, cs));
    const int slot = ci % kRing;
    BT(hipMemcpyAsync(hring + (size_t)slot * n, dsch, (size_t)n * sizeof(DevSched),
                      hipMemcpyDeviceToHost, cs));
    BT(hipEventRecord(ev_ring[slot], cs));
    if (ci >= kLag) {
      const int chk = (ci - kLag) % kRing;
      BT(hipEventSynchronize(ev_ring[chk]));
      bool all = true;
      for (int i = 0; i < n; ++i) all = all && hring[(size_t)chk * n + i].done;
      if (all) break;
    }
  }
  BT(hipStreamSynchronize(cs));
  std::vector<DevSched> fin(n);
  BT(hipMemcpy(fin.data(), dsch, (size_t)n * sizeof(DevSched), hipMemcpyDeviceToHost));
  for (auto& cl : cls) {
    const MonArgs<T>& m0 = runs[cl.maps[0]].m;
    BT(launch_mon_col<T>(m0, cl.margv, (int)cl.maps.size(), MON_OUTPUT, cs));
    BT(launch_mon_row<T>(m0, cl.margv, (int)cl.maps.size(), MON_OUTPUT, cs));
  }
  BT(hipStreamSynchronize(cs));
#undef BT
  int worst = WF_OK;
  for (int i = 0; i < n; ++i) {
    if (reps) fill_report(&reps[i], fin[i], runs[i].ch, runs[i].pix);
    const int sti = fin[i].status;
    if (sti < 0) worst = std::min(worst, sti);
    else if (worst >= 0) worst = std::max(worst, sti);
  }
  ret = (wf_status)worst;
  cleanup();
  return ret;
}

// ----- iterative refinement: float32 solves, float64 residual ---------------
//
// x = S^-1 s is accumulated in float64 (state layout [kx][ky], unnormalised
// like every Fourier field here) on the float64 context:
//   round 0: solve the data with float32 sweeps (from a warm start if one
//   is given); x_acc = x of that solve;
//   then, while rho > rtol: evaluate Delta d = d_rec(x_acc) - d in float64
//   and solve -Delta d (observed pixels; 0 on masked ones) with float32
//   sweeps; x_acc += x of that solve.
// The filter is linear and (I + N S^-1) is its inverse on the observed
// pixels (Section 2), so each correction removes the residual of x_acc up
// to the float32 solve's own relative accuracy.  Output s = S x_acc, or the
// chain field u = S_chain x_acc when the first schedule asks for field mode 1.
wf_status ensure(void** p, size_t bytes) {
  return *p ? WF_OK : alloc(p, bytes);
}

wf_status solve_refined(Ctx* c32, Ctx* c64, const wf_inputs* in, const wf_schedule* first,
                        const wf_schedule* corr, int max_rounds, double rtol, const void* s_init,
                        void* s_out, wf_report* rep, double* trace, hipStream_t st) {
  const size_t ny = c32->ny, nx = c32->nx, nh = c32->nh;
  const size_t npix = ny * nx, modes = ny * nh;
  wf_status e;
  if ((e = ensure(&c32->ref_d, npix * 4)) != WF_OK) return e;
  if ((e = ensure(&c32->ref_npix, npix * 4)) != WF_OK) return e;
  if ((e = ensure(&c32->ref_sk, modes * 4)) != WF_OK) return e;
  if ((e = ensure(&c32->ref_out, npix * 4)) != WF_OK) return e;
  if (s_init && (e = ensure(&c32->ref_init, npix * 4)) != WF_OK) return e;
  if (in->p_oof && (e = ensure(&c32->ref_poof, modes * 4)) != WF_OK) return e;
  if (in->p_stripe && (e = ensure(&c32->ref_pst, ny * 4)) != WF_OK) return e;
  if ((e = ensure(&c64->ref_margs, 2 * sizeof(MonArgs<double>))) != WF_OK) return e;
  // float64 side: validation and the per-mode arrays (S + N_F, S, mask sign)
  std::vector<MapRun<double>> runs(1);
  MapRun<double>& r64 = runs[0];
  wf_status ss = map_setup<double>(c64, in, first, nullptr, s_out, c64->sch, r64, st);
  if (ss != WF_OK) return ss;
  // float32 copies of the inputs
  WF_TRY(launch_to_float((const double*)in->d, (int64_t)npix, (float*)c32->ref_d, st));
  WF_TRY(launch_to_float((const double*)in->n_pix, (int64_t)npix, (float*)c32->ref_npix, st));
  WF_TRY(launch_to_float((const double*)in->s_k, (int64_t)modes, (float*)c32->ref_sk, st));
  if (in->p_oof)
    WF_TRY(launch_to_float((const double*)in->p_oof, (int64_t)modes, (float*)c32->ref_poof, st));
  if (in->p_stripe)
    WF_TRY(launch_to_float((const double*)in->p_stripe, (int64_t)ny, (float*)c32->ref_pst, st));
  if (s_init)
    WF_TRY(launch_to_float((const double*)s_init, (int64_t)npix, (float*)c32->ref_init, st));
  wf_inputs in32 = *in;
  in32.d = c32->ref_d;
  in32.n_pix = c32->ref_npix;
  in32.s_k = c32->ref_sk;
  in32.p_oof = in->p_oof ? c32->ref_poof : nullptr;
  in32.p_stripe = in->p_stripe ? c32->ref_pst : nullptr;
  // monitor passes on the float64 context, x read directly from x_acc:
  // [0] residual and the next right-hand side, [1] output s = S x
  void* xacc = c64->dA;
  MonArgs<double> mh[2];
  for (int i = 0; i < 2; ++i) {
    mh[i] = mon_args<double>(c64, in, r64.ch);
    mh[i].tfirst = xacc;
    mh[i].x_direct = 1;
    mh[i].out_chain = 0;
    mh[i].rout = (float*)c32->ref_d;
  }
  mh[1].s_out = s_out;
  mh[1].out_chain = first->field_mode;  // 1: u = S_chain x instead of s = S x
  const MonArgs<double>* dm = (const MonArgs<double>*)c64->ref_margs;
  WF_TRY(hipMemcpyAsync(c64->ref_margs, mh, sizeof(mh), hipMemcpyHostToDevice, st));
  WF_TRY(hipStreamSynchronize(st));  // mh is this frame's memory
  const double d2 = r64.pix[3], nu = r64.pix[2];
  int sweeps = 0, rounds = 0, last_status = WF_OK;
  double prof_ms[4] = {0, 0, 0, 0};  // per-kernel timing of the float32 solves
  int prof_n[4] = {0, 0, 0, 0};
  double rho = INFINITY, rho_mask = INFINITY, dd2 = 0.0;
  for (int j = 0; j <= max_rounds; ++j) {
    wf_report rj;
    Chain chj;
    const void* init = (j == 0 && s_init) ? c32->ref_init : nullptr;
    const wf_status sj = solve_t<float>(c32, &in32, j == 0 ? first : corr, init, c32->ref_out,
                                        &rj, nullptr, st, &chj);
    if (sj < 0) return sj;
    last_status = sj;
    sweeps += rj.sweeps;
    for (int i = 0; i < 4; ++i) {
      prof_ms[i] += rj.kernel_ms[i];
      prof_n[i] += rj.kernel_launches[i];
    }
    rounds = j + 1;
    WF_TRY(launch_accum_x(c32->tA, (const float*)c32->sc, rj.lambda * chj.tau_first, (int)ny,
                          (int)nx, j == 0, xacc, st));
    // float64 residual of x_acc; its negative is the next right-hand side
    WF_TRY(launch_mon_col<double>(mh[0], dm, 1, MON_REFINE, st));
    WF_TRY(launch_mon_row<double>(mh[0], dm, 1, MON_REFINE, st));
    WF_TRY(launch_pair_sum(c64->part, (int)(ny / kRWM), c64->stats, st));
    WF_TRY(hipMemcpyAsync(c64->h_stats, c64->stats, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    WF_TRY(hipStreamSynchronize(st));
    dd2 = c64->h_stats[0];
    rho = std::sqrt(dd2 / d2);
    rho_mask = nu * std::sqrt(c64->h_stats[1]) / std::sqrt(d2);
    if (!std::isfinite(dd2)) return WF_ENONFINITE;
    if (trace) {
      double* tr = trace + 4 * j;
      tr[0] = j;
      tr[1] = sweeps;
      tr[2] = rho;
      tr[3] = rho_mask;
    }
    if (rho <= rtol) break;
  }
  WF_TRY(launch_mon_col<double>(mh[1], dm + 1, 1, MON_OUTPUT, st));
  WF_TRY(launch_mon_row<double>(mh[1], dm + 1, 1, MON_OUTPUT, st));
  WF_TRY(hipStreamSynchronize(st));
  const int status = rho <= rtol ? WF_OK : WF_NOT_CONVERGED;
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    rep->status = status;
    rep->sweeps = sweeps;
    rep->n_levels = r64.ch.n_levels;
    rep->lambda = 1.0;
    rep->rho = rho;
    rep->rho_mask = rho_mask;
    rep->dd2 = dd2;
    rep->d2 = d2;
    rep->masked_x_norm = std::sqrt(c64->h_stats[1]);
    rep->refine_rounds = rounds;
    rep->n_records = rounds;
    for (int i = 0; i < 4; ++i) {
      rep->kernel_ms[i] = prof_ms[i];
      rep->kernel_launches[i] = prof_n[i];
    }
    (void)last_status;
  }
  return (wf_status)status;
}

// ----- the entry point that allocates nothing ------------------------------
//
// wf_solve_noalloc carves a context's workspace out of this array instead of
// allocating it.  Every GPU the library runs on holds its own copy for the
// life of the process; host code reaches it only through the address
// hipGetSymbolAddress returns on that device (the array's name is a host-side
// stand-in).  Calls that overlap on one GPU share it and race.
constexpr size_t kStaticBytes = size_t(32) << 20;
constexpr int kStaticMaxSweeps = 1 << 16;
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// the scratch array's device address on the current device, looked up once
wf_status scratch_on_device(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return WF_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return WF_EDEVICE;
    g_scratch_ptr[dev] = p;
  }
  *out = (unsigned char*)g_scratch_ptr[dev];
  return WF_OK;
}

constexpr size_t kCarveAlign = 256;

// Place every device buffer of c, then the schedule arrays, from base
// (nullptr: only count).  Returns the bytes used.
size_t carve_static(Ctx* c, unsigned char* base, int lam_cap, int trace_cap) {
  size_t off = 0;
  auto take = [&](void** p, size_t bytes) {
    if (base) *p = base + off;
    off = (off + bytes + kCarveAlign - 1) / kCarveAlign * kCarveAlign;
  };
  for_each_buffer(c, take);
  take((void**)&c->lam, (size_t)lam_cap * sizeof(double));
  take((void**)&c->trace, (size_t)trace_cap * kTraceCols * sizeof(double));
  if (base) {
    c->lam_cap = lam_cap;
    c->trace_cap = trace_cap;
  }
  return off;
}

template <class T>
wf_status solve_noalloc_t(const wf_shape* sh, const wf_inputs* in, const wf_schedule* sch,
                          const void* s_init, void* s_out, wf_report* rep, double* trace,
                          hipStream_t st) {
  Ctx c;
  c.ny = sh->ny;
  c.nx = sh->nx;
  c.prec = sh->precision;
  c.esz = sizeof(T);
  c.nh = c.nx / 2 + 1;
  c.kpm = ((c.nh + kTCM - 1) / kTCM) * kTCM;
  c.no_alloc = true;
  const int lam_cap = sch->max_sweeps + 1;
  const int trace_cap = (sch->max_sweeps + sch->monitor_every - 1) / sch->monitor_every;
  if (carve_static(&c, nullptr, lam_cap, trace_cap) > kStaticBytes) return WF_ESCRATCH;
  WF_TRY(hipGetDevice(&c.device));
  unsigned char* base = nullptr;
  wf_status ss = scratch_on_device(c.device, &base);
  if (ss != WF_OK) return ss;
  carve_static(&c, base, lam_cap, trace_cap);
  // host staging in plain memory of this call
  DevSched h_ring[kRing];
  double h_stats[16];
  alignas(16) unsigned char h_args[sizeof(SweepArgs<double>)];
  alignas(16) unsigned char h_margs[sizeof(MonArgs<double>)];
  alignas(16) unsigned char h_ctrl[sizeof(CtrlArgs)];
  c.h_ring = h_ring;
  c.h_stats = h_stats;
  c.h_args = h_args;
  c.h_margs = h_margs;
  c.h_ctrl = h_ctrl;
  // twiddle tables (the largest supported length is 4096), computed in
  // double and rounded once, as for a context
  static thread_local T tw[2][2 * 4096];
  for (int a = 0; a < 2; ++a) {
    const int n = a == 0 ? c.nx : c.ny;
    for (int j = 0; j < n; ++j) {
      const double ang = 2.0 * M_PI * (double)j / (double)n;
      tw[a][2 * j] = (T)std::cos(ang);
      tw[a][2 * j + 1] = (T)(-std::sin(ang));
    }
  }
  WF_TRY(hipMemcpyAsync(c.twx, tw[0], (size_t)c.nx * 2 * sizeof(T), hipMemcpyHostToDevice, st));
  WF_TRY(hipMemcpyAsync(c.twy, tw[1], (size_t)c.ny * 2 * sizeof(T), hipMemcpyHostToDevice, st));
  const wf_status r = solve_t<T>(&c, in, sch, s_init, s_out, rep, trace, st);
  (void)hipStreamSynchronize(st);  // the staging above is this call's memory
  return r;
}

template <class T>
wf_status fft_t(Ctx* c, const void* src, void* dst, bool forward, hipStream_t st) {
  Chain ch;
  SweepArgs<T> a = sweep_args<T>(c, nullptr, ch);
  std::memcpy(c->h_args, &a, sizeof(a));
  WF_TRY(hipMemcpyAsync(c->d_args, c->h_args, sizeof(a), hipMemcpyHostToDevice, st));
  const SweepArgs<T>* argv = (const SweepArgs<T>*)c->d_args;
  if (forward) {
    WF_TRY(launch_row<T>(kTileDefault, ROW_R2C, a, argv, 1, 0, (const T*)src, nullptr, st));
    WF_TRY(launch_col<T>(kTileDefault, COL_FWD_OUT, a, argv, 1, 0, dst, 0.0, st));
  } else {
    WF_TRY(launch_col<T>(kTileDefault, COL_INV_IN, a, argv, 1, 0, const_cast<void*>(src), 0.0, st));
    WF_TRY(launch_row<T>(kTileDefault, ROW_C2R, a, argv, 1, 0, nullptr, (T*)dst, st));
  }
  WF_TRY(hipStreamSynchronize(st));
  return WF_OK;
}

}  // namespace

extern "C" {

wf_status wf_ctx_create(const wf_shape* shape, void** out) {
  if (!shape || !out) return WF_EINVAL;
  *out = nullptr;
  if (shape->precision != WF_F32 && shape->precision != WF_F64) return WF_EINVAL;
  if (!supported(shape->ny, shape->nx, shape->precision)) return WF_EUNSUPPORTED;
  Ctx* c = nullptr;
  wf_status s = create(shape, &c);
  if (s == WF_OK) *out = c;
  return s;
}

void wf_ctx_destroy(void* ctx) {
  if (ctx) free_ctx((Ctx*)ctx);
}

void wf_schedule_default(wf_schedule* s) {
  if (!s) return;
  std::memset(s, 0, sizeof(*s));
  s->kind = WF_SCHED_ADAPTIVE;
  s->lambda0 = 1.0e4;
  s->shrink_exp = 0.7;
  s->plateau_rtol = 1.0e-2;
  s->snap_eps = 1.0e-3;
  s->rtol = 1.0e-6;
  s->max_sweeps = 20000;
  s->monitor_every = 16;
  s->beta[0] = 0.9;
  s->beta[1] = 0.9;
  s->beta[2] = 1.0;
  s->floor_frac = 0.5;
  s->chain = WF_CHAIN_THREE;
  s->stop_full = 0;
  s->field_mode = 0;
}

wf_status wf_solve(void* ctx, const wf_inputs* in, const wf_schedule* sch, const void* s_init,
                   void* s_out, wf_report* rep, double* trace, hipStream_t stream) {
  Ctx* c = (Ctx*)ctx;
  if (!c || !in || !sch || !s_out || !in->d || !in->s_k || !in->n_pix) return WF_EINVAL;
  wf_status v = check_schedule(sch);
  if (v != WF_OK) return v;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != c->device) return WF_EINVAL;
  if (c->prec == WF_F64) return solve_t<double>(c, in, sch, s_init, s_out, rep, trace, stream);
  return solve_t<float>(c, in, sch, s_init, s_out, rep, trace, stream);
}

wf_status wf_solve_noalloc(const wf_shape* shape, const wf_inputs* in, const wf_schedule* sch,
                           const void* s_init, void* s_out, wf_report* rep, double* trace,
                           hipStream_t stream) {
  if (!shape || !in || !sch || !s_out || !in->d || !in->s_k || !in->n_pix) return WF_EINVAL;
  if (shape->precision != WF_F32 && shape->precision != WF_F64) return WF_EINVAL;
  if (!supported(shape->ny, shape->nx, shape->precision)) return WF_EUNSUPPORTED;
  wf_status v = check_schedule(sch);
  if (v != WF_OK) return v;
  if (sch->max_sweeps > kStaticMaxSweeps) return WF_ESCRATCH;
  if (shape->precision == WF_F64)
    return solve_noalloc_t<double>(shape, in, sch, s_init, s_out, rep, trace, stream);
  return solve_noalloc_t<float>(shape, in, sch, s_init, s_out, rep, trace, stream);
}

size_t wf_noalloc_scratch_bytes(void) { return kStaticBytes; }

wf_status wf_solve_refined(void* ctx32, void* ctx64, const wf_inputs* in,
                           const wf_schedule* first, const wf_schedule* corr, int32_t max_rounds,
                           double rtol, const void* s_init, void* s_out, wf_report* rep,
                           double* trace, hipStream_t stream) {
  Ctx* c32 = (Ctx*)ctx32;
  Ctx* c64 = (Ctx*)ctx64;
  if (!c32 || !c64 || !in || !first || !corr || !s_out || !in->d || !in->s_k || !in->n_pix)
    return WF_EINVAL;
  if (c32->prec != WF_F32 || c64->prec != WF_F64) return WF_EINVAL;
  if (c32->ny != c64->ny || c32->nx != c64->nx || c32->device != c64->device) return WF_EINVAL;
  if (max_rounds < 0 || !(rtol >= 0)) return WF_EINVAL;
  wf_status v = check_schedule(first);
  if (v == WF_OK) v = check_schedule(corr);
  if (v != WF_OK) return v;
  if (corr->field_mode != 0) return WF_EINVAL;  // first: 0 or 1 (check_schedule)
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != c32->device) return WF_EINVAL;
  return solve_refined(c32, c64, in, first, corr, max_rounds, rtol, s_init, s_out, rep, trace,
                       stream);
}

wf_status wf_solve_batch(void* const* ctxs, int32_t n, const wf_inputs* inputs,
                         const wf_schedule* sch, const void* const* s_init, void* const* s_out,
                         wf_report* reps, hipStream_t stream) {
  if (!ctxs || !inputs || !sch || !s_out || n < 1 || n > WF_BATCH_MAX) return WF_EINVAL;
  wf_status v = check_schedule(sch);
  if (v != WF_OK) return v;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return WF_EDEVICE;
  std::vector<Ctx*> cs(n);
  for (int i = 0; i < n; ++i) {
    Ctx* c = (Ctx*)ctxs[i];
    const wf_inputs& in = inputs[i];
    if (!c || !s_out[i] || !in.d || !in.s_k || !in.n_pix) return WF_EINVAL;
    if (c->device != dev || c->prec != ((Ctx*)ctxs[0])->prec) return WF_EINVAL;
    for (int j = 0; j < i; ++j)
      if (cs[j] == c) return WF_EINVAL;  // each map needs its own context
    cs[i] = c;
  }
  if (cs[0]->prec == WF_F64)
    return solve_batch_t<double>(cs.data(), n, inputs, sch, s_init, s_out, reps, stream);
  return solve_batch_t<float>(cs.data(), n, inputs, sch, s_init, s_out, reps, stream);
}

wf_status wf_inverse_noise_weight(void* ctx, const wf_inputs* in, double alpha,
                                  const wf_schedule* sch, const void* s_init, void* out,
                                  wf_report* rep, double* trace, hipStream_t stream) {
  Ctx* c = (Ctx*)ctx;
  if (!c || !in || !sch || !out || !in->d || !in->n_pix) return WF_EINVAL;
  if (!(alpha > 0) || !std::isfinite(alpha)) return WF_EINVAL;
  if (sch->field_mode != 0) return WF_EINVAL;
  const int64_t nmodes = (int64_t)c->ny * c->nh;
  if (!c->alpha_sk) {
    wf_status as = alloc(&c->alpha_sk, (size_t)nmodes * c->esz);
    if (as != WF_OK) return as;
  }
  wf_inputs w = *in;
  w.s_k = c->alpha_sk;
  const int64_t npix = (int64_t)c->ny * c->nx;
  wf_status st;
  if (c->prec == WF_F64) {
    WF_TRY(launch_fill<double>((double*)c->alpha_sk, nmodes, alpha, stream));
    st = wf_solve(ctx, &w, sch, s_init, out, rep, trace, stream);
    if (st >= 0) WF_TRY(launch_scale<double>((double*)out, npix, 1.0 / alpha, stream));
  } else {
    WF_TRY(launch_fill<float>((float*)c->alpha_sk, nmodes, alpha, stream));
    st = wf_solve(ctx, &w, sch, s_init, out, rep, trace, stream);
    if (st >= 0) WF_TRY(launch_scale<float>((float*)out, npix, 1.0 / alpha, stream));
  }
  if (st >= 0) WF_TRY(hipStreamSynchronize(stream));
  return st;
}

wf_status wf_rfft2(void* ctx, const void* x, void* X, hipStream_t stream) {
  Ctx* c = (Ctx*)ctx;
  if (!c || !x || !X) return WF_EINVAL;
  if (c->prec == WF_F64) return fft_t<double>(c, x, X, true, stream);
  return fft_t<float>(c, x, X, true, stream);
}

wf_status wf_irfft2(void* ctx, const void* X, void* x, hipStream_t stream) {
  Ctx* c = (Ctx*)ctx;
  if (!c || !x || !X) return WF_EINVAL;
  if (c->prec == WF_F64) return fft_t<double>(c, X, x, false, stream);
  return fft_t<float>(c, X, x, false, stream);
}

wf_status wf_ctx_set_profiling(void* ctx, int32_t enable) {
  Ctx* c = (Ctx*)ctx;
  if (!c) return WF_EINVAL;
  c->profiling = enable ? 1 : 0;
  return WF_OK;
}

int32_t wf_supported(int32_t ny, int32_t nx, int32_t precision) { return supported(ny, nx, precision); }

int32_t wf_tile_count(void) { return kNumTiles; }

wf_status wf_ctx_set_tile(void* ctx, int32_t tile) {
  Ctx* c = (Ctx*)ctx;
  if (!c || tile < 0 || tile >= kNumTiles) return WF_EINVAL;
  // the default tiling is built for every size; the others for float32
  // maps whose sides are both tuned lengths
  const bool built = tile == kTileDefault || (c->prec == WF_F32 && tuned_length(c->nx) &&
                                               tuned_length(c->ny));
  if (!built) return WF_EUNSUPPORTED;
  const TileCfg& t = kTiles[tile];
  if (c->ny % t.TR != 0 || (c->nx / 2) % t.TC != 0) return WF_EUNSUPPORTED;
  c->tile = tile;
  return WF_OK;
}

namespace {
// the autotuners' probe: a cooling ramp from 1e3 over the probe's first half
// (the sweep kernels do not depend on lambda's value; this keeps the probe a
// valid solve), no stop before the budget, monitor every 16 sweeps
wf_schedule probe_schedule(int sweeps, std::vector<double>& lam) {
  lam.resize(sweeps);
  for (int k = 0; k < sweeps; ++k)
    lam[k] = k < sweeps / 2 ? std::pow(1.0e3, 1.0 - 2.0 * k / sweeps) : 1.0;
  wf_schedule sch;
  wf_schedule_default(&sch);
  sch.kind = WF_SCHED_FIXED;
  sch.lambda = lam.data();
  sch.n_lambda = sweeps;
  sch.rtol = 0.0;
  sch.max_sweeps = sweeps;
  sch.monitor_every = std::min(16, sweeps);
  return sch;
}
}  // namespace

wf_status wf_autotune(void* ctx, const wf_inputs* in, int32_t sweeps, void* scratch,
                      double* ms, int32_t* best, hipStream_t stream) {
  Ctx* c = (Ctx*)ctx;
  if (!c || !in || !scratch || sweeps < 1 || sweeps > 4096) return WF_EINVAL;
  if (!in->d || !in->s_k || !in->n_pix) return WF_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != c->device) return WF_EINVAL;
  std::vector<double> lam;
  const wf_schedule sch = probe_schedule(sweeps, lam);
  const int old_tile = c->tile, old_prof = c->profiling;
  c->profiling = 0;
  double best_ms = INFINITY;
  int best_tile = -1;
  wf_status err = WF_OK;
  for (int tile = 0; tile < kNumTiles; ++tile) {
    if (ms) ms[tile] = -1.0;
    if (wf_ctx_set_tile(ctx, tile) != WF_OK) continue;
    wf_status st = wf_solve(ctx, in, &sch, nullptr, scratch, nullptr, nullptr, stream);  // warm-up
    const auto t0 = std::chrono::steady_clock::now();
    for (int rep = 0; rep < 2 && st >= 0; ++rep)
      st = wf_solve(ctx, in, &sch, nullptr, scratch, nullptr, nullptr, stream);
    const double t =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() /
        2.0;
    if (st < 0) {
      err = st;
      break;
    }
    if (ms) ms[tile] = t;
    if (t < best_ms) {
      best_ms = t;
      best_tile = tile;
    }
  }
  c->profiling = old_prof;
  c->tile = (err == WF_OK && best_tile >= 0) ? best_tile : old_tile;
  if (best) *best = c->tile;
  return err;
}

wf_status wf_autotune_batch(void* const* ctxs, int32_t n, const wf_inputs* inputs,
                            int32_t sweeps, void* const* s_out, double* ms, int32_t* best,
                            hipStream_t stream) {
  if (!ctxs || !inputs || !s_out || n < 1 || n > WF_BATCH_MAX || sweeps < 1 || sweeps > 4096)
    return WF_EINVAL;
  for (int i = 0; i < n; ++i)
    if (!ctxs[i]) return WF_EINVAL;
  std::vector<double> lam;
  const wf_schedule sch = probe_schedule(sweeps, lam);
  std::vector<char> grouped(n, 0);
  wf_status err = WF_OK;
  for (int i = 0; i < n && err == WF_OK; ++i) {
    if (grouped[i]) continue;
    // the maps of map i's shape, tuned together
    const Ctx* ci = (const Ctx*)ctxs[i];
    std::vector<int> g;
    for (int j = i; j < n; ++j) {
      const Ctx* cj = (const Ctx*)ctxs[j];
      if (!grouped[j] && cj->ny == ci->ny && cj->nx == ci->nx) {
        g.push_back(j);
        grouped[j] = 1;
      }
    }
    const int m = (int)g.size();
    std::vector<void*> gc(m), go(m);
    std::vector<wf_inputs> gi(m);
    std::vector<int> old(m);
    for (int k = 0; k < m; ++k) {
      gc[k] = ctxs[g[k]];
      go[k] = s_out[g[k]];
      gi[k] = inputs[g[k]];
      old[k] = ((Ctx*)gc[k])->tile;
    }
    double tms[kNumTiles];
    double best_ms = INFINITY;
    int best_tile = -1;
    for (int tile = 0; tile < kNumTiles; ++tile) {
      tms[tile] = -1.0;
      bool built = true;
      for (void* c : gc) built = built && wf_ctx_set_tile(c, tile) == WF_OK;
      if (!built) continue;
      // warm-up (records the batch's graph), then two timed batched solves
      wf_status st = wf_solve_batch(gc.data(), m, gi.data(), &sch, nullptr, go.data(), nullptr,
                                    stream);
      const auto t0 = std::chrono::steady_clock::now();
      for (int rep = 0; rep < 2 && st >= 0; ++rep)
        st = wf_solve_batch(gc.data(), m, gi.data(), &sch, nullptr, go.data(), nullptr, stream);
      const double t = std::chrono::duration<double, std::milli>(
                           std::chrono::steady_clock::now() - t0).count() / 2.0;
      if (st < 0) {
        err = st;
        break;
      }
      tms[tile] = t;
      if (t < best_ms) {
        best_ms = t;
        best_tile = tile;
      }
    }
    for (int k = 0; k < m; ++k) {
      Ctx* c = (Ctx*)gc[k];
      c->tile = (err == WF_OK && best_tile >= 0) ? best_tile : old[k];
      if (ms)
        for (int tile = 0; tile < kNumTiles; ++tile) ms[(size_t)g[k] * kNumTiles + tile] = tms[tile];
    }
  }
  if (best)
    for (int i = 0; i < n; ++i) best[i] = ((Ctx*)ctxs[i])->tile;
  return err;
}

int32_t wf_ctx_get_tile(void* ctx) {
  Ctx* c = (Ctx*)ctx;
  return c ? c->tile : -1;
}

const char* wf_strerror(int32_t s) {
  switch (s) {
    case WF_OK: return "ok";
    case WF_NOT_CONVERGED: return "sweep budget exhausted before the residual target";
    case WF_EINVAL: return "invalid argument";
    case WF_ENOTPD: return "a messenger covariance tau_i is not positive (empty noise term)";
    case WF_ENONFINITE: return "non-finite value in the inputs or the iteration";
    case WF_EDEVICE: return "HIP runtime error";
    case WF_ENOMEM: return "device allocation failed";
    case WF_EUNSUPPORTED: return "map size or precision not supported";
    case WF_ESCRATCH: return "workspace larger than the static scratch of wf_solve_noalloc";
    default: return "unknown status";
  }
}

}  // extern "C"
