// Host side of the C-ABI: context, device memory, preparation of the sorted
// system and lists, PME tables, and the solver driver.
//
// Solver (paper: Tinker-HP's preconditioned conjugate gradient, Eq. 18):
// block-Jacobi PCG with z = alpha r.  One iteration enqueues
//   direction p = z + beta p -> spread and FFT convolution of p (auxiliary
//   stream) beside the real-space matvec -> PME gather (with p.Tp)
//   -> update (x, r, z, r.z, z.z) -> device-side test of
//   DEBYE * sqrt(z.z / N_pol) <= tol.
// When the test passes the residual is recomputed from scratch in FP64; if
// that true residual is still above the tolerance it replaces the recurrence
// residual and the same sequence continues.  In mixed mode (FP32 pair and
// PME arithmetic inside the iteration) one such replacement is also made
// early, which keeps the FP32 drift below the tolerance.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <map>
#include <string>
#include <vector>

#include "../../include/sibfa_pol.h"
#include "common.h"
#include "kernels.h"
#include "nlist.h"

using namespace sibfa;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct sibfa_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  // library-owned second stream: the reciprocal half of each PME step
  // (spreading + FFT convolution) runs on it concurrently with the
  // real-space kernel on `stream`; ev_fork / ev_join order the two
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipEvent_t ev_bricks = nullptr;   // the PME brick lists are built (auxiliary stream)
  sibfa_alloc_fn af = nullptr;
  sibfa_free_fn ff = nullptr;
  void* user = nullptr;
  std::string err;

  sibfa_params prm{};
  int n = 0, npol = 0, periodic = 0;
  double box[3] = {0, 0, 0};
  bool have_sys = false, have_mult = false, have_pol = false, has_thole = false;
  bool dirty_sort = true, dirty_mult = true, dirty_pol = true, dirty_lists = true;
  // molecule ids and polarizabilities validated since they were last set:
  // later re-sorts report position errors at the list build's readback and
  // skip their own
  bool ids_ok = false, pol_ok = false;
  bool e0_valid = false, mu_valid = false, mu_have = false;
  double e_real = 0, e_rec = 0, e_self = 0;
  sibfa_stats stats{};

  std::vector<DevBuf> bufs;   // every allocation, freed on destroy / resize

  // caller-order copies
  double *xyz_c = nullptr, *q_c = nullptr, *dip_c = nullptr, *quad_c = nullptr;
  double *alpha_c = nullptr, *thole_c = nullptr, *mu_c = nullptr;
  int* mol_c = nullptr;
  // cells
  int nc[3] = {1, 1, 1}, ncell = 1;
  int *cell_of = nullptr, *cell_count = nullptr, *cell_start = nullptr, *cursor = nullptr;
  int4* cellmax = nullptr;   // per-cell list count maxima
  int *perm = nullptr, *inv_perm = nullptr, *mol_count = nullptr, *mol_s = nullptr;
  int* scan_tmp = nullptr;
  // records
  double4 *sp = nullptr, *sd = nullptr, *sth = nullptr;
  double2* sth2 = nullptr;
  float4 *sp32 = nullptr, *sd32 = nullptr, *sth32 = nullptr;
  float2* sth232 = nullptr;
  double* sa = nullptr;
  int *is_pol = nullptr, *pol_scan = nullptr, *polidx = nullptr, *polsite = nullptr;
  // polarizable-site arrays (sized n: npol <= n)
  double4* pp = nullptr;
  float4* pp32 = nullptr;
  double *pa = nullptr, *alpha_s = nullptr, *ainv_s = nullptr;
  // lists
  int cap[4] = {0, 0, 0, 0};
  int* nb[4] = {nullptr, nullptr, nullptr, nullptr};
  int* ncnt[4] = {nullptr, nullptr, nullptr, nullptr};
  int* ncnear = nullptr;   // near entries of the all list
  // all-list split radius squared: every polarizable pair beyond it has a
  // Thole exponent x = a r^3 s_i s_j >= 50 (no damping)
  double rsplit2 = 0.0;
  // z.z decay per iteration seen in the first run of the last solve: sizes
  // the first batch of the next one (-1: none yet)
  double rate_hint = -1.0;
  DevBuf nbbuf[4];
  // [0..3] list maxima, [4] binning errors (bits 2, 8), [5] list errors
  // (bit 1), [6] finiteness flag, [7] polarizability errors (bit 4),
  // [8..11] solver stop flag, [12..13] z.z of the last test (double),
  // [16..31] eight slot totals (doubles), [32..35] polarizability extents
  // (doubles)
  int* dints = nullptr;
  // solver vectors (pol order)
  double4 *E0 = nullptr, *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr,
          *t = nullptr;
  float4 *p32 = nullptr, *x32 = nullptr;
  // site vectors
  double4 *mu_s = nullptr, *Freal = nullptr;
  float4* mu_s32 = nullptr;
  // PME
  PmeView pm{};
  std::vector<DevBuf> pmebufs;
  int nbricks = 0;
  int *bcount = nullptr, *bcursor = nullptr, *brick_of = nullptr, *bscan_tmp = nullptr;
  int *bstart_pol = nullptr, *border_pol = nullptr, *bstart_all = nullptr, *border_all = nullptr;
  // cached pol-list pair coefficients (FP64, or FP32 in mixed mode)
  DevBuf coefbuf, icoefbuf, coef32buf;   // FP64 always; FP32 in mixed mode
  bool coef_valid = false;
  // the potential grid holds (or, on the auxiliary stream, will hold) the
  // permanent multipoles' potential, started while the lists were built
  bool phi_e0 = false;
  // second direction buffer (the spread kernel reads one and writes the other)
  double4* p2 = nullptr;
  // molecular block preconditioner (sized n when params.precond asks for it)
  PcView pcv{};
  float4* p2_32 = nullptr;
  // reductions
  Reduce red{};
  double* h_pinned = nullptr;   // small host staging (list totals)
  double* h_part = nullptr;     // host copies of reduction partials [S_COUNT][max_blocks]
  int* h_ints = nullptr;
  unsigned long long* dsums = nullptr;   // list entry totals
  long long pair_totals[4] = {0, 0, 0, 0};
  bool totals_valid = false;
  // virial requests: forces scratch when the caller passes no forces, and
  // the device and host copies of the virial slot totals (allocated on the
  // first request)
  double* fvir = nullptr;
  double* vir_tot = nullptr;
  double* h_vir = nullptr;
  // predictor of the warm-start guess: order (<= 1: the last dipoles) and a
  // ring of the last kPredMax dipole sets (caller order; in bufs)
  int pred_order = 0;
  double* hist = nullptr;
  int hist_head = 0, hist_count = 0;
  // molecular dynamics: masses, virtual sites, bonds, velocities and
  // accelerations (mdbufs, replaced by every sibfa_md_init)
  bool md_on = false;
  std::vector<DevBuf> mdbufs;
  MdArgs md{};
  double* md_force = nullptr;
  // truncated-CG forces: work vectors (tcgbufs, sized for the last order)
  std::vector<DevBuf> tcgbufs;
  int tcg_cap = -1;
  size_t tcg_np = 0;
  // reduced charge transfer: inputs, lookup tables and work buffers
  // (ctbufs, replaced by every sibfa_set_charge_transfer)
  bool ct_on = false;
  std::vector<DevBuf> ctbufs;
  CtArgs ct{};
  double4 *ct_spw = nullptr, *ct_zero4 = nullptr;
  double2* ct_zero2 = nullptr;
  // local frames: device copies of the frames and local quantities, the
  // frame groups and site references, and the force-path buffers (all in
  // framebufs, replaced by every sibfa_set_local_frames)
  bool have_frames = false, dirty_rot = false, rot_alpha = false;
  int ngroups = 0;
  std::vector<DevBuf> framebufs;
  int* frames_d = nullptr;
  double *dloc = nullptr, *qloc = nullptr, *aloc = nullptr;
  int *gframe = nullptr, *gstart = nullptr, *gsites = nullptr, *sstart = nullptr, *sref = nullptr;
  double *Cs = nullptr, *Fg = nullptr, *GS = nullptr;
  double4* FS = nullptr;
  // profiling: HIP events on the context stream around each phase
  bool prof = false;
  unsigned prof_mask = ~0u;   // phases timed while profiling
  std::vector<hipEvent_t> evpool;
  size_t evused = 0;
  // tag: solver iteration of a batched launch (-1 outside batches); launches
  // enqueued after the device stop flag was raised return at once and are
  // counted in the phase time but not in its launch count
  struct Mark { int phase; hipEvent_t a, b; int tag; bool work; };
  std::vector<Mark> marks;
  int cur_tag = -1;
  static_assert(SIBFA_PH_COUNT <= 16, "phases fit the profile record");
  double prof_ms[16] = {0};
  int prof_calls[16] = {0};
};

namespace {

sibfa_status fail(sibfa_ctx c, sibfa_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

sibfa_status hip_fail(sibfa_ctx c, hipError_t e, const char* where) {
  return fail(c, SIBFA_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call)                                   \
  do {                                                  \
    hipError_t _e = (call);                             \
    if (_e != hipSuccess) return hip_fail(c, _e, #call); \
  } while (0)

void* dev_alloc(sibfa_ctx c, size_t bytes) {
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) & ~(size_t)255;
  void* ptr = nullptr;
  if (c->af) ptr = c->af(bytes, c->user);
  else if (hipMalloc(&ptr, bytes) != hipSuccess) ptr = nullptr;
  return ptr;
}

void dev_free(sibfa_ctx c, void* ptr) {
  if (!ptr) return;
  if (c->ff) {
    // a caching allocator hands the block out again at once, ordered only
    // against its own stream: let the work of both library streams that
    // may still read it finish first (frees happen on resizes and
    // teardown, not in the evaluation path)
    (void)hipStreamSynchronize(c->stream);
    if (c->aux && c->aux != c->stream) (void)hipStreamSynchronize(c->aux);
    c->ff(ptr, c->user);
  } else {
    (void)hipFree(ptr);
  }
}

template <typename T>
bool alloc_into(sibfa_ctx c, std::vector<DevBuf>& list, T*& out, size_t count) {
  void* ptr = dev_alloc(c, count * sizeof(T));
  if (!ptr) return false;
  list.push_back({ptr, count * sizeof(T)});
  out = static_cast<T*>(ptr);
  return true;
}

void free_list(sibfa_ctx c, std::vector<DevBuf>& list) {
  for (auto& b : list) dev_free(c, b.p);
  list.clear();
}

bool factor_radices(int K, int* rad, int* nrad) {
  int m = K, k = 0;
  while (m % 4 == 0 && k < 16) { rad[k++] = 4; m /= 4; }
  while (m % 2 == 0 && k < 16) { rad[k++] = 2; m /= 2; }
  while (m % 3 == 0 && k < 16) { rad[k++] = 3; m /= 3; }
  while (m % 5 == 0 && k < 16) { rad[k++] = 5; m /= 5; }
  *nrad = k;
  return m == 1;
}

// Cardinal B-spline values M_p(t) at the integers t = 0..p-1 (recursion
// M_n(u) = (u M_{n-1}(u) + (n-u) M_{n-1}(u-1))/(n-1), M_1 = 1 on [0,1)).
std::vector<long double> bspline_at_integers(int p) {
  std::vector<long double> lev(p, 0.0L), nxt(p, 0.0L);
  lev[0] = 1.0L;
  for (int n = 2; n <= p; ++n) {
    for (int t = 0; t < p; ++t) {
      const long double u = t;
      const long double a = (t <= n - 2) ? lev[t] : 0.0L;
      const long double b = (t >= 1 && t - 1 <= n - 2) ? lev[t - 1] : 0.0L;
      nxt[t] = (u * a + (n - u) * b) / (n - 1);
    }
    lev = nxt;
  }
  return lev;
}

// |sum_{k=0}^{p-2} M_p(k+1) exp(2 pi i m k / K)|^2, a vanishing value (odd
// order, Nyquist index of an even grid) replaced by the mean of its
// neighbours.
std::vector<double> bspline_moduli(int K, int p) {
  const std::vector<long double> M = bspline_at_integers(p);
  std::vector<double> mod(K);
  const long double twopi = 6.283185307179586476925286766559L;
  for (int m = 0; m < K; ++m) {
    long double re = 0, im = 0;
    for (int k = 0; k <= p - 2; ++k) {
      const long double ang = twopi * m * k / K;
      re += M[k + 1] * cosl(ang);
      im += M[k + 1] * sinl(ang);
    }
    mod[m] = (double)(re * re + im * im);
  }
  for (int m = 0; m < K; ++m)
    if (mod[m] < 1e-7) mod[m] = 0.5 * (mod[(m - 1 + K) % K] + mod[(m + 1) % K]);
  return mod;
}

SysView make_view(sibfa_ctx c) {
  SysView s{};
  s.n = c->n;
  s.npol = c->npol;
  s.periodic = c->periodic;
  for (int a = 0; a < 3; ++a) {
    s.box[a] = c->periodic ? c->box[a] : 1.0;
    s.ibox[a] = c->periodic ? 1.0 / c->box[a] : 1.0;
  }
  s.cutoff2 = c->prm.cutoff * c->prm.cutoff;
  s.beta = c->prm.ewald_beta;
  s.uniform_thole = c->has_thole ? 0 : 1;
  s.thole_a = c->prm.thole_a;
  s.sp = c->sp; s.sd = c->sd; s.sth = c->sth; s.sth2 = c->sth2; s.sa = c->sa;
  s.polidx = c->polidx;
  s.sp32 = c->sp32; s.sd32 = c->sd32; s.sth32 = c->sth32; s.sth232 = c->sth232;
  s.polsite = c->polsite; s.pp = c->pp; s.pp32 = c->pp32; s.pa = c->pa;
  s.alpha = c->alpha_s; s.ainv = c->ainv_s;
  s.nb_all = c->nb[0]; s.nc_all = c->ncnt[0]; s.cap_all = c->cap[0];
  s.nc_near = c->ncnear;
  s.nb_in = c->nb[1]; s.nc_in = c->ncnt[1]; s.cap_in = c->cap[1];
  s.nb_pol = c->nb[2]; s.nc_pol = c->ncnt[2]; s.cap_pol = c->cap[2];
  s.nb_ipol = c->nb[3]; s.nc_ipol = c->ncnt[3]; s.cap_ipol = c->cap[3];
  s.cpol = static_cast<const double2*>(c->coefbuf.p);
  s.cpol32 = static_cast<const float2*>(c->coef32buf.p);
  s.cipol = static_cast<const double2*>(c->icoefbuf.p);
  return s;
}

FrameArgs make_frames(sibfa_ctx c) {
  FrameArgs f{};
  f.n = c->n;
  f.ngroups = c->ngroups;
  f.periodic = c->periodic;
  for (int a = 0; a < 3; ++a) {
    f.box[a] = c->periodic ? c->box[a] : 1.0;
    f.ibox[a] = c->periodic ? 1.0 / c->box[a] : 1.0;
  }
  f.xyz = c->xyz_c;
  f.frames = c->frames_d;
  f.dloc = c->dloc; f.qloc = c->qloc; f.aloc = c->rot_alpha ? c->aloc : nullptr;
  f.dip = c->dip_c; f.quad = c->quad_c; f.alpha = c->alpha_c;
  f.inv_perm = c->inv_perm;
  f.FS = c->FS; f.GS = c->GS; f.mu_s = c->mu_s;
  f.C = c->Cs;
  f.gframe = c->gframe; f.gstart = c->gstart; f.gsites = c->gsites;
  f.Fg = c->Fg;
  f.sstart = c->sstart; f.sref = c->sref;
  return f;
}

bool mixed(sibfa_ctx c) { return c->prm.precision == SIBFA_MIXED; }

sibfa_status check_params(sibfa_ctx c, const sibfa_params* p, const double* box) {
  if (!p) return fail(c, SIBFA_E_ARG, "params is NULL");
  if (!(p->tol_debye > 0) || p->max_iter < 1)
    return fail(c, SIBFA_E_ARG, "tol_debye must be > 0 and max_iter >= 1");
  if (!(p->thole_a > 0) || !std::isfinite(p->thole_a))
    return fail(c, SIBFA_E_ARG, "thole_a must be positive");
  if (p->precond != SIBFA_PRECOND_DIAG && p->precond != SIBFA_PRECOND_MOLBLOCK)
    return fail(c, SIBFA_E_ARG, "precond must be SIBFA_PRECOND_DIAG or SIBFA_PRECOND_MOLBLOCK");
  if (p->precision != SIBFA_FP64 && p->precision != SIBFA_MIXED)
    return fail(c, SIBFA_E_ARG, "unknown precision");
  if (box) {
    for (int a = 0; a < 3; ++a)
      if (!(box[a] > 0) || !std::isfinite(box[a])) return fail(c, SIBFA_E_ARG, "box edges must be positive");
    if (!(p->cutoff > 0)) return fail(c, SIBFA_E_ARG, "cutoff must be positive");
    if (!(p->cutoff < 0.5 * std::min(box[0], std::min(box[1], box[2]))))
      return fail(c, SIBFA_E_ARG, "cutoff must be below half the smallest box edge");
    if (!(p->ewald_beta > 0)) return fail(c, SIBFA_E_ARG, "ewald_beta must be positive");
    if (p->order < 4 || p->order > 6) return fail(c, SIBFA_E_ARG, "order must be 4, 5 or 6");
    for (int a = 0; a < 3; ++a) {
      int rad[16], nr;
      if (p->grid[a] < 2 * p->order || p->grid[a] % 2 != 0 || !factor_radices(p->grid[a], rad, &nr))
        return fail(c, SIBFA_E_ARG, "grid sizes must be even, >= 2*order, with factors 2, 3, 5 only");
      if (p->grid[a] > 1024) return fail(c, SIBFA_E_ARG, "grid sizes above 1024 are not supported");
    }
  }
  return SIBFA_OK;
}

void release_system(sibfa_ctx c) {
  c->rate_hint = -1.0;
  free_list(c, c->bufs);
  c->fvir = nullptr;      // both lived in bufs
  c->vir_tot = nullptr;
  free_list(c, c->mdbufs);
  c->md_on = false;
  free_list(c, c->ctbufs);
  c->ct_on = false;
  free_list(c, c->tcgbufs);
  c->tcg_cap = -1;
  c->hist = nullptr;       // lived in bufs
  c->hist_head = c->hist_count = 0;
  free_list(c, c->framebufs);
  c->have_frames = c->dirty_rot = c->rot_alpha = false;
  c->ngroups = 0;
  free_list(c, c->pmebufs);
  for (int k = 0; k < 4; ++k) {
    dev_free(c, c->nbbuf[k].p);
    c->nbbuf[k] = DevBuf{};
    c->nb[k] = nullptr;
    c->cap[k] = 0;
  }
  dev_free(c, c->coefbuf.p);
  c->coefbuf = DevBuf{};
  dev_free(c, c->icoefbuf.p);
  c->icoefbuf = DevBuf{};
  dev_free(c, c->coef32buf.p);
  c->coef32buf = DevBuf{};
  if (c->h_part) {
    (void)hipHostFree(c->h_part);
    c->h_part = nullptr;
  }
  c->coef_valid = false;
  c->have_sys = c->have_mult = c->have_pol = false;
  c->e0_valid = c->mu_valid = c->mu_have = false;
}

sibfa_status sync_read(sibfa_ctx c) {
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  return SIBFA_OK;
}

// Totals of up to 8 slots: summed on the device (one block per slot, fixed
// order) and read back with one copy.
sibfa_status read_totals(sibfa_ctx c, std::initializer_list<int> slots, double* out) {
  SlotList sl{};
  for (int s : slots) {
    sl.slot[sl.n] = s;
    sl.nparts[sl.n] = c->red.nparts[s];
    ++sl.n;
  }
  double* dtot = reinterpret_cast<double*>(c->dints + 16);
  launch_slot_totals(c->red, sl, dtot, c->stream);
  HIP_TRY(hipMemcpyAsync(c->h_pinned + 48, dtot, sl.n * sizeof(double), hipMemcpyDeviceToHost,
                         c->stream));
  sibfa_status st = sync_read(c);
  if (st != SIBFA_OK) return st;
  for (int k = 0; k < sl.n; ++k) out[k] = c->h_pinned[48 + k];
  return SIBFA_OK;
}

// ------------------------------------------------------------ profiling
hipEvent_t next_event(sibfa_ctx c) {
  if (c->evused < c->evpool.size()) return c->evpool[c->evused++];
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  c->evpool.push_back(e);
  c->evused++;
  return e;
}

void fold_marks(sibfa_ctx c) {
  if (c->marks.empty()) return;
  (void)hipStreamSynchronize(c->stream);
  (void)hipStreamSynchronize(c->aux);
  for (auto& m : c->marks) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, m.a, m.b) == hipSuccess) {
      c->prof_ms[m.phase] += ms;
      c->prof_calls[m.phase] += m.work ? 1 : 0;
    }
  }
  c->marks.clear();
  c->evused = 0;
}

// Brackets the launches of one phase with events when profiling is on.
// attach: the phase is a single kernel launched with start() and stop() as
// its own dispatch events (hipExtLaunchKernelGGL), which time the kernel
// itself rather than marker packets around it; the launcher must record
// both.
struct Phase {
  sibfa_ctx c;
  int ph;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  bool attach;
  Phase(sibfa_ctx cc, int p, hipStream_t s = nullptr, bool att = false)
      : c(cc), ph(p), st(s ? s : cc->stream), attach(att) {
    if (p >= 0 && c->prof && ((c->prof_mask >> p) & 1u)) {
      if (c->marks.size() > 4096 && c->cur_tag < 0) fold_marks(c);
      a = next_event(c);
      if (a && attach) {
        b = next_event(c);
        if (!b) a = nullptr;
      } else if (a) {
        (void)hipEventRecord(a, st);
      }
    }
  }
  hipEvent_t start() const { return attach ? a : nullptr; }
  hipEvent_t stop() const { return attach ? b : nullptr; }
  ~Phase() {
    if (c->prof && a) {
      if (!attach) {
        b = next_event(c);
        if (b) (void)hipEventRecord(b, st);
      }
      if (b) c->marks.push_back({ph, a, b, c->cur_tag, true});
    }
  }
};

void conv(sibfa_ctx c, bool mix, hipStream_t st, int erec_slot = S_EREC, bool virial = false) {
  PmeView pm = c->pm;
  pm.erec_slot = erec_slot;
  launch_convolution(pm, c->red, mix, st, virial);
  c->phi_e0 = false;
}

// The auxiliary stream starts after everything enqueued so far on the main
// stream; the main stream continues once the auxiliary work is done.
// With the overlap switched off (environment SIBFA_PME_OVERLAP=0) the
// auxiliary stream is the main stream and both are no-ops.
void fork(sibfa_ctx c) {
  if (c->aux == c->stream) return;
  (void)hipEventRecord(c->ev_fork, c->stream);
  (void)hipStreamWaitEvent(c->aux, c->ev_fork, 0);
}
void join(sibfa_ctx c) {
  if (c->aux == c->stream) return;
  (void)hipEventRecord(c->ev_join, c->aux);
  (void)hipStreamWaitEvent(c->stream, c->ev_join, 0);
}

// ------------------------------------------------------------ preparation
// Errors of the last binning (h_ints[4] holds the device word).
sibfa_status binning_errors(sibfa_ctx c) {
  if (c->h_ints[4] & 2) return fail(c, SIBFA_E_ARG, "molecule ids must lie in [0, n_sites)");
  if (c->h_ints[4] & 8)
    return fail(c, SIBFA_E_ARG, "xyz contains NaN or Inf, or (periodic) a coordinate beyond "
                                "1e6 box edges");
  return SIBFA_OK;
}

sibfa_status alloc_lists(sibfa_ctx c, const int want[4]) {
  for (int k = 0; k < 4; ++k) {
    const int rows = (k < 2) ? c->n : std::max(c->npol, 1);
    // the row count of lists 2 and 3 follows the number of polarizable
    // sites, which a change of polarizabilities may raise: check the bytes
    if (c->nb[k] && c->cap[k] >= want[k] &&
        c->nbbuf[k].bytes >= (size_t)rows * c->cap[k] * sizeof(int))
      continue;
    dev_free(c, c->nbbuf[k].p);
    const size_t bytes = (size_t)rows * want[k] * sizeof(int);
    void* ptr = dev_alloc(c, bytes);
    if (!ptr) { c->nbbuf[k] = DevBuf{}; c->nb[k] = nullptr; c->cap[k] = 0;
                return fail(c, SIBFA_E_NOMEM, "neighbour list allocation failed"); }
    c->nbbuf[k] = {ptr, bytes};
    c->nb[k] = static_cast<int*>(ptr);
    c->cap[k] = want[k];
  }
  const size_t cbytes = (size_t)std::max(c->npol, 1) * c->cap[2] * sizeof(double2);
  if (c->coefbuf.bytes < cbytes) {
    dev_free(c, c->coefbuf.p);
    void* ptr = dev_alloc(c, cbytes);
    if (!ptr) { c->coefbuf = DevBuf{}; return fail(c, SIBFA_E_NOMEM, "pair coefficient allocation failed"); }
    c->coefbuf = {ptr, cbytes};
  }
  if (c->prm.precision == SIBFA_MIXED) {
    const size_t fbytes = (size_t)std::max(c->npol, 1) * c->cap[2] * sizeof(float2);
    if (c->coef32buf.bytes < fbytes) {
      dev_free(c, c->coef32buf.p);
      void* ptr = dev_alloc(c, fbytes);
      if (!ptr) { c->coef32buf = DevBuf{}; return fail(c, SIBFA_E_NOMEM, "pair coefficient allocation failed"); }
      c->coef32buf = {ptr, fbytes};
    }
  }
  const size_t ibytes = (size_t)std::max(c->npol, 1) * c->cap[3] * sizeof(double2);
  if (c->icoefbuf.bytes < ibytes) {
    dev_free(c, c->icoefbuf.p);
    void* ptr = dev_alloc(c, ibytes);
    if (!ptr) { c->icoefbuf = DevBuf{}; return fail(c, SIBFA_E_NOMEM, "pair coefficient allocation failed"); }
    c->icoefbuf = {ptr, ibytes};
  }
  c->coef_valid = false;
  return SIBFA_OK;
}

// beside: enqueued once, right after the first list launch (work for the
// auxiliary stream that the host should not make the list build wait for).
template <class Beside>
sibfa_status build_lists(sibfa_ctx c, Beside beside) {
  int want[4];
  if (c->periodic) {
    const double V = c->box[0] * c->box[1] * c->box[2];
    const double sph = 4.0 / 3.0 * kPi * std::pow(c->prm.cutoff, 3);
    const double e_all = c->n / V * sph, e_pol = c->npol / V * sph;
    want[0] = std::min(c->n, (int)(1.3 * e_all) + 64);
    want[2] = std::min(std::max(c->npol, 1), (int)(1.3 * e_pol) + 64);
  } else {
    want[0] = std::max(c->n, 1);
    want[2] = std::max(c->npol, 1);
  }
  want[1] = std::max(c->cap[1], 8);
  want[3] = std::max(c->cap[3], 8);
  for (int attempt = 0; attempt < 3; ++attempt) {
    for (int k = 0; k < 4; ++k) want[k] = std::max(want[k], c->cap[k]);
    sibfa_status st = alloc_lists(c, want);
    if (st != SIBFA_OK) return st;
    launch_fill_ints({{c->dints + 5, 1}}, 0, c->stream);
    NlistArgs a{};
    a.periodic = c->periodic;
    for (int d = 0; d < 3; ++d) {
      a.nc[d] = c->nc[d];
      a.box[d] = c->periodic ? c->box[d] : 1.0;
      a.ibox[d] = c->periodic ? 1.0 / c->box[d] : 1.0;
    }
    a.cutoff2 = c->periodic ? c->prm.cutoff * c->prm.cutoff : INFINITY;
    a.cell_start = c->cell_start;
    a.sp = c->sp;
    a.mol_s = c->mol_s;
    a.polidx = c->polidx;
    a.mol_count = c->mol_count;
    a.nb_all = c->nb[0]; a.nc_all = c->ncnt[0]; a.cap_all = c->cap[0];
    a.nc_near = c->ncnear;
    a.rsplit2 = c->rsplit2;
    a.nb_in = c->nb[1]; a.nc_in = c->ncnt[1]; a.cap_in = c->cap[1];
    a.nb_pol = c->nb[2]; a.nc_pol = c->ncnt[2]; a.cap_pol = c->cap[2];
    a.nb_ipol = c->nb[3]; a.nc_ipol = c->ncnt[3]; a.cap_ipol = c->cap[3];
    a.cellmax = c->cellmax;
    a.err = c->dints + 5;
    {
      Phase ph(c, SIBFA_PH_LISTS);
      launch_nlist(a, c->ncell, c->stream);
      launch_cellmax_reduce(c->cellmax, c->ncell, c->dints, c->stream);
    }
    if (attempt == 0) beside();
    HIP_TRY(hipMemcpyAsync(c->h_ints, c->dints, 8 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    sibfa_status s2 = sync_read(c);
    if (s2 != SIBFA_OK) return s2;
    if ((s2 = binning_errors(c)) != SIBFA_OK) return s2;
    if (c->h_ints[5] & 1)
      return fail(c, SIBFA_E_ARG,
                  "the sites of a molecule must lie within the cutoff of each other");
    bool over = false;
    for (int k = 0; k < 4; ++k)
      if (c->h_ints[k] > c->cap[k]) { over = true; want[k] = c->h_ints[k] + 16; }
    c->stats.max_neighbors = c->h_ints[0];
    if (!over) {
      c->totals_valid = false;   // list entry totals: summed when asked for
      return SIBFA_OK;
    }
  }
  return fail(c, SIBFA_E_NOMEM, "neighbour lists kept overflowing");
}

sibfa_status prepare(sibfa_ctx c) {
  if (!c->have_sys) return fail(c, SIBFA_E_STATE, "sibfa_set_system has not been called");
  if (!c->have_mult) return fail(c, SIBFA_E_STATE, "sibfa_set_multipoles has not been called");
  if (!c->have_pol) return fail(c, SIBFA_E_STATE, "sibfa_set_polarizabilities has not been called");
  hipStream_t s = c->stream;
  RecArgs ra{};
  ra.n = c->n;
  ra.periodic = c->periodic;
  for (int a = 0; a < 3; ++a) {
    ra.box[a] = c->periodic ? c->box[a] : 1.0;
    ra.ibox[a] = c->periodic ? 1.0 / c->box[a] : 1.0;
  }
  ra.perm = c->perm;
  ra.xyz = c->xyz_c; ra.mol = c->mol_c; ra.q = c->q_c; ra.dip = c->dip_c; ra.quad = c->quad_c;
  ra.alpha = c->alpha_c; ra.thole = c->has_thole ? c->thole_c : nullptr;
  ra.thole_default = c->prm.thole_a;
  ra.sp = c->sp; ra.sd = c->sd; ra.sth = c->sth; ra.sth2 = c->sth2;
  ra.sp32 = c->sp32; ra.sd32 = c->sd32; ra.sth32 = c->sth32; ra.sth232 = c->sth232;
  ra.sa = c->sa; ra.mol_s = c->mol_s; ra.inv_perm = c->inv_perm; ra.is_pol = c->is_pol;
  ra.pol_scan = c->pol_scan; ra.polidx = c->polidx; ra.polsite = c->polsite;
  ra.pp = c->pp; ra.pp32 = c->pp32; ra.pa = c->pa; ra.alpha_s = c->alpha_s; ra.ainv_s = c->ainv_s;
  ra.err = c->dints + 7;
  // local frames: global d, Theta (alpha) at the current positions, then
  // the records are rebuilt from them as after new multipoles
  if (c->have_frames && c->dirty_rot) {
    launch_rotate(make_frames(c), s);
    c->dirty_rot = false;
    c->dirty_mult = true;
    if (c->rot_alpha) c->dirty_pol = true;
  }
  // work still queued on the auxiliary stream by an earlier call that
  // failed reads the records rewritten below
  if (c->dirty_sort || c->dirty_mult || c->dirty_pol || c->dirty_lists) join(c);

  // a re-sort rewrites all per-site records in one pass
  const bool resort = c->dirty_sort;
  if (c->dirty_sort) {
    launch_fill_ints({{c->cell_count, (size_t)c->ncell + 1}, {c->cursor, (size_t)c->ncell},
                      {c->mol_count, (size_t)c->n}, {c->dints + 4, 1}}, 0, s);
    BinArgs b{};
    b.n = c->n;
    b.periodic = c->periodic;
    for (int a = 0; a < 3; ++a) {
      b.nc[a] = c->nc[a];
      b.box[a] = ra.box[a];
      b.ibox[a] = ra.ibox[a];
    }
    b.xyz = c->xyz_c; b.mol = c->mol_c; b.cell_of = c->cell_of; b.cell_count = c->cell_count;
    b.mol_count = c->mol_count; b.err = c->dints + 4;
    {
      Phase ph(c, SIBFA_PH_LISTS);
      launch_bin(b, s);
      launch_exclusive_scan(c->cell_count, c->cell_start, c->ncell + 1, c->scan_tmp, s);
      launch_scatter(c->cell_of, c->cell_start, c->cursor, c->perm, c->n, s);
      launch_sort_cells(c->cell_start, c->ncell, c->perm, s);
      launch_rec_all(ra, s);
    }
    if (!c->ids_ok) {
      HIP_TRY(hipMemcpyAsync(c->h_ints + 4, c->dints + 4, sizeof(int), hipMemcpyDeviceToHost, s));
      sibfa_status st = sync_read(c);
      if (st != SIBFA_OK) return st;
      if ((st = binning_errors(c)) != SIBFA_OK) return st;
      c->ids_ok = true;
    }
    c->dirty_sort = false;
    c->dirty_mult = c->dirty_pol = c->dirty_lists = true;
    c->e0_valid = false;
  }
  if (c->dirty_mult) {
    if (!resort) launch_rec_mult(ra, s);
    c->dirty_mult = false;
    c->e0_valid = false;
  }
  if (c->dirty_pol) {
    launch_fill_int(c->dints + 7, 0, 1, s);
    if (!resort) launch_rec_pol(ra, s);
    launch_exclusive_scan(c->is_pol, c->pol_scan, c->n + 1, c->scan_tmp, s);
    launch_rec_polsites(ra, s);
    // a re-sort permutes the same polarizabilities: count, definiteness
    // and extents are unchanged
    if (!c->pol_ok) {
      double* dext = reinterpret_cast<double*>(c->dints + 32);
      launch_pol_extents(ra, dext, s);
      HIP_TRY(hipMemcpyAsync(c->h_ints, c->pol_scan + c->n, sizeof(int), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemcpyAsync(c->h_ints + 7, c->dints + 7, sizeof(int), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemcpyAsync(c->h_pinned + 56, dext, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
      sibfa_status st = sync_read(c);
      if (st != SIBFA_OK) return st;
      if (c->h_ints[7] & 4)
        return fail(c, SIBFA_E_ARG, "every nonzero polarizability must be positive definite");
      c->npol = c->h_ints[0];
      // x = a r^3 s_i s_j with s = abar^-1/2 is at least
      // a_min r^3 / abar_max, so x >= 50 beyond r^3 = 50 abar_max / a_min
      const double amax = c->h_pinned[56], tmin = c->h_pinned[57];
      if (c->npol == 0 || !(amax > 0.0)) c->rsplit2 = 0.0;
      else if (!(tmin > 0.0)) c->rsplit2 = INFINITY;
      else {
        const double rs = 1.001 * std::cbrt(50.0 * amax / tmin);
        c->rsplit2 = rs * rs;
      }
      c->pol_ok = true;
    }
    c->stats.n_polarizable = c->npol;
    c->dirty_pol = false;
    c->dirty_lists = true;
    c->e0_valid = false;
  }
  if (c->dirty_lists) {
    // PME brick lists and the reciprocal potential of the permanent
    // multipoles need the sorted records but not the neighbour lists: they
    // run on the auxiliary stream beside the list build, forked here but
    // enqueued after the list launch, so that the GPU starts the lists
    // while the host is still enqueueing them.  The main stream waits for
    // the brick lists after the list kernels (its dipole spreading and
    // force PME read them); the potential is joined by its consumer.
    // (FP64 in both modes: it runs beside the list build, and the
    // reciprocal energy is a large term of E_elec, which is a small sum)
    const bool two = c->aux != c->stream;
    if (c->periodic && two) (void)hipEventRecord(c->ev_fork, c->stream);
    auto beside_lists = [c, two]() {
      if (!c->periodic) return;
      hipStream_t a = c->aux;
      if (two) (void)hipStreamWaitEvent(a, c->ev_fork, 0);
      {
        Phase ph(c, SIBFA_PH_LISTS, a);
        SysView sv = make_view(c);
        for (int pol = 0; pol < 2; ++pol) {
          int* start = pol ? c->bstart_pol : c->bstart_all;
          int* order = pol ? c->border_pol : c->border_all;
          const int cnt = pol ? c->npol : c->n;
          launch_fill_ints({{c->bcount, (size_t)c->nbricks + 1}, {c->bcursor, (size_t)c->nbricks}},
                           0, a);
          launch_brick_bin(sv, c->pm, pol, c->brick_of, c->bcount, a);
          launch_exclusive_scan(c->bcount, start, c->nbricks + 1, c->bscan_tmp, a);
          if (cnt > 0) {
            launch_scatter(c->brick_of, start, c->bcursor, order, cnt, a);
            // increasing site index within each brick: reproducible sums
            launch_sort_cells(start, c->nbricks, order, a);
          }
        }
      }
      if (two) {
        (void)hipEventRecord(c->ev_bricks, a);
        (void)hipStreamWaitEvent(c->stream, c->ev_bricks, 0);
      }
      Phase ph(c, SIBFA_PH_FIELD_RECIP, a);
      launch_spread_mult(make_view(c), c->pm, nullptr, false, a);
      conv(c, false, a, S_EREC0);
      c->phi_e0 = true;
    };
    sibfa_status st = build_lists(c, beside_lists);
    if (st != SIBFA_OK) return st;
    c->dirty_lists = false;
    c->e0_valid = false;
  }
  return SIBFA_OK;
}

// ------------------------------------------------------------ compute steps

// t = T v (v in pol order, double + float copy)
// The pair coefficients of the polarizable list, computed once in FP64
// (and rounded to the FP32 table in mixed mode), on stream st.
void enqueue_coef(sibfa_ctx c, hipStream_t st) {
  Phase ph(c, SIBFA_PH_PAIRCOEF, st);
  SysView s = make_view(c);
  launch_pol_coef(s, static_cast<double2*>(c->coefbuf.p),
                  mixed(c) ? static_cast<float2*>(c->coef32buf.p) : nullptr,
                  static_cast<double2*>(c->icoefbuf.p), st);
  if (c->prm.precond == SIBFA_PRECOND_MOLBLOCK) launch_pc_build(s, c->pcv, st);
  c->coef_valid = true;
}

sibfa_status ensure_coef(sibfa_ctx c) {
  if (c->coef_valid || c->npol == 0) return SIBFA_OK;
  enqueue_coef(c, c->stream);
  return SIBFA_OK;
}

// t = T v, each part timed as its own phase when timed (else untimed).
void matvec_parts(sibfa_ctx c, double4* v, float4* v32, double4* out, int dot_slot, bool mix,
                  bool timed) {
  SysView s = make_view(c);
  auto P = [timed](int ph) { return timed ? ph : -1; };
  if (c->periodic) {
    // as in the solver loop: reciprocal chain on the main stream, the
    // real-space part beside it
    fork(c);
    {
      Phase ph2(c, P(SIBFA_PH_MATVEC), c->aux, true);
      launch_matvec_real(s, c->red, v, v32, out, dot_slot, mix, c->aux,
                         c->aux != c->stream ? c->ev_join : nullptr, ph2.start(), ph2.stop());
    }
    {
      Phase ph(c, P(SIBFA_PH_SPREAD));
      launch_spread_dip(s, c->pm, v, mix, c->stream);
    }
    {
      Phase ph(c, P(SIBFA_PH_FFT));
      conv(c, mix, c->stream);
    }
    if (c->aux != c->stream) (void)hipStreamWaitEvent(c->stream, c->ev_join, 0);
  } else {
    Phase ph2(c, P(SIBFA_PH_MATVEC), c->stream, true);
    launch_matvec_real(s, c->red, v, v32, out, dot_slot, mix, c->stream, nullptr, ph2.start(),
                       ph2.stop());
  }
  Phase ph3(c, P(SIBFA_PH_MATVEC_RECIP));
  launch_matvec_recip(s, c->pm, c->red, v, out, dot_slot, mix, c->stream);
}

// t = T v.  mix: FP32 pair/PME arithmetic (cached FP32 coefficients);
// otherwise FP64 (cached FP64 coefficients, kept in both modes).  Callers
// run ensure_coef first.  An FP64 product in a mixed-precision context is
// timed whole, as a phase of its own, so that the per-kernel phases hold
// the launches of the context's own precision only.
void matvec(sibfa_ctx c, double4* v, float4* v32, double4* out, int dot_slot, bool mix) {
  if (!mix && mixed(c)) {
    Phase ph(c, SIBFA_PH_MATVEC_FP64);
    matvec_parts(c, v, v32, out, dot_slot, false, false);
    return;
  }
  matvec_parts(c, v, v32, out, dot_slot, mix, true);
}

sibfa_status compute_E0(sibfa_ctx c) {
  SysView s = make_view(c);
  const bool mix = mixed(c);
  // auxiliary stream: the reciprocal permanent potential (unless already
  // started beside the list build) and the polarizable-pair coefficients,
  // both beside the real-space field on the main stream
  bool forked = false;
  if (c->periodic && !c->phi_e0) {
    fork(c);
    forked = true;
    Phase ph(c, SIBFA_PH_FIELD_RECIP, c->aux);
    launch_spread_mult(s, c->pm, nullptr, false, c->aux);
    conv(c, false, c->aux, S_EREC0);
  }
  if (!c->coef_valid && c->npol > 0) {
    if (!forked) fork(c);
    forked = true;
    enqueue_coef(c, c->aux);
  }
  {
    Phase ph(c, SIBFA_PH_FIELD_REAL);
    launch_perm(s, c->red, c->E0, mix, c->stream);
  }
  join(c);
  c->phi_e0 = false;
  if (c->periodic) {
    Phase ph(c, SIBFA_PH_FIELD_RECIP);
    launch_gather_field(s, c->pm, c->E0, false, c->stream);
  }
  // the energy partials stay in their slots (nothing else writes them)
  // and are read with the polarization energy
  c->e0_valid = true;
  return SIBFA_OK;
}

double rms_debye(sibfa_ctx c, double zz) {
  return c->npol > 0 ? kDebye * std::sqrt(zz / c->npol) : 0.0;
}

// The newest dipoles (mu_c) join the predictor's history.
void push_history(sibfa_ctx c, hipStream_t st) {
  if (c->pred_order < 2) return;
  const size_t len = 3 * (size_t)c->n;
  if (!c->hist && !alloc_into(c, c->bufs, c->hist, (size_t)kPredMax * len)) {
    c->pred_order = 0;   // no memory for the history: plain warm starts
    return;
  }
  (void)hipMemcpyAsync(c->hist + (size_t)c->hist_head * len, c->mu_c, len * sizeof(double),
                       hipMemcpyDeviceToDevice, st);
  c->hist_head = (c->hist_head + 1) % kPredMax;
  c->hist_count = std::min(c->hist_count + 1, kPredMax);
}

// Warm-start guess into x (and x32): the kept dipoles, or with a predictor
// of order k and at least two history entries, the value at the next step
// of the polynomial of degree k' - 1 through the k' = min(k, entries)
// newest ones (equally spaced): coefficients (-1)^(j+1) C(k', j), j = 1..k'
// from the newest back.
void warm_guess(sibfa_ctx c, const SysView& s, hipStream_t st) {
  const int k = std::min(c->pred_order, c->hist_count);
  if (k < 2) {
    launch_caller_to_pol(s, c->perm, c->mu_c, c->x, c->x32, st);
    return;
  }
  PredArgs pa{};
  pa.k = k;
  double binom = 1.0;   // C(k, j)
  for (int j = 1; j <= k; ++j) {
    binom = binom * (k - j + 1) / j;
    pa.slot[j - 1] = (c->hist_head - j + 2 * kPredMax) % kPredMax;
    pa.coef[j - 1] = (j % 2 == 1 ? 1.0 : -1.0) * binom;
  }
  launch_predict(s, c->perm, c->hist, 3 * (size_t)c->n, pa, c->x, c->x32, st);
}

sibfa_status solve(sibfa_ctx c, bool warm) {
  SysView s = make_view(c);
  hipStream_t st = c->stream;
  const bool mix = mixed(c);
  if (c->npol == 0) {
    c->stats.iterations = 0;
    c->stats.restarts = 0;
    c->stats.true_rms_debye = 0.0;
    c->mu_valid = c->mu_have = true;
    launch_fill_double(c->mu_c, 0.0, 3 * (size_t)c->n, st);
    return SIBFA_OK;
  }
  ensure_coef(c);
  const bool blk = c->prm.precond == SIBFA_PRECOND_MOLBLOCK;
  if (warm && c->mu_have) warm_guess(c, s, st);
  else if (blk) launch_pc_apply(s, c->pcv, c->E0, c->x, st);
  else launch_precond(s, c->E0, c->x, st);
  launch_copy4(c->x, c->x, c->x32, c->npol, st);
  const double tol = c->prm.tol_debye;
  const double zz_stop = (tol / kDebye) * (tol / kDebye) * c->npol;
  // Mixed precision: the FP32 matvec makes the recurrence residual drift
  // from E - T x by about the FP32 rounding of T p per iteration.  The
  // residual is replaced by the FP64 true residual once, when the recurrence
  // has fallen by kReplace in z.z, and the sequence goes on with the same
  // directions; the drift accumulated after that point is proportional to
  // the (by then small) residual.  Each later stop is confirmed the same
  // way, also in FP64, and the sequence continues if the true residual is
  // still above the tolerance.
  constexpr double kReplace = 1e-8;
  int it = 0, restarts = 0;
  int kk = 0;            // iterations of the running sequence (slot parity)
  bool fresh = true;     // no sequence yet: the first true residual sets p = z
  bool read_res = true;  // read the new true residual back (not after the
                         // early replacement, which is far from converged)
  double zz_replace = -1.0;
  double rho_true = 0.0;
  // Batch sizing: z.z of the last update read back with the stop flag and
  // its decay per iteration, to size the next batch so that it ends about
  // where the run will stop (fewer launches that return at once, fewer
  // host round trips).
  // The first batch of a solve uses the decay rate of the previous solve
  // (positions move little between evaluations), so that it usually ends
  // where the first run stops instead of after a default four iterations.
  double zz_last = -1.0, rate = c->rate_hint;
  bool first_run = true;
  sibfa_status result = SIBFA_OK;
  int* flag = c->dints + 8;                                    // [0..3]
  double* zz_dev = reinterpret_cast<double*>(c->dints + 12);  // after flag
  // z.z of a cold mixed start's first residual, left on the device: the
  // stop tests scale the replacement factor by it there, and the host reads
  // it with the first batch's flag (one host round trip fewer)
  double* zz0_dev = reinterpret_cast<double*>(c->dints + 36);
  const double* zz_ref = nullptr;
  for (;;) {
    // residual from scratch: FP64 operator, except the very first residual
    // of a cold start in mixed mode (FP32 operator; the early replacement
    // below removes its rounding)
    const bool fp32_res = fresh && mix && !(warm && c->mu_have);
    matvec(c, c->x, c->x32, c->t, -1, fp32_res);
    if (blk)
      launch_pc_init_residual(s, c->pcv, c->red, c->E0, c->t, c->r, c->z,
                              fresh ? c->p : nullptr, fresh ? c->p32 : nullptr,
                              fresh ? S_RZ0 : S_RZ0 + (kk & 1), st);
    else if (fresh)
      launch_init_residual(s, c->red, c->E0, c->t, c->r, c->z, c->p, c->p32, S_RZ0, st);
    else
      launch_init_residual(s, c->red, c->E0, c->t, c->r, c->z, nullptr, nullptr,
                           S_RZ0 + (kk & 1), st);
    if (read_res && fp32_res) {
      // far from the tolerance (FP32 operator, cold start): no read back
      SlotList sl{};
      sl.n = 1;
      sl.slot[0] = S_ZZ;
      sl.nparts[0] = c->red.nparts[S_ZZ];
      launch_slot_totals(c->red, sl, zz0_dev, st);
      zz_ref = zz0_dev;
      zz_last = -1.0;
    } else if (read_res) {
      double zz0 = 0.0;
      sibfa_status e = read_totals(c, {S_ZZ}, &zz0);
      if (e != SIBFA_OK) return e;
      rho_true = rms_debye(c, zz0);
      zz_last = zz0;
      if (rho_true <= tol) {
        if (!fp32_res) break;
        fresh = false;   // confirm with the FP64 operator
        continue;
      }
    }
    read_res = true;
    if (it >= c->prm.max_iter || restarts > 8) { result = SIBFA_E_NOT_CONVERGED; break; }
    if (fresh) {
      // with zz_ref the kernels take kReplace as a factor of *zz_ref
      if (mix) zz_replace = zz_ref ? kReplace : kReplace * zz_last;
    } else {
      ++restarts;
    }
    fresh = false;
    // Iterations are enqueued in batches; a stop test after each update
    // (folded into the next direction update, or a one-block kernel at the
    // end of a batch) raises a flag in device memory that makes the
    // remaining enqueued kernels return at once, so the host reads the flag
    // once per batch instead of synchronising every iteration.
    launch_fill_int(flag, 0, 4, st);
    c->red.stop = flag;
    c->pm.stop = flag;
    int j = 0, j_done = 0, reason = 0;   // iterations of this run
    for (;;) {
      if (c->prof && c->marks.size() > 4096) fold_marks(c);
      int nb = 4;
      if (rate > 0.0 && rate < 1.0 && (zz_last > 0.0 || zz_ref)) {
        // deferred start: the first run ends at z.z = kReplace z.z0
        const double ratio = zz_ref ? zz_replace
                                    : (zz_replace > zz_stop ? zz_replace : zz_stop) / zz_last;
        const double est = std::ceil(std::log(ratio) / std::log(rate));
        nb = est < 1.0 ? 1 : (est > 12.0 ? 12 : (int)est);
      }
      const int j0 = j;
      for (int b = 0; b < nb && it + j < c->prm.max_iter; ++b) {
        const int k = kk + j;
        c->cur_tag = j;
        // with two streams, the direction kernel's own completion records
        // the fork event (a separate marker cost the main stream ~5 us)
        const bool fork_by_dir = k > 0 && c->periodic && c->aux != c->stream;
        if (k > 0) {
          // p = z + beta p, after the stop test of the previous iteration
          // when that was enqueued in this batch
          const int num = S_RZ0 + (k & 1), den = S_RZ0 + ((k - 1) & 1);
          Phase ph(c, SIBFA_PH_UPDATE);
          launch_direction(s, c->red, num, den, c->z, c->p, c->p32, b > 0 ? flag : nullptr, j,
                           zz_stop, zz_replace, zz_ref, st, fork_by_dir ? c->ev_fork : nullptr);
        }
        // the reciprocal chain (the critical path) on the main stream, the
        // real-space matvec beside it on the auxiliary stream: both stream
        // events then fall off the critical path
        if (c->periodic) {
          if (fork_by_dir) (void)hipStreamWaitEvent(c->aux, c->ev_fork, 0);
          else fork(c);
          {
            Phase ph(c, SIBFA_PH_MATVEC, c->aux, true);
            // the matvec's completion records the join event itself
            launch_matvec_real(s, c->red, c->p, c->p32, c->q, S_PQ, mix, c->aux,
                               c->aux != c->stream ? c->ev_join : nullptr, ph.start(),
                               ph.stop());
          }
          {
            Phase ph(c, SIBFA_PH_SPREAD);
            launch_spread_dip(s, c->pm, c->p, mix, st);
          }
          {
            Phase ph(c, SIBFA_PH_FFT);
            conv(c, mix, st);
          }
          if (c->aux != c->stream) (void)hipStreamWaitEvent(c->stream, c->ev_join, 0);
        } else {
          Phase ph(c, SIBFA_PH_MATVEC, st, true);
          launch_matvec_real(s, c->red, c->p, c->p32, c->q, S_PQ, mix, st, nullptr, ph.start(),
                             ph.stop());
        }
        {
          Phase ph(c, SIBFA_PH_MATVEC_RECIP);
          launch_matvec_recip(s, c->pm, c->red, c->p, c->q, S_PQ, mix, st);
        }
        {
          Phase ph(c, SIBFA_PH_UPDATE);
          if (blk)
            launch_pc_update(s, c->pcv, c->red, S_RZ0 + (k & 1), S_RZ0 + ((k + 1) & 1), c->x,
                             c->r, c->z, c->p, c->q, st);
          else
            launch_update(s, c->red, S_RZ0 + (k & 1), S_RZ0 + ((k + 1) & 1), c->x, c->r, c->z,
                          c->p, c->q, st);
          // the last iteration of a batch is tested here, the others by
          // the next direction update
          if (b == nb - 1 || it + j + 1 >= c->prm.max_iter)
            launch_check(c->red, flag, zz_dev, j + 1, zz_stop, zz_replace, zz_ref, st);
        }
        ++j;
      }
      c->cur_tag = -1;
      HIP_TRY(hipMemcpyAsync(c->h_ints + 8, flag, 4 * sizeof(int) + sizeof(double),
                             hipMemcpyDeviceToHost, st));
      if (zz_ref)
        HIP_TRY(hipMemcpyAsync(c->h_pinned + 60, zz0_dev, sizeof(double), hipMemcpyDeviceToHost, st));
      sibfa_status e = sync_read(c);
      if (e != SIBFA_OK) {
        c->red.stop = nullptr;
        c->pm.stop = nullptr;
        return e;
      }
      if (zz_ref) {   // the deferred z.z0: host values from here on
        zz_last = c->h_pinned[60];
        zz_replace = kReplace * zz_last;
        zz_ref = nullptr;
      }
      const int stop = c->h_ints[8];
      const int ran = stop ? c->h_ints[10] - j0 : j - j0;   // iterations this batch
      double zz_now;
      std::memcpy(&zz_now, c->h_ints + 12, sizeof(double));
      if (ran > 0 && zz_last > 0.0 && zz_now > 0.0) rate = std::pow(zz_now / zz_last, 1.0 / ran);
      zz_last = zz_now;
      if (stop) {
        j_done = c->h_ints[10];
        reason = c->h_ints[9];
        for (auto& m : c->marks)
          if (m.tag >= j_done) m.work = false;
        for (auto& m : c->marks) m.tag = -1;
        break;
      }
      for (auto& m : c->marks) m.tag = -1;
      if (it + j >= c->prm.max_iter) {
        j_done = j;
        break;
      }
    }
    c->red.stop = nullptr;
    c->pm.stop = nullptr;
    if (first_run && rate > 0.0 && rate < 1.0) c->rate_hint = rate;
    first_run = false;
    it += j_done;
    kk += j_done;
    if (reason == 3) {
      zz_replace = -1.0;
      read_res = false;
    }
    if (reason == 2) result = SIBFA_E_NOT_SPD;
    if (result == SIBFA_E_NOT_SPD) break;
    // the next residual is an FP64 one (only a cold start's first is FP32),
    // so x32 needs no refresh here
  }
  c->stats.iterations = it;
  c->stats.restarts = restarts;
  c->stats.true_rms_debye = rho_true;
  launch_pol_to_caller(s, c->perm, c->x, c->mu_c, st);
  c->mu_have = true;
  c->mu_valid = (result == SIBFA_OK);
  if (result == SIBFA_OK) push_history(c, st);
  if (result == SIBFA_E_NOT_SPD)
    return fail(c, result, "p.Tp <= 0: the polarization matrix is not positive definite");
  if (result == SIBFA_E_NOT_CONVERGED)
    return fail(c, result, "solver did not reach the tolerance within max_iter");
  return SIBFA_OK;
}

// Truncated conjugate gradient (TCG-n): `order` steps of the solver above
// from the direct-field guess (or the kept dipoles when warm), with no
// convergence test, host round trip
// or residual replacement, then the optional peek step x += omega alpha r.
// The same matvec, update and direction kernels; a check kernel after each
// update still raises the device flag on p.Tp <= 0 (a zero residual raises
// it first, harmlessly), read back with the energy.
sibfa_status solve_tcg(sibfa_ctx c, int order, double omega, bool warm, double* mu_out,
                       double* e_pol) {
  SysView s = make_view(c);
  hipStream_t st = c->stream;
  const bool mix = mixed(c);
  // the solver vectors (x, r) are overwritten: the last solve's dipoles
  // stay in mu_c for warm starts, and the next energy call solves again
  c->mu_valid = false;
  if (c->npol == 0) {
    if (mu_out) launch_fill_double(mu_out, 0.0, 3 * (size_t)c->n, st);
    if (e_pol) *e_pol = 0.0;
    return sync_read(c);
  }
  ensure_coef(c);
  if (warm) warm_guess(c, s, st);
  else launch_precond(s, c->E0, c->x, st);
  launch_copy4(c->x, c->x, c->x32, c->npol, st);
  matvec(c, c->x, c->x32, c->t, -1, mix);
  launch_init_residual(s, c->red, c->E0, c->t, c->r, c->z, c->p, c->p32, S_RZ0, st);
  int* flag = c->dints + 8;
  double* zz_dev = reinterpret_cast<double*>(c->dints + 12);
  launch_fill_int(flag, 0, 4, st);
  for (int k = 0; k < order; ++k) {
    if (k > 0)
      launch_direction(s, c->red, S_RZ0 + (k & 1), S_RZ0 + ((k - 1) & 1), c->z, c->p, c->p32,
                       nullptr, k, 0.0, -1.0, nullptr, st);
    matvec(c, c->p, c->p32, c->q, S_PQ, mix);
    launch_update(s, c->red, S_RZ0 + (k & 1), S_RZ0 + ((k + 1) & 1), c->x, c->r, c->z, c->p, c->q,
                  st);
    launch_check(c->red, flag, zz_dev, k + 1, 0.0, -1.0, nullptr, st);
  }
  if (omega != 0.0) launch_axpy4(s, c->x, c->z, omega, st);
  launch_dot(s, c->red, c->x, c->E0, S_MUE, st);
  if (mu_out) launch_pol_to_caller(s, c->perm, c->x, mu_out, st);
  HIP_TRY(hipMemcpyAsync(c->h_ints + 8, flag, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
  double mue = 0.0;
  sibfa_status e = read_totals(c, {S_MUE}, &mue);
  if (e != SIBFA_OK) return e;
  if (c->h_ints[8] && c->h_ints[9] == 2)
    return fail(c, SIBFA_E_NOT_SPD, "p.Tp <= 0: the polarization matrix is not positive definite");
  if (e_pol) *e_pol = -0.5 * kCoulomb * mue;
  return SIBFA_OK;
}

// Forces (caller order, kcal/mol/A) of the combined density of the records
// in sv and the dipoles v (polarizable order), FP64: the force kernels and,
// periodic, the PME force pass, all on the main stream.
void force_eval(sibfa_ctx c, const SysView& sv, const double4* v, double* out) {
  hipStream_t sm = c->stream;
  launch_mu_sites(sv, v, c->mu_s, c->mu_s32, sm);
  if (c->periodic) {
    launch_spread_mult(sv, c->pm, c->mu_s, false, sm);
    conv(c, false, sm, S_CTREC);
  }
  launch_force(sv, c->red, c->mu_s, c->mu_s32, c->Freal, false, false, sm);
  if (c->periodic)
    launch_gather_force(sv, c->pm, c->red, c->mu_s, c->Freal, c->perm, out, false, false, sm);
  else
    launch_forces_out(c->n, c->perm, c->Freal, out, sm);
}

double dot_now(sibfa_ctx c, const SysView& s, const double4* a, const double4* b,
               sibfa_status* st) {
  launch_dot(s, c->red, a, b, S_TCGD, c->stream);
  double v = 0.0;
  const sibfa_status r = read_totals(c, {S_TCGD}, &v);
  if (r != SIBFA_OK) *st = r;
  return v;
}

// TCG-n energy and forces (FP64).  The forward pass is the iteration of
// solve_tcg with every vector kept; the reverse pass propagates
// dE/d(everything) back through it, which leaves
//   dE = Ebar . dE0 + sum_k abar_k . dT b_k
// over the (n + 1) products T b_k of the forward pass.  The forces are then
//   F = F(M, -Ebar) - F(0, Ebar) + 1/2 sum_k [F(0, abar_k + b_k) - F(0, abar_k - b_k)],
// F(M, v) the force of the combined density (records M, dipoles v) and
// F(0, v) that of the dipoles alone: F(M, v) = F_MM + F_Mmu(v) + F_mumu(v),
// F_Mmu linear and F_mumu quadratic in v, and the bilinear T terms follow
// from the polarization identity.
sibfa_status tcg_forces(sibfa_ctx c, int n, double omega, bool warm, double* e_pol,
                        double* e_elec, double* forces, double* mu_out) {
  SysView s = make_view(c);
  hipStream_t st = c->stream;
  const size_t np = std::max(c->npol, 1);
  const size_t nn = c->n;
  // work vectors: X, R, Z [n + 1], P, Q, QB [n], then t, MU, EB, XB, RB, ZB,
  // PB, PBn, QBc, TB, tmp; records without multipoles; force scratch
  const int nvec = 3 * (n + 1) + 3 * n + 12;
  if (c->tcg_cap < n || c->tcg_np < np) {
    free_list(c, c->tcgbufs);
    c->tcg_cap = -1;
    double4* base = nullptr;
    double4 *sp0, *sd0, *sth0;
    double2* sth20;
    double *f1, *f2;
    if (!alloc_into(c, c->tcgbufs, base, (size_t)nvec * np) ||
        !alloc_into(c, c->tcgbufs, sp0, nn) || !alloc_into(c, c->tcgbufs, sd0, nn) ||
        !alloc_into(c, c->tcgbufs, sth0, nn) || !alloc_into(c, c->tcgbufs, sth20, nn) ||
        !alloc_into(c, c->tcgbufs, f1, 3 * nn) || !alloc_into(c, c->tcgbufs, f2, 3 * nn)) {
      free_list(c, c->tcgbufs);
      return fail(c, SIBFA_E_NOMEM, "truncated-CG force buffers");
    }
    c->tcg_cap = n;
    c->tcg_np = np;
  }
  double4* base = static_cast<double4*>(c->tcgbufs[0].p);
  double4* sp0 = static_cast<double4*>(c->tcgbufs[1].p);
  double4* sd0 = static_cast<double4*>(c->tcgbufs[2].p);
  double4* sth0 = static_cast<double4*>(c->tcgbufs[3].p);
  double2* sth20 = static_cast<double2*>(c->tcgbufs[4].p);
  double* f1 = static_cast<double*>(c->tcgbufs[5].p);
  double* f2 = static_cast<double*>(c->tcgbufs[6].p);
  auto vec = [&](int k) { return base + (size_t)k * np; };
  double4** X = new double4*[n + 1];
  double4** R = new double4*[n + 1];
  double4** Z = new double4*[n + 1];
  double4** P = new double4*[std::max(n, 1)];
  double4** Q = new double4*[std::max(n, 1)];
  double4** QBk = new double4*[std::max(n, 1)];
  int at = 0;
  for (int k = 0; k <= n; ++k) { X[k] = vec(at++); R[k] = vec(at++); Z[k] = vec(at++); }
  for (int k = 0; k < n; ++k) { P[k] = vec(at++); Q[k] = vec(at++); QBk[k] = vec(at++); }
  double4 *T0 = vec(at++), *MU = vec(at++), *EB = vec(at++), *XB = vec(at++), *RB = vec(at++),
          *ZB = vec(at++), *PB = vec(at++), *PBn = vec(at++), *QB = vec(at++), *TB = vec(at++),
          *TMP = vec(at++), *TMP2 = vec(at++);
  std::vector<double> rho(n + 1), sig(n), gam(n), bet(n), rhob(n + 1, 0.0);
  sibfa_status err = SIBFA_OK;
  float4* v32 = c->p32;
  auto Tv = [&](double4* v, double4* out) {
    launch_copy4(v, v, v32, c->npol, st);
    matvec(c, v, v32, out, -1, false);
  };
  ensure_coef(c);
  // ---- forward
  if (warm) {
    warm_guess(c, s, st);
    launch_copy4(c->x, X[0], nullptr, c->npol, st);
  } else {
    launch_precond(s, c->E0, X[0], st);
  }
  Tv(X[0], T0);
  launch_lincomb4(s, R[0], 1.0, c->E0, -1.0, T0, st);
  launch_precond(s, R[0], Z[0], st);
  rho[0] = dot_now(c, s, R[0], Z[0], &err);
  for (int k = 0; k < n; ++k) {
    if (k == 0) launch_copy4(Z[0], P[0], nullptr, c->npol, st);
    Tv(P[k], Q[k]);
    sig[k] = dot_now(c, s, P[k], Q[k], &err);
    if (!(sig[k] > 0.0) && rho[k] != 0.0) {
      err = fail(c, SIBFA_E_NOT_SPD, "p.Tp <= 0: the polarization matrix is not positive definite");
      break;
    }
    // a zero residual (the iterate is exact) stays put: gamma = 0
    gam[k] = sig[k] > 0.0 ? rho[k] / sig[k] : 0.0;
    launch_lincomb4(s, X[k + 1], 1.0, X[k], gam[k], P[k], st);
    launch_lincomb4(s, R[k + 1], 1.0, R[k], -gam[k], Q[k], st);
    launch_precond(s, R[k + 1], Z[k + 1], st);
    rho[k + 1] = dot_now(c, s, R[k + 1], Z[k + 1], &err);
    if (k < n - 1) {
      bet[k] = rho[k] != 0.0 ? rho[k + 1] / rho[k] : 0.0;
      launch_lincomb4(s, P[k + 1], 1.0, Z[k + 1], bet[k], P[k], st);
    }
  }
  if (err != SIBFA_OK) {
    delete[] X; delete[] R; delete[] Z; delete[] P; delete[] Q; delete[] QBk;
    return err;
  }
  launch_lincomb4(s, MU, 1.0, X[n], omega, Z[n], st);
  const double mue = dot_now(c, s, MU, c->E0, &err);
  // ---- reverse, seeded with d(-1/2 mu.E0) (no Coulomb factor: the force
  // evaluations below apply it)
  const double hf = -0.5;
  launch_lincomb4(s, EB, hf, MU, 0.0, nullptr, st);            // from E0 in -1/2 f mu.E0
  launch_lincomb4(s, XB, hf, c->E0, 0.0, nullptr, st);         // mubar -> xbar_n
  launch_lincomb4(s, ZB, omega * hf, c->E0, 0.0, nullptr, st); // zbar_n
  launch_lincomb4(s, RB, 0.0, c->E0, 0.0, nullptr, st);        // rbar_n = 0
  for (int k = n - 1; k >= 0; --k) {
    launch_lincomb4(s, PB, 0.0, c->E0, 0.0, nullptr, st);      // pbar_k = 0
    if (k < n - 1) {
      launch_lincomb4(s, ZB, 1.0, ZB, 1.0, PBn, st);
      const double betab = dot_now(c, s, PBn, P[k], &err);
      launch_lincomb4(s, PB, 1.0, PB, bet[k], PBn, st);
      if (rho[k] != 0.0) {
        rhob[k + 1] += betab / rho[k];
        rhob[k] -= betab * rho[k + 1] / (rho[k] * rho[k]);
      }
    }
    launch_lincomb4(s, RB, 1.0, RB, rhob[k + 1], Z[k + 1], st);
    launch_lincomb4(s, ZB, 1.0, ZB, rhob[k + 1], R[k + 1], st);
    launch_precond(s, ZB, TMP, st);
    launch_lincomb4(s, RB, 1.0, RB, 1.0, TMP, st);
    double gammab = -dot_now(c, s, RB, Q[k], &err);
    launch_lincomb4(s, QB, -gam[k], RB, 0.0, nullptr, st);
    gammab += dot_now(c, s, XB, P[k], &err);
    launch_lincomb4(s, PB, 1.0, PB, gam[k], XB, st);
    double sigb = 0.0;
    if (sig[k] > 0.0) {
      rhob[k] += gammab / sig[k];
      sigb = -gammab * rho[k] / (sig[k] * sig[k]);
    }
    launch_lincomb4(s, PB, 1.0, PB, sigb, Q[k], st);
    launch_lincomb4(s, QB, 1.0, QB, sigb, P[k], st);
    launch_copy4(QB, QBk[k], nullptr, c->npol, st);
    Tv(QB, TMP);
    launch_lincomb4(s, PB, 1.0, PB, 1.0, TMP, st);
    // level k: rbar_k continues from RB, zbar_k starts at zero
    launch_lincomb4(s, ZB, 0.0, ZB, 0.0, nullptr, st);
    launch_copy4(PB, PBn, nullptr, c->npol, st);
  }
  // initial steps: p0 = z0, rho0 = r0.z0, z0 = alpha r0, r0 = E0 - T x0
  launch_lincomb4(s, ZB, 1.0, ZB, 1.0, PBn, st);
  launch_lincomb4(s, RB, 1.0, RB, rhob[0], Z[0], st);
  launch_lincomb4(s, ZB, 1.0, ZB, rhob[0], R[0], st);
  launch_precond(s, ZB, TMP, st);
  launch_lincomb4(s, RB, 1.0, RB, 1.0, TMP, st);
  launch_lincomb4(s, EB, 1.0, EB, 1.0, RB, st);
  launch_lincomb4(s, TB, -1.0, RB, 0.0, nullptr, st);
  Tv(TB, TMP);
  launch_lincomb4(s, XB, 1.0, XB, 1.0, TMP, st);
  if (!warm) {   // x0 = alpha E0
    launch_precond(s, XB, TMP, st);
    launch_lincomb4(s, EB, 1.0, EB, 1.0, TMP, st);
  }
  // ---- forces
  if (forces) {
    launch_zero_records(s, sp0, sd0, sth0, sth20, st);
    SysView s0 = s;
    s0.sp = sp0; s0.sd = sd0; s0.sth = sth0; s0.sth2 = sth20;
    launch_lincomb4(s, TMP, -1.0, EB, 0.0, nullptr, st);
    force_eval(c, s, TMP, forces);                         // F(M, -Ebar)
    force_eval(c, s0, EB, f1);                             // F(0, Ebar)
    launch_axpy_d(3 * nn, -1.0, f1, forces, st);
    // pairs (QB_k, P_k) and (TB, X0)
    for (int k = 0; k <= n; ++k) {
      const double4* a = k < n ? QBk[k] : TB;
      const double4* b = k < n ? P[k] : X[0];
      launch_lincomb4(s, TMP, 1.0, a, 1.0, b, st);
      launch_lincomb4(s, TMP2, 1.0, a, -1.0, b, st);
      force_eval(c, s0, TMP, f1);
      force_eval(c, s0, TMP2, f2);
      launch_axpy_d(3 * nn, 0.5, f1, forces, st);
      launch_axpy_d(3 * nn, -0.5, f2, forces, st);
    }
  }
  if (mu_out) launch_pol_to_caller(s, c->perm, MU, mu_out, st);
  delete[] X; delete[] R; delete[] Z; delete[] P; delete[] Q; delete[] QBk;
  if (err != SIBFA_OK) return err;
  double tot[4] = {0, 0, 0, 0};
  sibfa_status r = c->periodic ? read_totals(c, {S_EREAL, S_AUX, S_ESELF, S_EREC0}, tot)
                               : read_totals(c, {S_EREAL, S_AUX}, tot);
  if (r != SIBFA_OK) return r;
  if (e_pol) *e_pol = -0.5 * kCoulomb * mue;
  if (e_elec) *e_elec = kCoulomb * (tot[0] + tot[1] + tot[2] + tot[3]);
  return SIBFA_OK;
}

// Spreading brick edge along an axis of K points: the largest size <=
// kBrick whose last (partial) brick still spans order - 1 points, so that
// every grid point lies in the tiles of at most two bricks per axis; 0 if
// none fits.
int brick_edge(int K, int order) {
  for (int b = kBrick; b >= order - 1 && b >= 1; --b) {
    const int rem = K % b;
    if (rem == 0 || rem >= order - 1) return b;
  }
  return 0;
}

sibfa_status setup_pme(sibfa_ctx c) {
  free_list(c, c->pmebufs);
  PmeView& pm = c->pm;
  pm = PmeView{};
  if (!c->periodic) {
    pm.order = 5;
    return SIBFA_OK;
  }
  const int order = c->prm.order;
  pm.order = order;
  for (int a = 0; a < 3; ++a) {
    pm.K[a] = c->prm.grid[a];
    pm.scale[a] = pm.K[a] / c->box[a];
    int rad[16];
    factor_radices(pm.K[a], rad, &pm.nrad[a]);
    pm.radcode[a] = 0;
    for (int k = 0; k < pm.nrad[a]; ++k) pm.radcode[a] |= (unsigned)(rad[k] - 2) << (2 * k);
  }
  pm.kxh = pm.K[0] / 2 + 1;
  pm.beta = c->prm.ewald_beta;
  for (int a = 0; a < 3; ++a) {
    pm.Bb[a] = brick_edge(pm.K[a], order);
    if (pm.Bb[a] == 0) return fail(c, SIBFA_E_ARG, "no spreading brick size fits this grid");
    pm.nb[a] = (pm.K[a] + pm.Bb[a] - 1) / pm.Bb[a];
  }
  c->nbricks = pm.nb[0] * pm.nb[1] * pm.nb[2];
  pm.tile_size = (pm.Bb[0] + order - 1) * (pm.Bb[1] + order - 1) * (pm.Bb[2] + order - 1);
  {
    const size_t nbk = (size_t)c->nbricks;
    if (!alloc_into(c, c->pmebufs, c->bcount, nbk + 1) ||
        !alloc_into(c, c->pmebufs, c->bcursor, nbk) ||
        !alloc_into(c, c->pmebufs, c->brick_of, (size_t)c->n) ||
        !alloc_into(c, c->pmebufs, c->bscan_tmp, scan_temp_ints((int)nbk + 1) + 16) ||
        !alloc_into(c, c->pmebufs, c->bstart_pol, nbk + 1) ||
        !alloc_into(c, c->pmebufs, c->border_pol, (size_t)c->n) ||
        !alloc_into(c, c->pmebufs, c->bstart_all, nbk + 1) ||
        !alloc_into(c, c->pmebufs, c->border_all, (size_t)c->n))
      return fail(c, SIBFA_E_NOMEM, "PME brick allocation failed");
    pm.bstart_pol = c->bstart_pol;
    pm.border_pol = c->border_pol;
    pm.bstart_all = c->bstart_all;
    pm.border_all = c->border_all;
  }
  const size_t nr = (size_t)pm.K[0] * pm.K[1] * pm.K[2];
  const size_t nh = (size_t)pm.kxh * pm.K[1] * pm.K[2];
  double *Q, *phi, *G;
  double2* C;
  float *Q32, *phi32, *G32;
  float2* C32;
  if (!alloc_into(c, c->pmebufs, Q, nr) || !alloc_into(c, c->pmebufs, phi, nr) ||
      !alloc_into(c, c->pmebufs, C, nh) || !alloc_into(c, c->pmebufs, G, nh) ||
      !alloc_into(c, c->pmebufs, Q32, nr) || !alloc_into(c, c->pmebufs, phi32, nr) ||
      !alloc_into(c, c->pmebufs, C32, nh) || !alloc_into(c, c->pmebufs, G32, nh) ||
      !alloc_into(c, c->pmebufs, pm.tiles, (size_t)c->nbricks * pm.tile_size) ||
      !alloc_into(c, c->pmebufs, pm.tiles32, (size_t)c->nbricks * pm.tile_size))
    return fail(c, SIBFA_E_NOMEM, "PME grid allocation failed");
  pm.Q = Q; pm.phi = phi; pm.C = C; pm.G = G;
  pm.Q32 = Q32; pm.phi32 = phi32; pm.C32 = C32; pm.G32 = G32;
  launch_fill_double(Q, 0.0, nr, c->stream);
  launch_fill_float(Q32, 0.f, nr, c->stream);
  // twiddles
  const long double twopi = 6.283185307179586476925286766559L;
  for (int a = 0; a < 3; ++a) {
    const int K = pm.K[a];
    std::vector<double2> tw(K);
    std::vector<float2> tw32(K);
    for (int k = 0; k < K; ++k) {
      const long double ang = -twopi * k / K;
      tw[k] = make_double2((double)cosl(ang), (double)sinl(ang));
      tw32[k] = make_float2((float)cosl(ang), (float)sinl(ang));
    }
    double2* d;
    float2* f;
    if (!alloc_into(c, c->pmebufs, d, K) || !alloc_into(c, c->pmebufs, f, K))
      return fail(c, SIBFA_E_NOMEM, "PME table allocation failed");
    HIP_TRY(hipMemcpy(d, tw.data(), K * sizeof(double2), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(f, tw32.data(), K * sizeof(float2), hipMemcpyHostToDevice));
    pm.tw[a] = d;
    pm.tw32[a] = f;
  }
  // influence function G(m) = B(m) C(m) on the half spectrum
  std::vector<double> mod[3];
  for (int a = 0; a < 3; ++a) mod[a] = bspline_moduli(pm.K[a], order);
  const double V = c->box[0] * c->box[1] * c->box[2];
  const double beta = c->prm.ewald_beta;
  std::vector<double> g(nh);
  std::vector<float> g32(nh);
  for (int kz = 0; kz < pm.K[2]; ++kz) {
    const int mz = kz <= pm.K[2] / 2 ? kz : kz - pm.K[2];
    for (int ky = 0; ky < pm.K[1]; ++ky) {
      const int my = ky <= pm.K[1] / 2 ? ky : ky - pm.K[1];
      for (int kx = 0; kx < pm.kxh; ++kx) {
        const double fx = kx / c->box[0], fy = my / c->box[1], fz = mz / c->box[2];
        const double m2 = fx * fx + fy * fy + fz * fz;
        double val = 0.0;
        if (kx != 0 || my != 0 || mz != 0) {
          val = std::exp(-kPi * kPi * m2 / (beta * beta)) / (kPi * V * m2);
          val /= mod[0][kx] * mod[1][ky] * mod[2][kz];
        }
        const size_t idx = ((size_t)kz * pm.K[1] + ky) * pm.kxh + kx;
        g[idx] = val;
        g32[idx] = (float)val;
      }
    }
  }
  HIP_TRY(hipMemcpy(G, g.data(), nh * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(G32, g32.data(), nh * sizeof(float), hipMemcpyHostToDevice));
  return SIBFA_OK;
}

sibfa_status finite_check(sibfa_ctx c, const double* dev, size_t count, const char* what) {
  // device-side test; one int comes back
  launch_fill_int(c->dints + 6, 0, 1, c->stream);
  launch_nonfinite(dev, count, c->dints + 6, c->stream);
  HIP_TRY(hipMemcpyAsync(c->h_ints + 6, c->dints + 6, sizeof(int), hipMemcpyDeviceToHost,
                         c->stream));
  sibfa_status st = sync_read(c);
  if (st != SIBFA_OK) return st;
  if (c->h_ints[6]) return fail(c, SIBFA_E_ARG, std::string(what) + " contains NaN or Inf");
  return SIBFA_OK;
}

}  // namespace

// ============================================================ C-ABI
extern "C" {

void sibfa_default_params(sibfa_params* p) {
  if (!p) return;
  p->ewald_beta = 0.4;
  p->cutoff = 9.0;
  p->grid[0] = p->grid[1] = p->grid[2] = 32;
  p->order = 5;
  p->thole_a = 0.28;
  p->tol_debye = 1e-8;
  p->max_iter = 200;
  p->precision = SIBFA_FP64;
  p->precond = SIBFA_PRECOND_DIAG;
}

sibfa_status sibfa_create(sibfa_ctx* out, int device, void* hip_stream, sibfa_alloc_fn alloc_fn,
                          sibfa_free_fn free_fn, void* user) {
  if (!out) return SIBFA_E_ARG;
  *out = nullptr;
  if ((alloc_fn == nullptr) != (free_fn == nullptr)) return SIBFA_E_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SIBFA_E_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return SIBFA_E_DEVICE;
  sibfa_ctx c = new sibfa_ctx_s();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->af = alloc_fn;
  c->ff = free_fn;
  c->user = user;
  sibfa_default_params(&c->prm);
  if (hipHostMalloc((void**)&c->h_pinned, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->h_ints, 16 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
    sibfa_destroy(c);
    return SIBFA_E_NOMEM;
  }
  const char* ov = std::getenv("SIBFA_PME_OVERLAP");
  if (ov && std::atoi(ov) == 0) {
    c->aux = c->stream;
  } else if (hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess ||
             // the events order the two streams of one device only: no
             // system-scope fence (kernel boundaries already make device
             // memory coherent across the device)
             hipEventCreateWithFlags(&c->ev_fork,
                                     hipEventDisableTiming | hipEventDisableSystemFence) != hipSuccess ||
             hipEventCreateWithFlags(&c->ev_join,
                                     hipEventDisableTiming | hipEventDisableSystemFence) != hipSuccess ||
             hipEventCreateWithFlags(&c->ev_bricks,
                                     hipEventDisableTiming | hipEventDisableSystemFence) != hipSuccess) {
    sibfa_destroy(c);
    return SIBFA_E_DEVICE;
  }
  *out = c;
  return SIBFA_OK;
}

void sibfa_destroy(sibfa_ctx c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  if (c->aux && c->aux != c->stream) (void)hipStreamSynchronize(c->aux);
  release_system(c);
  for (hipEvent_t e : c->evpool) (void)hipEventDestroy(e);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  if (c->ev_bricks) (void)hipEventDestroy(c->ev_bricks);
  if (c->aux && c->aux != c->stream) (void)hipStreamDestroy(c->aux);
  if (c->h_pinned) (void)hipHostFree(c->h_pinned);
  if (c->h_ints) (void)hipHostFree(c->h_ints);
  if (c->h_vir) (void)hipHostFree(c->h_vir);
  delete c;
}

const char* sibfa_last_error(sibfa_ctx c) { return c ? c->err.c_str() : "NULL context"; }

size_t sibfa_footprint_bytes(int n_sites, int n_polarizable, const double* box,
                             const sibfa_params* p) {
  if (n_sites <= 0 || n_polarizable < 0 || n_polarizable > n_sites || !p) return 0;
  const size_t n = n_sites, np = std::max(n_polarizable, 1);
  size_t bytes = 0;
  bytes += n * (3 + 1 + 3 + 6 + 6 + 1 + 3) * sizeof(double);        // caller copies
  bytes += n * (4 + 4 + 4 + 2) * sizeof(double) + n * (4 + 4 + 4 + 2) * sizeof(float);
  bytes += n * 12 * sizeof(int) + n * (1 + 6 + 6) * sizeof(double) + n * 24;  // pol arrays
  bytes += n * (2 * 32 + 16);                                         // mu_s, Freal
  bytes += np * (7 * 32 + 2 * 16);                                    // solver vectors
  size_t cap_all, cap_pol;
  if (box) {
    const double V = box[0] * box[1] * box[2];
    const double sph = 4.0 / 3.0 * kPi * std::pow(p->cutoff, 3);
    cap_all = std::min(n, (size_t)(1.3 * n / V * sph) + 64);
    cap_pol = std::min(np, (size_t)(1.3 * np / V * sph) + 64);
    const size_t nr = (size_t)p->grid[0] * p->grid[1] * p->grid[2];
    const size_t nh = (size_t)(p->grid[0] / 2 + 1) * p->grid[1] * p->grid[2];
    bytes += nr * 2 * (8 + 4) + nh * (16 + 8 + 8 + 4);
    size_t tiles = 1;
    for (int a = 0; a < 3; ++a) {
      const int e = std::max(brick_edge(p->grid[a], p->order), 1);
      tiles *= (size_t)((p->grid[a] + e - 1) / e) * (e + p->order - 1);
    }
    bytes += tiles * (8 + 4);
    size_t cells = 1;   // cell grid as in sibfa_set_system: count, start, cursor, maxima
    for (int a = 0; a < 3; ++a)
      cells *= (size_t)std::max(1, std::min(1024, (int)std::floor(box[a] / (0.5 * p->cutoff))));
    bytes += cells * (3 * sizeof(int) + sizeof(int4));
  } else {
    cap_all = n;
    cap_pol = np;
  }
  bytes += (n * (cap_all + 8) + np * (cap_pol + 8)) * sizeof(int);
  bytes += 4 * n * sizeof(int);
  // cached pair coefficients: FP64 for the polarizable and same-molecule
  // lists, plus an FP32 copy of the former in mixed precision
  bytes += np * (cap_pol + 8) * 2 * sizeof(double);
  if (p->precision == SIBFA_MIXED) bytes += np * cap_pol * 2 * sizeof(float);
  if (p->precond == SIBFA_PRECOND_MOLBLOCK)   // group sizes, members, packed inverses
    bytes += n * ((1 + kPcMax) * sizeof(int) + kPcPacked * sizeof(double));
  return bytes + (1 << 20);
}

sibfa_status sibfa_set_system(sibfa_ctx c, int n_sites, const double* xyz, const int32_t* mol,
                              const double* box, const sibfa_params* params) {
  if (!c) return SIBFA_E_ARG;
  if (n_sites <= 0 || !xyz || !mol) return fail(c, SIBFA_E_ARG, "n_sites > 0, xyz and mol required");
  sibfa_status st = check_params(c, params, box);
  if (st != SIBFA_OK) return st;
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipStreamSynchronize(c->stream));
  release_system(c);
  c->prm = *params;
  c->n = n_sites;
  c->npol = 0;
  c->periodic = box ? 1 : 0;
  for (int a = 0; a < 3; ++a) c->box[a] = box ? box[a] : 0.0;
  c->stats = sibfa_stats{};
  c->stats.n_sites = n_sites;
  // cell grid: edge >= cutoff/2 (periodic); one cell for clusters
  if (c->periodic) {
    for (int a = 0; a < 3; ++a)
      c->nc[a] = std::max(1, std::min(1024, (int)std::floor(c->box[a] / (0.5 * c->prm.cutoff))));
  } else {
    c->nc[0] = c->nc[1] = c->nc[2] = 1;
  }
  c->ncell = c->nc[0] * c->nc[1] * c->nc[2];
  const size_t n = n_sites;
  auto& L = c->bufs;
  c->pcv = PcView{};
  bool ok = alloc_into(c, L, c->xyz_c, 3 * n) && alloc_into(c, L, c->q_c, n) &&
            alloc_into(c, L, c->dip_c, 3 * n) && alloc_into(c, L, c->quad_c, 6 * n) &&
            alloc_into(c, L, c->alpha_c, 6 * n) && alloc_into(c, L, c->thole_c, n) &&
            alloc_into(c, L, c->mu_c, 3 * n) && alloc_into(c, L, c->mol_c, n) &&
            alloc_into(c, L, c->cell_of, n) && alloc_into(c, L, c->cell_count, c->ncell + 1) &&
            alloc_into(c, L, c->cell_start, c->ncell + 1) && alloc_into(c, L, c->cursor, c->ncell) &&
            alloc_into(c, L, c->cellmax, c->ncell) &&
            alloc_into(c, L, c->perm, n) && alloc_into(c, L, c->inv_perm, n) &&
            alloc_into(c, L, c->mol_count, n) && alloc_into(c, L, c->mol_s, n) &&
            alloc_into(c, L, c->scan_tmp, scan_temp_ints((int)std::max<size_t>(n + 1, c->ncell + 1)) + 16) &&
            alloc_into(c, L, c->sp, n) && alloc_into(c, L, c->sd, n) && alloc_into(c, L, c->sth, n) &&
            alloc_into(c, L, c->sth2, n) && alloc_into(c, L, c->sp32, n) &&
            alloc_into(c, L, c->sd32, n) && alloc_into(c, L, c->sth32, n) &&
            alloc_into(c, L, c->sth232, n) && alloc_into(c, L, c->sa, n) &&
            alloc_into(c, L, c->is_pol, n + 1) && alloc_into(c, L, c->pol_scan, n + 1) &&
            alloc_into(c, L, c->polidx, n) && alloc_into(c, L, c->polsite, n) &&
            alloc_into(c, L, c->pp, n) && alloc_into(c, L, c->pp32, n) && alloc_into(c, L, c->pa, n) &&
            alloc_into(c, L, c->alpha_s, 6 * n) && alloc_into(c, L, c->ainv_s, 6 * n) &&
            alloc_into(c, L, c->dints, 16 + 16 + 8) && alloc_into(c, L, c->dsums, 8) && alloc_into(c, L, c->E0, n) && alloc_into(c, L, c->x, n) &&
            alloc_into(c, L, c->r, n) && alloc_into(c, L, c->z, n) && alloc_into(c, L, c->p, n) &&
            alloc_into(c, L, c->q, n) && alloc_into(c, L, c->t, n) && alloc_into(c, L, c->p32, n) &&
            alloc_into(c, L, c->x32, n) && alloc_into(c, L, c->p2, n) && alloc_into(c, L, c->p2_32, n) && alloc_into(c, L, c->mu_s, n) &&
            alloc_into(c, L, c->mu_s32, n) && alloc_into(c, L, c->Freal, n);
  if (ok && c->prm.precond == SIBFA_PRECOND_MOLBLOCK)
    ok = alloc_into(c, L, c->pcv.n, n) && alloc_into(c, L, c->pcv.mem, (size_t)kPcMax * n) &&
         alloc_into(c, L, c->pcv.inv, (size_t)kPcPacked * n);
  for (int k = 0; k < 4 && ok; ++k) ok = alloc_into(c, L, c->ncnt[k], n);
  ok = ok && alloc_into(c, L, c->ncnear, n);
  // partial sums: one per block of the largest reducing launch (site
  // kernels use >= 16 sites per block; the z pass at most K1 * (K0/2+1);
  // the brick-parallel PME gathers one per spreading brick)
  size_t mb = n / 4 + 8192;
  if (c->periodic) {
    mb += (size_t)c->prm.grid[1] * (c->prm.grid[0] / 2 + 1);
    size_t bricks = 1;
    for (int a = 0; a < 3; ++a) {
      const int e = std::max(brick_edge(c->prm.grid[a], c->prm.order), 1);
      bricks *= (size_t)((c->prm.grid[a] + e - 1) / e);
    }
    mb = std::max(mb, bricks);
  }
  const int max_blocks = (int)mb;
  double* partials;
  ok = ok && alloc_into(c, L, partials, (size_t)S_COUNT * max_blocks);
  if (ok && hipHostMalloc((void**)&c->h_part, (size_t)S_COUNT * max_blocks * sizeof(double),
                          hipHostMallocDefault) != hipSuccess) {
    c->h_part = nullptr;
    ok = false;
  }
  if (!ok) {
    release_system(c);
    return fail(c, SIBFA_E_NOMEM, "device allocation failed");
  }
  c->red = Reduce{};
  c->red.partials = partials;
  c->red.max_blocks = max_blocks;
  launch_fill_double(partials, 0.0, (size_t)S_COUNT * max_blocks, c->stream);
  launch_fill_int(c->is_pol + n, 0, 1, c->stream);
  HIP_TRY(hipMemcpyAsync(c->xyz_c, xyz, 3 * n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->mol_c, mol, n * sizeof(int), hipMemcpyDeviceToDevice, c->stream));
  st = finite_check(c, c->xyz_c, 3 * n, "xyz");
  if (st != SIBFA_OK) { release_system(c); return st; }
  st = setup_pme(c);
  if (st != SIBFA_OK) { release_system(c); return st; }
  c->have_sys = true;
  c->dirty_sort = true;
  c->ids_ok = c->pol_ok = false;
  return SIBFA_OK;
}

sibfa_status sibfa_update_positions(sibfa_ctx c, const double* xyz) {
  if (!c) return SIBFA_E_ARG;
  if (!c->have_sys) return fail(c, SIBFA_E_STATE, "sibfa_set_system has not been called");
  if (!xyz) return fail(c, SIBFA_E_ARG, "xyz is NULL");
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipMemcpyAsync(c->xyz_c, xyz, 3 * (size_t)c->n * sizeof(double), hipMemcpyDeviceToDevice,
                         c->stream));
  // non-finite coordinates are caught by the cell binning of the next call
  // that computes (reported there as SIBFA_E_ARG)
  c->dirty_sort = true;
  c->dirty_rot = c->have_frames;
  c->e0_valid = false;
  c->mu_valid = false;
  return SIBFA_OK;
}

sibfa_status sibfa_set_multipoles(sibfa_ctx c, const double* q, const double* dip, const double* quad) {
  if (!c) return SIBFA_E_ARG;
  if (!c->have_sys) return fail(c, SIBFA_E_STATE, "sibfa_set_system has not been called");
  if (!q) return fail(c, SIBFA_E_ARG, "q is NULL");
  HIP_TRY(hipSetDevice(c->device));
  const size_t n = c->n;
  hipStream_t s = c->stream;
  HIP_TRY(hipMemcpyAsync(c->q_c, q, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (dip) HIP_TRY(hipMemcpyAsync(c->dip_c, dip, 3 * n * sizeof(double), hipMemcpyDeviceToDevice, s));
  else launch_fill_double(c->dip_c, 0.0, 3 * n, s);
  if (quad) HIP_TRY(hipMemcpyAsync(c->quad_c, quad, 6 * n * sizeof(double), hipMemcpyDeviceToDevice, s));
  else launch_fill_double(c->quad_c, 0.0, 6 * n, s);
  sibfa_status st = finite_check(c, c->q_c, n, "q");
  if (st == SIBFA_OK) st = finite_check(c, c->dip_c, 3 * n, "dip");
  if (st == SIBFA_OK) st = finite_check(c, c->quad_c, 6 * n, "quad");
  if (st != SIBFA_OK) return st;
  c->have_mult = true;
  c->have_frames = false;   // global multipoles given: local frames off
  c->ct_on = false;         // the lone-pair checks were made against the old ones
  c->dirty_mult = true;
  c->e0_valid = false;
  c->mu_valid = false;
  return SIBFA_OK;
}

sibfa_status sibfa_set_polarizabilities(sibfa_ctx c, const double* alpha, const double* thole) {
  if (!c) return SIBFA_E_ARG;
  if (!c->have_sys) return fail(c, SIBFA_E_STATE, "sibfa_set_system has not been called");
  if (!alpha) return fail(c, SIBFA_E_ARG, "alpha is NULL");
  HIP_TRY(hipSetDevice(c->device));
  const size_t n = c->n;
  HIP_TRY(hipMemcpyAsync(c->alpha_c, alpha, 6 * n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  c->has_thole = thole != nullptr;
  if (thole) HIP_TRY(hipMemcpyAsync(c->thole_c, thole, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  sibfa_status st = finite_check(c, c->alpha_c, 6 * n, "alpha");
  if (st == SIBFA_OK && thole) st = finite_check(c, c->thole_c, n, "thole");
  if (st != SIBFA_OK) return st;
  c->have_pol = true;
  c->have_frames = false;   // new polarizabilities: local frames off
  c->ct_on = false;
  c->dirty_pol = true;
  c->pol_ok = false;
  c->e0_valid = false;
  c->mu_valid = false;
  c->mu_have = false;
  c->hist_count = 0;
  return SIBFA_OK;
}

sibfa_status sibfa_set_local_frames(sibfa_ctx c, const int32_t* frames, const double* dip_local,
                                   const double* quad_local, const double* alpha_local) {
  if (!c) return SIBFA_E_ARG;
  if (!c->have_sys) return fail(c, SIBFA_E_STATE, "sibfa_set_system has not been called");
  if (!c->have_mult) return fail(c, SIBFA_E_STATE, "sibfa_set_multipoles has not been called");
  if (!c->have_pol) return fail(c, SIBFA_E_STATE, "sibfa_set_polarizabilities has not been called");
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (c->aux && c->aux != c->stream) HIP_TRY(hipStreamSynchronize(c->aux));
  if (!frames) {
    // off: the global multipoles stay those of the last rotation
    c->have_frames = false;
    return SIBFA_OK;
  }
  const int n = c->n;
  std::vector<int> hf(3 * (size_t)n), hm(n);
  HIP_TRY(hipMemcpy(hf.data(), frames, 3 * (size_t)n * sizeof(int), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(hm.data(), c->mol_c, (size_t)n * sizeof(int), hipMemcpyDeviceToHost));
  // distinct frames in order of first use; every site's frame is three
  // distinct sites of its own molecule, or (-1, -1, -1)
  std::vector<int> group_of(n, -1), gf, gcount;
  {
    std::map<std::array<int, 3>, int> gid;   // frame -> group, numbered by first use
    for (int i = 0; i < n; ++i) {
      const int o = hf[3 * i], a = hf[3 * i + 1], b = hf[3 * i + 2];
      if (o < 0 && a < 0 && b < 0) continue;
      if (o < 0 || a < 0 || b < 0 || o >= n || a >= n || b >= n || o == a || o == b || a == b)
        return fail(c, SIBFA_E_ARG, "frame of site " + std::to_string(i) +
                                        ": three distinct site indices in [0, n_sites) or -1 -1 -1");
      if (hm[o] != hm[i] || hm[a] != hm[i] || hm[b] != hm[i])
        return fail(c, SIBFA_E_ARG, "frame of site " + std::to_string(i) +
                                        ": the frame sites must belong to the site's molecule");
      const std::array<int, 3> key{o, a, b};
      auto it = gid.find(key);
      int g;
      if (it == gid.end()) {
        g = (int)gcount.size();
        gid.emplace(key, g);
        gf.insert(gf.end(), {o, a, b});
        gcount.push_back(0);
      } else {
        g = it->second;
      }
      group_of[i] = g;
      gcount[g]++;
    }
  }
  const int G = (int)gcount.size();
  std::vector<int> gstart(G + 1, 0), gsites;
  for (int g = 0; g < G; ++g) gstart[g + 1] = gstart[g] + gcount[g];
  gsites.resize(std::max(gstart[G], 1));
  {
    std::vector<int> cur(gstart.begin(), gstart.end() - 1);
    for (int i = 0; i < n; ++i)
      if (group_of[i] >= 0) gsites[cur[group_of[i]]++] = i;   // increasing site index
  }
  std::vector<int> sstart(n + 1, 0), sref(std::max(3 * G, 1));
  for (int g = 0; g < G; ++g)
    for (int k = 0; k < 3; ++k) sstart[gf[3 * g + k] + 1]++;
  for (int i = 0; i < n; ++i) sstart[i + 1] += sstart[i];
  {
    std::vector<int> cur(sstart.begin(), sstart.end() - 1);
    for (int g = 0; g < G; ++g)
      for (int k = 0; k < 3; ++k) sref[cur[gf[3 * g + k]]++] = 3 * g + k;   // increasing g
  }
  free_list(c, c->framebufs);
  c->have_frames = false;
  auto& L = c->framebufs;
  const size_t nn = n;
  const bool ok = alloc_into(c, L, c->frames_d, 3 * nn) && alloc_into(c, L, c->dloc, 3 * nn) &&
                  alloc_into(c, L, c->qloc, 6 * nn) &&
                  (!alpha_local || alloc_into(c, L, c->aloc, 6 * nn)) &&
                  alloc_into(c, L, c->gframe, std::max<size_t>(3 * (size_t)G, 1)) &&
                  alloc_into(c, L, c->gstart, (size_t)G + 1) &&
                  alloc_into(c, L, c->gsites, gsites.size()) &&
                  alloc_into(c, L, c->sstart, nn + 1) && alloc_into(c, L, c->sref, sref.size()) &&
                  alloc_into(c, L, c->Cs, 9 * nn) &&
                  alloc_into(c, L, c->Fg, std::max<size_t>(9 * (size_t)G, 1)) &&
                  alloc_into(c, L, c->FS, nn) && alloc_into(c, L, c->GS, 6 * nn);
  if (!ok) {
    free_list(c, c->framebufs);
    return fail(c, SIBFA_E_NOMEM, "local frame allocation failed");
  }
  hipStream_t st = c->stream;
  HIP_TRY(hipMemcpyAsync(c->frames_d, frames, 3 * nn * sizeof(int), hipMemcpyDeviceToDevice, st));
  if (dip_local) HIP_TRY(hipMemcpyAsync(c->dloc, dip_local, 3 * nn * sizeof(double), hipMemcpyDeviceToDevice, st));
  else launch_fill_double(c->dloc, 0.0, 3 * nn, st);
  if (quad_local) HIP_TRY(hipMemcpyAsync(c->qloc, quad_local, 6 * nn * sizeof(double), hipMemcpyDeviceToDevice, st));
  else launch_fill_double(c->qloc, 0.0, 6 * nn, st);
  if (alpha_local) HIP_TRY(hipMemcpyAsync(c->aloc, alpha_local, 6 * nn * sizeof(double), hipMemcpyDeviceToDevice, st));
  if (G > 0) HIP_TRY(hipMemcpyAsync(c->gframe, gf.data(), 3 * (size_t)G * sizeof(int), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(c->gstart, gstart.data(), gstart.size() * sizeof(int), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(c->gsites, gsites.data(), gsites.size() * sizeof(int), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(c->sstart, sstart.data(), sstart.size() * sizeof(int), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(c->sref, sref.data(), sref.size() * sizeof(int), hipMemcpyHostToDevice, st));
  sibfa_status r = finite_check(c, c->dloc, 3 * nn, "dip_local");
  if (r == SIBFA_OK) r = finite_check(c, c->qloc, 6 * nn, "quad_local");
  if (r == SIBFA_OK && alpha_local) r = finite_check(c, c->aloc, 6 * nn, "alpha_local");
  if (r != SIBFA_OK) {
    free_list(c, c->framebufs);
    return r;
  }
  c->ngroups = G;
  c->have_frames = true;
  c->ct_on = false;   // the lone-pair checks were made against the old multipoles
  c->rot_alpha = alpha_local != nullptr;
  c->dirty_rot = true;
  if (c->rot_alpha) c->pol_ok = false;   // the rotated tensors are validated again
  c->e0_valid = false;
  c->mu_valid = false;
  return SIBFA_OK;
}

sibfa_status sibfa_permanent_field(sibfa_ctx c, double* field_out) {
  if (!c) return SIBFA_E_ARG;
  if (!field_out) return fail(c, SIBFA_E_ARG, "field_out is NULL");
  HIP_TRY(hipSetDevice(c->device));
  sibfa_status st = prepare(c);
  if (st != SIBFA_OK) return st;
  if (!c->e0_valid && (st = compute_E0(c)) != SIBFA_OK) return st;
  launch_pol_to_caller(make_view(c), c->perm, c->E0, field_out, c->stream);
  return sync_read(c);
}

sibfa_status sibfa_apply_T(sibfa_ctx c, const double* pin, double* tp_out) {
  if (!c) return SIBFA_E_ARG;
  if (!pin || !tp_out) return fail(c, SIBFA_E_ARG, "p and tp_out are required");
  HIP_TRY(hipSetDevice(c->device));
  sibfa_status st = prepare(c);
  if (st != SIBFA_OK) return st;
  ensure_coef(c);
  SysView s = make_view(c);
  launch_caller_to_pol(s, c->perm, pin, c->q, c->p32, c->stream);
  matvec(c, c->q, c->p32, c->t, -1, mixed(c));
  launch_pol_to_caller(s, c->perm, c->t, tp_out, c->stream);
  return sync_read(c);
}

sibfa_status sibfa_solve_induced(sibfa_ctx c, int warm_start, double* mu_out, int* iters,
                                 double* true_rms_debye) {
  if (!c) return SIBFA_E_ARG;
  HIP_TRY(hipSetDevice(c->device));
  sibfa_status st = prepare(c);
  if (st != SIBFA_OK) return st;
  if (!c->e0_valid && (st = compute_E0(c)) != SIBFA_OK) return st;
  st = solve(c, warm_start != 0);
  if (mu_out && c->mu_have)
    (void)hipMemcpyAsync(mu_out, c->mu_c, 3 * (size_t)c->n * sizeof(double), hipMemcpyDeviceToDevice,
                         c->stream);
  if (iters) *iters = c->stats.iterations;
  if (true_rms_debye) *true_rms_debye = c->stats.true_rms_debye;
  // the host scalars come from the solver's own (synchronized) stop test;
  // the dipole copy stays enqueued, so a following call's work queues
  // behind it without a host round trip
  if (st != SIBFA_OK) return st;
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SIBFA_OK : hip_fail(c, e, "kernel launch");
}

sibfa_status sibfa_solve_tcg(sibfa_ctx c, int order, double omega, int warm_start,
                             double* mu_out, double* e_pol) {
  if (!c) return SIBFA_E_ARG;
  if (order < 1 || order > SIBFA_TCG_MAX_ORDER)
    return fail(c, SIBFA_E_ARG, "order must lie in 1.." + std::to_string(SIBFA_TCG_MAX_ORDER));
  if (!std::isfinite(omega)) return fail(c, SIBFA_E_ARG, "omega must be finite");
  HIP_TRY(hipSetDevice(c->device));
  sibfa_status st = prepare(c);
  if (st != SIBFA_OK) return st;
  if (warm_start && !c->mu_have)
    return fail(c, SIBFA_E_STATE, "warm start without dipoles (solve or set_dipoles first)");
  if (!c->e0_valid && (st = compute_E0(c)) != SIBFA_OK) return st;
  return solve_tcg(c, order, omega, warm_start != 0, mu_out, e_pol);
}

sibfa_status sibfa_tcg_energy_forces(sibfa_ctx c, int order, double omega, int warm_start,
                                     double* e_pol, double* e_elec, double* forces,
                                     double* mu_out) {
  if (!c) return SIBFA_E_ARG;
  if (order < 1 || order > SIBFA_TCG_MAX_ORDER)
    return fail(c, SIBFA_E_ARG, "order must lie in 1.." + std::to_string(SIBFA_TCG_MAX_ORDER));
  if (!std::isfinite(omega)) return fail(c, SIBFA_E_ARG, "omega must be finite");
  HIP_TRY(hipSetDevice(c->device));
  sibfa_status st = prepare(c);
  if (st != SIBFA_OK) return st;
  if (warm_start && !c->mu_have)
    return fail(c, SIBFA_E_STATE, "warm start without dipoles (solve or set_dipoles first)");
  if (!c->e0_valid && (st = compute_E0(c)) != SIBFA_OK) return st;
  join(c);
  // a warm start writes the guess into the solver vectors: the next energy
  // call solves again (warm from the kept dipoles)
  c->mu_valid = false;
  if (c->npol == 0) {
    if (forces) force_eval(c, make_view(c), c->x, forces);
    if (mu_out) launch_fill_double(mu_out, 0.0, 3 * (size_t)c->n, c->stream);
    double tot[4] = {0, 0, 0, 0};
    st = c->periodic ? read_totals(c, {S_EREAL, S_AUX, S_ESELF, S_EREC0}, tot)
                     : read_totals(c, {S_EREAL, S_AUX}, tot);
    if (st != SIBFA_OK) return st;
    if (e_pol) *e_pol = 0.0;
    if (e_elec) *e_elec = kCoulomb * (tot[0] + tot[1] + tot[2] + tot[3]);
    return SIBFA_OK;
  }
  return tcg_forces(c, order, omega, warm_start != 0, e_pol, e_elec, forces, mu_out);
}

// Totals of the virial slots (33 of them, S_VRI .. S_COUNT - 1) in one
// device-to-host copy.
sibfa_status read_virial_totals(sibfa_ctx c, double* out) {
  constexpr int nv = S_COUNT - S_VRI;
  if (!c->vir_tot) {
    if (!alloc_into(c, c->bufs, c->vir_tot, 48))
      return fail(c, SIBFA_E_NOMEM, "virial totals allocation failed");
  }
  if (!c->h_vir && hipHostMalloc((void**)&c->h_vir, 48 * sizeof(double), hipHostMallocDefault) !=
                       hipSuccess) {
    c->h_vir = nullptr;
    return fail(c, SIBFA_E_NOMEM, "virial host staging allocation failed");
  }
  for (int k0 = 0; k0 < nv; k0 += 8) {
    SlotList sl{};
    for (int k = k0; k < nv && k < k0 + 8; ++k) {
      sl.slot[sl.n] = S_VRI + k;
      sl.nparts[sl.n] = c->red.nparts[S_VRI + k];
      ++sl.n;
    }
    launch_slot_totals(c->red, sl, c->vir_tot + k0, c->stream);
  }
  HIP_TRY(hipMemcpyAsync(c->h_vir, c->vir_tot, nv * sizeof(double), hipMemcpyDeviceToHost,
                         c->stream));
  sibfa_status st = sync_read(c);
  if (st != SIBFA_OK) return st;
  for (int k = 0; k < nv; ++k) out[k] = c->h_vir[k];
  return SIBFA_OK;
}

sibfa_status sibfa_energy_forces(sibfa_ctx c, double* e_pol, double* e_elec, double* forces,
                                 double* virial) {
  if (!c) return SIBFA_E_ARG;
  HIP_TRY(hipSetDevice(c->device));
  sibfa_status st = prepare(c);
  if (st != SIBFA_OK) return st;
  if (!c->e0_valid && (st = compute_E0(c)) != SIBFA_OK) return st;
  if (!c->mu_valid && (st = solve(c, c->mu_have)) != SIBFA_OK) return st;
  // the virial comes out of the force kernels: forces into a scratch array
  // when the caller wants the virial only
  const bool want_vir = virial != nullptr;
  const bool frames_on = c->have_frames;
  if (want_vir && !forces) {
    if (!c->fvir && !alloc_into(c, c->bufs, c->fvir, 3 * (size_t)c->n))
      return fail(c, SIBFA_E_NOMEM, "force scratch allocation failed");
    forces = c->fvir;
  }
  SysView s = make_view(c);
  hipStream_t sm = c->stream;
  const bool mix = mixed(c);
  if (c->npol > 0) {
    // mu came from the last solve (mu_valid), whose x (polarizable order)
    // it is, and which ended on the FP64 true residual r = E - T x of
    // exactly these dipoles: x.T x = x.E - x.r gives the variational energy
    // (Eq. 17) without another matvec
    launch_dot(s, c->red, c->x, c->E0, S_MUE, sm, c->r, S_MUTMU);
  } else {
    launch_fill_double(reinterpret_cast<double*>(c->x), 0.0, 4, sm);
  }
  if (forces) {
    launch_mu_sites(s, c->x, c->mu_s, c->mu_s32, sm);
    if (c->periodic) {
      fork(c);
      Phase ph(c, SIBFA_PH_FORCE_RECIP, c->aux);
      launch_spread_mult(s, c->pm, c->mu_s, mix, c->aux);
      conv(c, mix, c->aux, S_EREC, want_vir);
    }
    {
      Phase ph(c, SIBFA_PH_FORCE_REAL);
      launch_force(s, c->red, c->mu_s, c->mu_s32, c->Freal, mix, want_vir, sm,
                   frames_on ? c->FS : nullptr, frames_on ? c->GS : nullptr);
    }
    if (c->periodic) {
      join(c);
      Phase ph(c, SIBFA_PH_FORCE_RECIP);
      launch_gather_force(s, c->pm, c->red, c->mu_s, c->Freal, c->perm, forces, mix, want_vir,
                          sm, frames_on ? c->FS : nullptr, frames_on ? c->GS : nullptr);
    } else {
      launch_forces_out(c->n, c->perm, c->Freal, forces, sm);
    }
    if (frames_on) {
      Phase ph(c, SIBFA_PH_FORCE_REAL);
      launch_frame_forces(make_frames(c), c->red, forces, want_vir, sm);
    }
  }
  if (want_vir) {
    // W = real-space pair terms + [E_rec of the combined density times the
    // identity - m-space sum + site terms]
    double v[S_COUNT - S_VRI];
    if ((st = read_virial_totals(c, v)) != SIBFA_OK) return st;
    double erec = 0.0;
    if (c->periodic && (st = read_totals(c, {S_EREC}, &erec)) != SIBFA_OK) return st;
    const double* vi = v;
    const double* vf = v + (S_VRF - S_VRI);
    const double* vk = v + (S_VRK - S_VRI);
    const double* vg = v + (S_VRG - S_VRI);
    const double* vr = v + (S_VRR - S_VRI);
    // m-space sum, symmetric: xx yy zz xy xz yz
    const int kidx[9] = {0, 3, 4, 3, 1, 5, 4, 5, 2};
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        const int k = 3 * a + b;
        double w = vi[k] + vf[k];
        if (c->periodic) w += (a == b ? erec : 0.0) - vk[kidx[k]] + vg[k];
        // the frame term is in kcal/mol already
        virial[k] = kCoulomb * w + (frames_on ? vr[k] : 0.0);
      }
  }
  double tot[6] = {0, 0, 0, 0, 0, 0};
  if (c->npol > 0)
    st = c->periodic ? read_totals(c, {S_EREAL, S_AUX, S_ESELF, S_EREC0, S_MUE, S_MUTMU}, tot)
                     : read_totals(c, {S_EREAL, S_AUX, S_MUE, S_MUTMU}, tot);
  else
    st = c->periodic ? read_totals(c, {S_EREAL, S_AUX, S_ESELF, S_EREC0}, tot)
                     : read_totals(c, {S_EREAL, S_AUX}, tot);
  if (st != SIBFA_OK) return st;
  c->e_real = tot[0] + tot[1];
  c->e_self = c->periodic ? tot[2] : 0.0;
  c->e_rec = c->periodic ? tot[3] : 0.0;
  const int mk = c->periodic ? 4 : 2;
  const double mue = c->npol > 0 ? tot[mk] : 0.0;
  const double mutmu = c->npol > 0 ? tot[mk] - tot[mk + 1] : 0.0;
  c->stats.e_pol = -0.5 * kCoulomb * mue;
  c->stats.e_pol_variational = kCoulomb * (0.5 * mutmu - mue);
  c->stats.e_elec_real = kCoulomb * c->e_real;
  c->stats.e_elec_recip = kCoulomb * c->e_rec;
  c->stats.e_elec_self = kCoulomb * c->e_self;
  c->stats.e_elec = c->stats.e_elec_real + c->stats.e_elec_recip + c->stats.e_elec_self;
  if (e_pol) *e_pol = c->stats.e_pol;
  if (e_elec) *e_elec = c->stats.e_elec;
  return SIBFA_OK;
}

// ------------------------------------------------------------ charge transfer
sibfa_status sibfa_set_charge_transfer(sibfa_ctx c, int n_lp, const int32_t* lp,
                                       const double* lp_par, int n_acc, const int32_t* acc,
                                       const double* acc_ah, const double* rvdw,
                                       const sibfa_ct_params* prm) {
  if (!c) return SIBFA_E_ARG;
  if (!c->have_sys) return fail(c, SIBFA_E_STATE, "sibfa_set_system has not been called");
  if (!c->have_mult || !c->have_pol)
    return fail(c, SIBFA_E_STATE, "multipoles and polarizabilities must be set first");
  if (n_lp < 0 || n_acc < 0 || (n_lp > 0 && (!lp || !lp_par)) || (n_acc > 0 && (!acc || !acc_ah)) ||
      !rvdw || !prm)
    return fail(c, SIBFA_E_ARG, "charge transfer: missing arrays or negative counts");
  const double pv[5] = {prm->eta, prm->cs, prm->cp, prm->t, prm->m};
  for (double v : pv)
    if (!std::isfinite(v)) return fail(c, SIBFA_E_ARG, "charge transfer: non-finite constants");
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (c->aux && c->aux != c->stream) HIP_TRY(hipStreamSynchronize(c->aux));
  const int n = c->n;
  const size_t nn = n;
  std::vector<int> hl(2 * (size_t)n_lp), ha(2 * (size_t)n_acc), hm(nn);
  std::vector<double> hlp(2 * (size_t)n_lp), hah(n_acc), hr(nn), hq(nn), hd(3 * nn), ht(6 * nn),
      hal(6 * nn);
  if (n_lp > 0) {
    HIP_TRY(hipMemcpy(hl.data(), lp, hl.size() * sizeof(int), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(hlp.data(), lp_par, hlp.size() * sizeof(double), hipMemcpyDeviceToHost));
  }
  if (n_acc > 0) {
    HIP_TRY(hipMemcpy(ha.data(), acc, ha.size() * sizeof(int), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(hah.data(), acc_ah, hah.size() * sizeof(double), hipMemcpyDeviceToHost));
  }
  HIP_TRY(hipMemcpy(hr.data(), rvdw, nn * sizeof(double), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(hm.data(), c->mol_c, nn * sizeof(int), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(hq.data(), c->q_c, nn * sizeof(double), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(hd.data(), c->dip_c, 3 * nn * sizeof(double), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(ht.data(), c->quad_c, 6 * nn * sizeof(double), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(hal.data(), c->alpha_c, 6 * nn * sizeof(double), hipMemcpyDeviceToHost));
  std::vector<double> hdl, hql, hall;   // local frames: the local values too
  if (c->have_frames) {
    hdl.resize(3 * nn);
    hql.resize(6 * nn);
    HIP_TRY(hipMemcpy(hdl.data(), c->dloc, 3 * nn * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(hql.data(), c->qloc, 6 * nn * sizeof(double), hipMemcpyDeviceToHost));
    if (c->rot_alpha) {
      hall.resize(6 * nn);
      HIP_TRY(hipMemcpy(hall.data(), c->aloc, 6 * nn * sizeof(double), hipMemcpyDeviceToHost));
    }
  }
  auto in = [&](int i) { return i >= 0 && i < n; };
  std::vector<int> lp_of(nn, -1);
  for (int p = 0; p < n_lp; ++p) {
    const int L = hl[2 * p], cr = hl[2 * p + 1];
    const std::string at = "lone pair " + std::to_string(p);
    if (!in(L) || !in(cr) || L == cr || hm[L] != hm[cr])
      return fail(c, SIBFA_E_ARG, at + ": site and carrier distinct, in range, one molecule");
    if (lp_of[L] >= 0) return fail(c, SIBFA_E_ARG, at + ": site listed twice");
    lp_of[L] = p;
    bool zero = hq[L] == 0.0;
    for (int k = 0; k < 3; ++k) zero = zero && hd[3 * (size_t)L + k] == 0.0;
    for (int k = 0; k < 6; ++k) zero = zero && ht[6 * (size_t)L + k] == 0.0 && hal[6 * (size_t)L + k] == 0.0;
    for (size_t k = 0; k < 3 && !hdl.empty(); ++k) zero = zero && hdl[3 * (size_t)L + k] == 0.0;
    for (size_t k = 0; k < 6 && !hql.empty(); ++k) zero = zero && hql[6 * (size_t)L + k] == 0.0;
    for (size_t k = 0; k < 6 && !hall.empty(); ++k) zero = zero && hall[6 * (size_t)L + k] == 0.0;
    if (!zero) return fail(c, SIBFA_E_ARG, at + ": a lone-pair site carries no multipoles or polarizability");
    if (!(hr[cr] > 0.0) || !std::isfinite(hr[cr]) || !std::isfinite(hlp[2 * p]) ||
        !std::isfinite(hlp[2 * p + 1]))
      return fail(c, SIBFA_E_ARG, at + ": finite parameters and a positive carrier radius");
  }
  for (int k = 0; k < n_acc; ++k) {
    const int a1 = ha[2 * k], a2 = ha[2 * k + 1];
    const std::string at = "acceptor " + std::to_string(k);
    if (!in(a1) || !in(a2) || a1 == a2 || hm[a1] != hm[a2])
      return fail(c, SIBFA_E_ARG, at + ": two distinct atoms of one molecule");
    if (!(hr[a1] > 0.0) || !(hr[a2] > 0.0) || !std::isfinite(hr[a1]) || !std::isfinite(hr[a2]) ||
        !std::isfinite(hah[k]))
      return fail(c, SIBFA_E_ARG, at + ": finite affinity and positive radii");
  }
  // site -> acceptors (as a1), lone pairs (as carrier), acceptor slots
  std::vector<int> a1s(nn + 1, 0), cars(nn + 1, 0), ats(nn + 1, 0);
  for (int k = 0; k < n_acc; ++k) { a1s[ha[2 * k] + 1]++; ats[ha[2 * k] + 1]++; ats[ha[2 * k + 1] + 1]++; }
  for (int p = 0; p < n_lp; ++p) cars[hl[2 * p + 1] + 1]++;
  for (int i = 0; i < n; ++i) { a1s[i + 1] += a1s[i]; cars[i + 1] += cars[i]; ats[i + 1] += ats[i]; }
  std::vector<int> a1r(std::max(a1s[n], 1)), carr(std::max(cars[n], 1)), atr(std::max(ats[n], 1));
  std::vector<int> vint;
  {
    std::vector<int> ca(a1s.begin(), a1s.end() - 1), cc(cars.begin(), cars.end() - 1),
        ct(ats.begin(), ats.end() - 1);
    for (int k = 0; k < n_acc; ++k) {
      a1r[ca[ha[2 * k]]++] = k;
      atr[ct[ha[2 * k]]++] = 2 * k;
      atr[ct[ha[2 * k + 1]]++] = 2 * k + 1;
    }
    for (int p = 0; p < n_lp; ++p) carr[cc[hl[2 * p + 1]]++] = p;
    for (int i = 0; i < n; ++i)
      if (ats[i + 1] > ats[i]) vint.push_back(i);
  }
  free_list(c, c->ctbufs);
  c->ct_on = false;
  auto& L = c->ctbufs;
  CtArgs& a = c->ct;
  a = CtArgs{};
  const size_t nl = std::max(n_lp, 1), na = std::max(n_acc, 1);
  int *dl, *da, *d_a1s, *d_a1r, *d_cs, *d_cr, *d_lpof, *d_ats, *d_atr, *d_vint;
  double *dlp, *dah, *dr;
  const bool ok =
      alloc_into(c, L, dl, 2 * nl) && alloc_into(c, L, dlp, 2 * nl) && alloc_into(c, L, da, 2 * na) &&
      alloc_into(c, L, dah, na) && alloc_into(c, L, dr, nn) && alloc_into(c, L, d_a1s, nn + 1) &&
      alloc_into(c, L, d_a1r, a1r.size()) && alloc_into(c, L, d_cs, nn + 1) &&
      alloc_into(c, L, d_cr, carr.size()) && alloc_into(c, L, d_lpof, nn) &&
      alloc_into(c, L, d_ats, nn + 1) && alloc_into(c, L, d_atr, atr.size()) &&
      alloc_into(c, L, d_vint, std::max<size_t>(vint.size(), 1)) &&
      alloc_into(c, L, a.Vlp, nl) && alloc_into(c, L, a.Gr, 3 * nl) && alloc_into(c, L, a.Vint, nn) &&
      alloc_into(c, L, a.w, nl) && alloc_into(c, L, a.Fl, 3 * nl) && alloc_into(c, L, a.Fc, 3 * nl) &&
      alloc_into(c, L, a.Fa, 6 * na) && alloc_into(c, L, a.ua, 2 * na) &&
      alloc_into(c, L, a.W_s, nn) && alloc_into(c, L, a.U_s, nn) && alloc_into(c, L, a.F_s, nn) &&
      alloc_into(c, L, a.flag_s, nn) && alloc_into(c, L, a.rng_s, nn) &&
      alloc_into(c, L, a.lp_rec, 8 * nl) && alloc_into(c, L, a.acc_rec, 8 * na) &&
      alloc_into(c, L, c->ct_spw, nn) && alloc_into(c, L, c->ct_zero4, nn) &&
      alloc_into(c, L, c->ct_zero2, nn);
  if (!ok) {
    free_list(c, c->ctbufs);
    return fail(c, SIBFA_E_NOMEM, "charge-transfer allocation failed");
  }
  auto up = [&](void* dst, const void* src, size_t bytes) {
    return bytes ? hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) : hipSuccess;
  };
  HIP_TRY(up(dl, hl.data(), hl.size() * sizeof(int)));
  HIP_TRY(up(dlp, hlp.data(), hlp.size() * sizeof(double)));
  HIP_TRY(up(da, ha.data(), ha.size() * sizeof(int)));
  HIP_TRY(up(dah, hah.data(), hah.size() * sizeof(double)));
  HIP_TRY(up(dr, hr.data(), nn * sizeof(double)));
  HIP_TRY(up(d_a1s, a1s.data(), a1s.size() * sizeof(int)));
  HIP_TRY(up(d_a1r, a1r.data(), a1r.size() * sizeof(int)));
  HIP_TRY(up(d_cs, cars.data(), cars.size() * sizeof(int)));
  HIP_TRY(up(d_cr, carr.data(), carr.size() * sizeof(int)));
  HIP_TRY(up(d_lpof, lp_of.data(), nn * sizeof(int)));
  HIP_TRY(up(d_ats, ats.data(), ats.size() * sizeof(int)));
  HIP_TRY(up(d_atr, atr.data(), atr.size() * sizeof(int)));
  HIP_TRY(up(d_vint, vint.data(), vint.size() * sizeof(int)));
  launch_fill_double(reinterpret_cast<double*>(c->ct_zero4), 0.0, 4 * nn, c->stream);
  launch_fill_double(reinterpret_cast<double*>(c->ct_zero2), 0.0, 2 * nn, c->stream);
  launch_fill_double(a.Vint, 0.0, nn, c->stream);
  launch_fill_double(a.Gr, 0.0, 3 * nl, c->stream);   // written only by the periodic gather
  a.n = n; a.n_lp = n_lp; a.n_acc = n_acc; a.n_vint = (int)vint.size();
  a.lp = dl; a.lp_par = dlp; a.acc = da; a.ah = dah; a.rvdw = dr;
  a.eta = prm->eta; a.cs = prm->cs; a.cp = prm->cp; a.t = prm->t; a.m = prm->m;
  a.a1_start = d_a1s; a.a1_ref = d_a1r; a.car_start = d_cs; a.car_ref = d_cr; a.lp_of = d_lpof;
  a.at_start = d_ats; a.at_ref = d_atr; a.vint_sites = d_vint;
  c->ct_on = true;
  return sync_read(c);
}

sibfa_status sibfa_ct_energy_forces(sibfa_ctx c, double* e_ct, double* forces) {
  if (!c) return SIBFA_E_ARG;
  if (!c->ct_on) return fail(c, SIBFA_E_STATE, "sibfa_set_charge_transfer has not been called");
  HIP_TRY(hipSetDevice(c->device));
  sibfa_status st = prepare(c);
  if (st != SIBFA_OK) return st;
  join(c);
  hipStream_t sm = c->stream;
  SysView s = make_view(c);
  CtArgs a = c->ct;
  a.perm = c->perm;
  a.inv_perm = c->inv_perm;
  launch_ct_potentials(s, a, sm);
  if (c->periodic && a.n_lp > 0) {
    launch_spread_mult(s, c->pm, nullptr, false, sm);
    conv(c, false, sm, S_CTREC);
    launch_ct_gather_pot(s, c->pm, a, sm);
  }
  launch_ct_pairs(s, a, c->red, sm);
  if (forces) {
    // local frames: the field and field gradient of the w and u charges at
    // the sites give the derivatives with respect to the rotated
    // multipoles, which the frame kernels turn into forces
    const bool fr = c->have_frames;
    double4* FS = fr ? c->FS : nullptr;
    double* GS = fr ? c->GS : nullptr;
    launch_ct_wforce(s, a, c->periodic ? c->ct_spw : nullptr, sm, FS, GS);
    if (c->periodic) {
      SysView sw = s;
      sw.sp = c->ct_spw;
      sw.sd = c->ct_zero4;
      sw.sth = c->ct_zero4;
      sw.sth2 = c->ct_zero2;
      launch_spread_mult(sw, c->pm, nullptr, false, sm);
      conv(c, false, sm, S_CTREC);
      // no self terms: the w charges sit at sites without multipoles
      launch_gather_force(s, c->pm, c->red, c->ct_zero4, a.F_s, c->perm, forces, false, false, sm,
                          FS, GS, false);
    } else {
      launch_forces_out(c->n, c->perm, a.F_s, forces, sm);
    }
    if (fr) {
      FrameArgs f = make_frames(c);
      f.aloc = nullptr;   // E_ct does not depend on the polarizabilities
      launch_frame_forces(f, c->red, forces, false, sm);
    }
  }
  double e = 0.0;
  if ((st = read_totals(c, {S_ECT}, &e)) != SIBFA_OK) return st;
  if (e_ct) *e_ct = e;
  return SIBFA_OK;
}

// ------------------------------------------------------------ dynamics
// Forces of the step on md_force: electrostatics and polarization, then
// the stand-in repulsion (over the lists the evaluation just built).
static sibfa_status md_forces(sibfa_ctx c, double* ep, double* ee) {
  sibfa_status r = sibfa_energy_forces(c, ep, ee, c->md_force, nullptr);
  if (r != SIBFA_OK) return r;
  if (c->md.rep_eps > 0.0)
    launch_md_repulsion(make_view(c), c->md, c->red, c->perm, c->stream);
  else
    c->red.nparts[S_EREP] = 0;
  return SIBFA_OK;
}

sibfa_status sibfa_md_init(sibfa_ctx c, const double* masses, const int32_t* vsites, int n_bonds,
                           const int32_t* bonds, const double* bond_k, const double* bond_r0,
                           const double* rep_radius, double rep_eps, const double* vel) {
  if (!c) return SIBFA_E_ARG;
  if (!c->have_sys) return fail(c, SIBFA_E_STATE, "sibfa_set_system has not been called");
  if (!masses) return fail(c, SIBFA_E_ARG, "masses is NULL");
  if (n_bonds < 0 || (n_bonds > 0 && (!bonds || !bond_k || !bond_r0)))
    return fail(c, SIBFA_E_ARG, "n_bonds >= 0 with bonds, bond_k and bond_r0");
  if (!(rep_eps >= 0.0) || !std::isfinite(rep_eps) || (rep_eps > 0.0 && !rep_radius))
    return fail(c, SIBFA_E_ARG, "rep_eps >= 0 finite, with rep_radius when positive");
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipStreamSynchronize(c->stream));
  const int n = c->n;
  const size_t nn = n;
  std::vector<double> hm(nn), hk(n_bonds), hr(n_bonds), hrho(nn, 0.0);
  std::vector<int> hv(2 * nn, -1), hb(2 * (size_t)n_bonds);
  HIP_TRY(hipMemcpy(hm.data(), masses, nn * sizeof(double), hipMemcpyDeviceToHost));
  if (vsites) HIP_TRY(hipMemcpy(hv.data(), vsites, 2 * nn * sizeof(int), hipMemcpyDeviceToHost));
  if (n_bonds > 0) {
    HIP_TRY(hipMemcpy(hb.data(), bonds, hb.size() * sizeof(int), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(hk.data(), bond_k, n_bonds * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(hr.data(), bond_r0, n_bonds * sizeof(double), hipMemcpyDeviceToHost));
  }
  if (rep_radius && rep_eps > 0.0)
    HIP_TRY(hipMemcpy(hrho.data(), rep_radius, nn * sizeof(double), hipMemcpyDeviceToHost));
  for (int i = 0; i < n; ++i)
    if (!(hrho[i] >= 0.0) || !std::isfinite(hrho[i]))
      return fail(c, SIBFA_E_ARG, "repulsion radii must be finite and >= 0");
  auto atom = [&](int i) { return i >= 0 && i < n && hm[i] > 0.0; };
  for (int i = 0; i < n; ++i) {
    if (!(hm[i] >= 0.0) || !std::isfinite(hm[i]))
      return fail(c, SIBFA_E_ARG, "masses must be finite and >= 0");
    const int p = hv[2 * i], q = hv[2 * i + 1];
    if (p < 0 && q < 0) {
      if (!(hm[i] > 0.0))
        return fail(c, SIBFA_E_ARG, "site " + std::to_string(i) + ": a massless site must be a virtual site");
    } else if (hm[i] != 0.0 || !atom(p) || !atom(q) || p == q) {
      return fail(c, SIBFA_E_ARG, "site " + std::to_string(i) +
                                      ": a virtual site is massless with two distinct atoms as parents");
    }
  }
  for (int b = 0; b < n_bonds; ++b) {
    const int i = hb[2 * b], j = hb[2 * b + 1];
    if (!atom(i) || !atom(j) || i == j || !(hk[b] >= 0.0) || !std::isfinite(hk[b]) ||
        !(hr[b] > 0.0) || !std::isfinite(hr[b]))
      return fail(c, SIBFA_E_ARG, "bond " + std::to_string(b) +
                                      ": two distinct atoms, k >= 0 and r0 > 0 finite");
  }
  // atom -> virtual sites and atom -> bonds, both in increasing order
  std::vector<int> vstart(nn + 1, 0), bstart(nn + 1, 0);
  for (int i = 0; i < n; ++i)
    if (hv[2 * i] >= 0) { vstart[hv[2 * i] + 1]++; vstart[hv[2 * i + 1] + 1]++; }
  for (int b = 0; b < n_bonds; ++b) { bstart[hb[2 * b] + 1]++; bstart[hb[2 * b + 1] + 1]++; }
  for (int i = 0; i < n; ++i) { vstart[i + 1] += vstart[i]; bstart[i + 1] += bstart[i]; }
  std::vector<int> vref(std::max(vstart[n], 1)), bref(std::max(bstart[n], 1));
  {
    std::vector<int> cv(vstart.begin(), vstart.end() - 1), cb(bstart.begin(), bstart.end() - 1);
    for (int i = 0; i < n; ++i)
      if (hv[2 * i] >= 0) { vref[cv[hv[2 * i]]++] = i; vref[cv[hv[2 * i + 1]]++] = i; }
    for (int b = 0; b < n_bonds; ++b) { bref[cb[hb[2 * b]]++] = b; bref[cb[hb[2 * b + 1]]++] = b; }
  }
  free_list(c, c->mdbufs);
  c->md_on = false;
  auto& L = c->mdbufs;
  const size_t nbk = std::max(n_bonds, 1);
  double *mass, *bk, *br0, *rho;
  int *vpar, *vs, *vr, *bd, *bs, *br;
  const bool ok = alloc_into(c, L, mass, nn) && alloc_into(c, L, vpar, 2 * nn) &&
                  alloc_into(c, L, rho, nn) &&
                  alloc_into(c, L, vs, nn + 1) && alloc_into(c, L, vr, vref.size()) &&
                  alloc_into(c, L, bd, 2 * nbk) && alloc_into(c, L, bk, nbk) &&
                  alloc_into(c, L, br0, nbk) && alloc_into(c, L, bs, nn + 1) &&
                  alloc_into(c, L, br, bref.size()) && alloc_into(c, L, c->md.vel, 3 * nn) &&
                  alloc_into(c, L, c->md.acc, 3 * nn) && alloc_into(c, L, c->md.accp, 3 * nn) &&
                  alloc_into(c, L, c->md_force, 3 * nn);
  if (!ok) {
    free_list(c, c->mdbufs);
    return fail(c, SIBFA_E_NOMEM, "dynamics allocation failed");
  }
  hipStream_t st = c->stream;
  HIP_TRY(hipMemcpy(mass, hm.data(), nn * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(rho, hrho.data(), nn * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(vpar, hv.data(), 2 * nn * sizeof(int), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(vs, vstart.data(), vstart.size() * sizeof(int), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(vr, vref.data(), vref.size() * sizeof(int), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(bs, bstart.data(), bstart.size() * sizeof(int), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(br, bref.data(), bref.size() * sizeof(int), hipMemcpyHostToDevice));
  if (n_bonds > 0) {
    HIP_TRY(hipMemcpy(bd, hb.data(), hb.size() * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(bk, hk.data(), n_bonds * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(br0, hr.data(), n_bonds * sizeof(double), hipMemcpyHostToDevice));
  }
  if (vel) HIP_TRY(hipMemcpyAsync(c->md.vel, vel, 3 * nn * sizeof(double), hipMemcpyDeviceToDevice, st));
  else launch_fill_double(c->md.vel, 0.0, 3 * nn, st);
  MdArgs& m = c->md;
  m.n = n;
  m.periodic = c->periodic;
  for (int a = 0; a < 3; ++a) {
    m.box[a] = c->periodic ? c->box[a] : 1.0;
    m.ibox[a] = c->periodic ? 1.0 / c->box[a] : 1.0;
  }
  m.xyz = c->xyz_c;
  m.force = c->md_force;
  m.mass = mass; m.vpar = vpar; m.vstart = vs; m.vref = vr;
  m.bonds = bd; m.bond_k = bk; m.bond_r0 = br0; m.bstart = bs; m.bref = br;
  m.rep_rho = rho;
  m.rep_eps = rep_eps;
  m.rep_force = c->md_force;
  if (vel) {
    sibfa_status fs = finite_check(c, c->md.vel, 3 * nn, "vel");
    if (fs != SIBFA_OK) { free_list(c, c->mdbufs); return fs; }
  }
  // virtual sites onto their midpoints, forces and accelerations at t = 0
  launch_md_vsites(m, st);
  c->dirty_sort = true;
  c->dirty_rot = c->have_frames;
  c->e0_valid = c->mu_valid = false;
  sibfa_status r = md_forces(c, nullptr, nullptr);
  if (r != SIBFA_OK) { free_list(c, c->mdbufs); return r; }
  launch_md_finish(m, c->red, 0.0, 0.0, st);
  r = sync_read(c);
  if (r != SIBFA_OK) { free_list(c, c->mdbufs); return r; }
  c->md_on = true;
  return SIBFA_OK;
}

sibfa_status sibfa_md_run(sibfa_ctx c, int n_steps, double dt_fs, double friction,
                          sibfa_md_stats* stats) {
  if (!c) return SIBFA_E_ARG;
  if (!c->md_on) return fail(c, SIBFA_E_STATE, "sibfa_md_init has not been called");
  if (n_steps < 0 || !(dt_fs > 0.0) || !std::isfinite(dt_fs))
    return fail(c, SIBFA_E_ARG, "n_steps >= 0 and a positive finite dt_fs");
  if (!(friction >= 0.0 && friction <= 1.0))
    return fail(c, SIBFA_E_ARG, "friction must lie in [0, 1]");
  HIP_TRY(hipSetDevice(c->device));
  for (int k = 0; k < n_steps; ++k) {
    launch_md_positions(c->md, dt_fs, c->stream);
    c->dirty_sort = true;
    c->dirty_rot = c->have_frames;
    c->e0_valid = c->mu_valid = false;
    double ep = 0.0, ee = 0.0;
    sibfa_status r = md_forces(c, &ep, &ee);
    if (r != SIBFA_OK) return r;
    launch_md_finish(c->md, c->red, dt_fs, friction, c->stream);
    double kb[3] = {0.0, 0.0, 0.0};
    if ((r = read_totals(c, {S_EKIN, S_EBOND, S_EREP}, kb)) != SIBFA_OK) return r;
    if (stats) {
      stats[k].e_pol = ep;
      stats[k].e_elec = ee;
      stats[k].e_kin = kb[0];
      stats[k].e_bond = kb[1];
      stats[k].e_rep = kb[2];
      stats[k].iterations = c->stats.iterations;
    }
  }
  return SIBFA_OK;
}

sibfa_status sibfa_md_get_state(sibfa_ctx c, double* xyz, double* vel) {
  if (!c) return SIBFA_E_ARG;
  if (!c->md_on) return fail(c, SIBFA_E_STATE, "sibfa_md_init has not been called");
  HIP_TRY(hipSetDevice(c->device));
  const size_t bytes = 3 * (size_t)c->n * sizeof(double);
  if (xyz) HIP_TRY(hipMemcpyAsync(xyz, c->xyz_c, bytes, hipMemcpyDeviceToDevice, c->stream));
  if (vel) HIP_TRY(hipMemcpyAsync(vel, c->md.vel, bytes, hipMemcpyDeviceToDevice, c->stream));
  return sync_read(c);
}

sibfa_status sibfa_get_dipoles(sibfa_ctx c, double* mu) {
  if (!c) return SIBFA_E_ARG;
  if (!mu) return fail(c, SIBFA_E_ARG, "mu is NULL");
  if (!c->mu_have) return fail(c, SIBFA_E_STATE, "no induced dipoles yet");
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipMemcpyAsync(mu, c->mu_c, 3 * (size_t)c->n * sizeof(double), hipMemcpyDeviceToDevice,
                         c->stream));
  return sync_read(c);
}

sibfa_status sibfa_set_dipoles(sibfa_ctx c, const double* mu) {
  if (!c) return SIBFA_E_ARG;
  if (!mu) return fail(c, SIBFA_E_ARG, "mu is NULL");
  if (!c->have_sys) return fail(c, SIBFA_E_STATE, "sibfa_set_system has not been called");
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipMemcpyAsync(c->mu_c, mu, 3 * (size_t)c->n * sizeof(double), hipMemcpyDeviceToDevice,
                         c->stream));
  sibfa_status st = finite_check(c, c->mu_c, 3 * (size_t)c->n, "mu");
  if (st != SIBFA_OK) return st;
  c->mu_have = true;
  c->mu_valid = false;
  push_history(c, c->stream);
  return SIBFA_OK;
}

static_assert(kPredMax == SIBFA_PREDICT_MAX_ORDER, "predictor history length");

sibfa_status sibfa_set_predictor(sibfa_ctx c, int order) {
  if (!c) return SIBFA_E_ARG;
  if (order < 0 || order > kPredMax)
    return fail(c, SIBFA_E_ARG, "order must lie in 0.." + std::to_string(kPredMax));
  c->pred_order = order;
  c->hist_count = 0;   // the history starts with the next dipoles
  c->hist_head = 0;
  return SIBFA_OK;
}

sibfa_status sibfa_neighbor_counts(sibfa_ctx c, int32_t* counts_out) {
  if (!c) return SIBFA_E_ARG;
  if (!counts_out) return fail(c, SIBFA_E_ARG, "counts_out is NULL");
  HIP_TRY(hipSetDevice(c->device));
  sibfa_status st = prepare(c);
  if (st != SIBFA_OK) return st;
  launch_counts_out(c->n, c->perm, c->ncnt[0], counts_out, c->stream);
  return sync_read(c);
}

sibfa_status sibfa_set_profiling_phases(sibfa_ctx c, unsigned phase_mask) {
  if (!c) return SIBFA_E_ARG;
  sibfa_status st = sibfa_set_profiling(c, phase_mask != 0);
  c->prof_mask = phase_mask;
  return st;
}

sibfa_status sibfa_set_profiling(sibfa_ctx c, int enable) {
  if (!c) return SIBFA_E_ARG;
  HIP_TRY(hipSetDevice(c->device));
  fold_marks(c);
  c->prof = enable != 0;
  c->prof_mask = ~0u;
  for (int k = 0; k < 16; ++k) {
    c->prof_ms[k] = 0.0;
    c->prof_calls[k] = 0;
  }
  return SIBFA_OK;
}

sibfa_status sibfa_get_profile(sibfa_ctx c, sibfa_profile* out) {
  if (!c || !out) return SIBFA_E_ARG;
  HIP_TRY(hipSetDevice(c->device));
  fold_marks(c);
  for (int k = 0; k < 16; ++k) {
    out->ms[k] = c->prof_ms[k];
    out->calls[k] = c->prof_calls[k];
  }
  if (!c->totals_valid && c->nb[0]) {
    launch_fill_int(reinterpret_cast<int*>(c->dsums), 0, 8, c->stream);
    const int rows[4] = {c->n, c->n, c->npol, c->npol};
    for (int k = 0; k < 4; ++k)
      if (rows[k] > 0) launch_sum_ints(c->ncnt[k], rows[k], c->dsums + k, c->stream);
    HIP_TRY(hipMemcpyAsync(c->h_pinned + 32, c->dsums, 4 * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, c->stream));
    sibfa_status s3 = sync_read(c);
    if (s3 != SIBFA_OK) return s3;
    for (int k = 0; k < 4; ++k)
      c->pair_totals[k] = (long long)reinterpret_cast<unsigned long long*>(c->h_pinned + 32)[k];
    c->totals_valid = true;
  }
  for (int k = 0; k < 4; ++k) out->pairs[k] = c->pair_totals[k];
  return SIBFA_OK;
}

sibfa_status sibfa_get_stats(sibfa_ctx c, sibfa_stats* out) {
  if (!c || !out) return SIBFA_E_ARG;
  *out = c->stats;
  return SIBFA_OK;
}

}  // extern "C"
