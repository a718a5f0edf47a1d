// C ABI of libaao.so (declared in include/aao.h): plans, workspace, the
// per-alpha host tables, the sweep (rows a1-a4), Alg. 2 (row a5), the
// transposed sweep and the gradients.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "aao.h"
#include "aao_noalloc.hpp"
#include "aao_host.hpp"
#include "aao_kernels.hpp"

using aao::cd;

namespace {

thread_local std::string g_err;

aao_status fail(aao_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(AAO_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));         \
  } while (0)

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// Bluestein length of a transform of n points: 0 if n is a power of two, else
// the smallest power of two >= 2n - 1.
int64_t blue_len(int64_t n) {
  if (is_pow2(n)) return 0;
  int64_t P = 1;
  while (P < 2 * n - 1) P <<= 1;
  return P;
}

// Points of one transform line held in LDS.
int64_t fft_line(int64_t n) { return is_pow2(n) ? n : blue_len(n); }

// Largest divisor of n that is at most cap (at least 1).
int largest_divisor(int n, int cap) {
  for (int d = std::max(1, std::min(n, cap)); d > 1; --d)
    if (n % d == 0) return d;
  return 1;
}

int ilog2(int64_t v) {
  int l = 0;
  while ((int64_t(1) << l) < v) ++l;
  return l;
}

// COCG tile shape in 2D (points per workgroup TX x TY).
#ifndef AAO_CG_TX2D
#define AAO_CG_TX2D 64
#endif
#ifndef AAO_CG_TY2D
#define AAO_CG_TY2D 16
#endif
// small COCG tiles once few systems remain: used when (active systems) x
// (large-tile count) is at most this many workgroups (0: never)
#ifndef AAO_CG_SMALL_WG
#define AAO_CG_SMALL_WG 256
#endif
#ifndef AAO_XCD_BANDS
#define AAO_XCD_BANDS 1
#endif
// Active-system checks of the COCG passes: every AAO_CG_CHECK_EARLY passes up
// to pass AAO_CG_CHECK_SWITCH, then every AAO_CG_CHECK_LATE, and every
// AAO_CG_CHECK_SMALL once the small tiles are in use.  A check reads the
// snapshot the previous one requested, so passes launched after the last
// system stopped run (exiting at once) until the second check after it:
// short intervals save those launches, but an interval of one pass makes the
// host wait on the pass it has just queued and the queue drains.
#ifndef AAO_CG_CHECK_EARLY
#define AAO_CG_CHECK_EARLY 2
#endif
#ifndef AAO_CG_CHECK_SWITCH
#define AAO_CG_CHECK_SWITCH 16
#endif
#ifndef AAO_CG_CHECK_LATE
#define AAO_CG_CHECK_LATE 4
#endif
#ifndef AAO_CG_CHECK_SMALL
#define AAO_CG_CHECK_SMALL 2
#endif
// The same for the chunked BiCGStab (three launches per iteration): every
// AAO_BICG_CHECK_EARLY iterations up to iteration AAO_CG_CHECK_SWITCH, then
// every AAO_BICG_CHECK_LATE.
#ifndef AAO_BICG_CHECK_EARLY
#define AAO_BICG_CHECK_EARLY 2
#endif
#ifndef AAO_BICG_CHECK_LATE
#define AAO_BICG_CHECK_LATE 4
#endif
// LDS budgets (KiB) of the transform over l and of the spatial FFT passes.
#ifndef AAO_XFORM_LDS_KB
#define AAO_XFORM_LDS_KB 24
#endif
// LDS budgets of the FFT inner solve's tiles (row lines; column tiles: a
// full 128-byte segment per row within the smaller budget, else at least 64
// bytes within the larger one)
#ifndef AAO_FFT_ROW_LDS_KB
#define AAO_FFT_ROW_LDS_KB 20
#endif
#ifndef AAO_FFT_COL_LDS_SMALL_KB
#define AAO_FFT_COL_LDS_SMALL_KB 40
#endif
#ifndef AAO_FFT_COL_LDS_KB
#define AAO_FFT_COL_LDS_KB 72
#endif

constexpr int kWorkSlots = 32;     // [class] for k > 0, [16 + class] for k == 0
constexpr int kCheckEvery = 8;     // Krylov iterations between host convergence checks
constexpr int kNormBlocks = 256;

struct Timed {
  int cls;
  hipEvent_t a, b;
};

}  // namespace

struct aao_plan {
  // problem
  int ndim = 1, nx = 0, ny = 1, N = 0, M = 0, L = 0, logL = 0, Lh = 0, B = 1;
  int precision = AAO_FP64, inner = AAO_INNER_COCG, inner_maxit = 1000;
  double dt = 0, inner_tol = 1e-12;
  // absolute floor of the inner stop inside aao_solve / windows / adjoint:
  // tau_w (< 0: the default of floor_tau), the stop tolerance of the current
  // solve and whether the current call uses the floor
  double floor_tol = -1;
  double solve_tol = 0;
  double floor_div = 1;  // tightening of the floor within the current solve
  bool floor_on = false;
  // per instance ||u0_b||_2^2 (primal, [0]) and ||g_b||_2^2 (adjoint, [1])
  std::vector<double> n2[2];
  std::vector<double> t, Q, QT;
  aao::Taps taps{}, tapsT{}, dtaps{};
  bool has_dnu = false, symmetric = false;
  double Anorm_inf = 0;
  hipStream_t stream = nullptr;
  // transforms over l
  int TN = 2, logTN = 1, ntiles = 0;
  // inner solves
  int S = 0, wps = 1, chunk = 256, nvec = 0;
  int wps_max = 1;  // BiCGStab: most workgroups per system (partial-sum stride)
  int cgTX = 1, cgTY = 1, cg_ntx = 1, cg_nty = 1, cg_ntiles = 1, Rx = 0, Ry = 0;
  int cgTXs = 0, cgTYs = 0, cg_ntxs = 0, cg_ntiles_s = 0;  // small tiling (cg_ntiles_s = 0: none)
  int fft_rows = 1, fft_cols = 1;
  bool bicg_tiled = false;  // BiCGStab phases 1 and 2 on the COCG tiles
  int Px = 0, Py = 0;  // Bluestein lengths of x / y for the FFT inner solve (0: power of two)
  int* hlist = nullptr;      // pinned: (count, tag) of the active-system snapshots, per slot; from
                             // byte 64 the end-of-sweep report (k_sweep_report)
  int rep_tag = 0;           // tag of the latest end-of-sweep report
  int snap_tag = 0;          // tag of the latest snapshot
  bool f32 = false;
  size_t csize = 16;
  // library-owned device tables and pinned staging
  char* dtab = nullptr;
  size_t off_tw = 0, off_sf = 0, off_sb = 0, off_m1 = 0, off_m2 = 0, off_sh = 0, off_q = 0,
         off_wx = 0, off_wy = 0, off_bx = 0, off_by = 0, off_bf = 0, off_hostend = 0, tab_bytes = 0;
  char* htab = nullptr;      // pinned mirror of the alpha-dependent tables (two slots)
  char* hread = nullptr;     // pinned readback area
  size_t hread_bytes = 0;
  // two slots of alpha-dependent tables: the sweep in flight reads one while
  // the next sweep's tables are built and uploaded into the other
  size_t atab_stride = 0;  // bytes of one slot (sf .. sh)
  int cur_slot = 0;
  double slot_alpha[2] = {-1, -1};
  int slot_adj[2] = {-1, -1};
  double slot_tw[2] = {-1, -1};  // tau_w the slot's inner floors were built with
  hipEvent_t slot_ev[2] = {nullptr, nullptr};  // recorded after each slot's upload
  // caller workspace
  char* ws = nullptr;
  size_t ws_bytes = 0, ws_need = 0;
  size_t off_vec = 0, off_part = 0, off_st = 0, off_fb = 0, off_norms = 0, off_cnt = 0,
         off_work = 0, off_gpart = 0, off_npart = 0, off_list = 0, off_win = 0;
  int fb_slots = 0, grad_blocks = 0;
  // state
  const double* u0 = nullptr;
  const double* frc = nullptr;  // source at the collocation times [B][L][M][N] (caller-owned)
  double w2 = 0, winf = 0;
  // stats
  bool timing = false;
  aao_kernel_stats stats{};
  std::vector<Timed> pending;
  std::vector<hipEvent_t> pool;
  int run_cls = -1;            // class of the open timing run (-1: none)
  hipEvent_t run_a = nullptr;  // its start event
  // elements processed per kernel class (first iteration / later iterations),
  // from the per-system iteration counts read back after each inner solve
  double work_first[AAO_NUM_KERNELS] = {}, work_later[AAO_NUM_KERNELS] = {};
  double bytes_direct[AAO_NUM_KERNELS] = {};  // algorithmic bytes counted directly (outer GMRES, fused COCG)
  double elems_direct[AAO_NUM_KERNELS] = {};
  double* hgm = nullptr;                      // pinned: GMRES partial sums down, coefficients up
  size_t hgm_bytes = 0;

  void* vec(int i) const { return ws + off_vec + (size_t)i * S * N * csize; }
  double* part() const { return reinterpret_cast<double*>(ws + off_part); }
  aao::SysState* st() const { return reinterpret_cast<aao::SysState*>(ws + off_st); }
  double* fb() const { return reinterpret_cast<double*>(ws + off_fb); }
  double* norms() const { return reinterpret_cast<double*>(ws + off_norms); }
  int* cnt() const { return reinterpret_cast<int*>(ws + off_cnt); }
  unsigned long long* work() const { return reinterpret_cast<unsigned long long*>(ws + off_work); }
  double* gpart() const { return reinterpret_cast<double*>(ws + off_gpart); }
  double* npart() const { return reinterpret_cast<double*>(ws + off_npart); }
  double* win() const { return reinterpret_cast<double*>(ws + off_win); }  // [B][N] window initial value
  int* dlist(int i = 2) const { return reinterpret_cast<int*>(ws + off_list) + (size_t)i * S; }
  double2* d_tw() const { return reinterpret_cast<double2*>(dtab + off_tw); }
  double* d_sf() const { return reinterpret_cast<double*>(dtab + off_sf + (size_t)cur_slot * atab_stride); }
  double* d_sb() const { return reinterpret_cast<double*>(dtab + off_sb + (size_t)cur_slot * atab_stride); }
  double2* d_m1() const { return reinterpret_cast<double2*>(dtab + off_m1 + (size_t)cur_slot * atab_stride); }
  double2* d_m2() const { return reinterpret_cast<double2*>(dtab + off_m2 + (size_t)cur_slot * atab_stride); }
  double2* d_sh() const { return reinterpret_cast<double2*>(dtab + off_sh + (size_t)cur_slot * atab_stride); }
  double* d_bf() const { return reinterpret_cast<double*>(dtab + off_bf + (size_t)cur_slot * atab_stride); }
  double* d_q() const { return reinterpret_cast<double*>(dtab + off_q); }
  double2* d_wx() const { return reinterpret_cast<double2*>(dtab + off_wx); }
  double2* d_wy() const { return reinterpret_cast<double2*>(dtab + off_wy); }
};

namespace {

// ------------------------------------------------------------------ timing
hipEvent_t get_event(aao_plan* p) {
  if (!p->pool.empty()) {
    hipEvent_t e = p->pool.back();
    p->pool.pop_back();
    return e;
  }
  // timing only (elapsed times are read after a stream synchronisation): no
  // system-scope fence, so recording does not write back and invalidate caches
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

// Timing brackets runs of consecutive launches of one kernel class with one
// pair of events (fewer event packets between kernels than one pair per
// launch); any other work enqueued on the stream first closes the open run.
void close_run(aao_plan* p) {
  if (p->run_cls < 0) return;
  hipEvent_t b = get_event(p);
  if (b) {
    (void)hipEventRecord(b, p->stream);
    p->pending.push_back({p->run_cls, p->run_a, b});
  } else {
    p->pool.push_back(p->run_a);
  }
  p->run_cls = -1;
  p->run_a = nullptr;
}

template <typename F>
hipError_t timed(aao_plan* p, int cls, F&& launch) {
  p->stats.launches[cls] += 1;
  if (!p->timing) return launch();
  if (p->run_cls != cls) {
    close_run(p);
    hipEvent_t a = get_event(p);
    if (!a) return launch();
    (void)hipEventRecord(a, p->stream);
    p->run_cls = cls;
    p->run_a = a;
  }
  return launch();
}

// Call after the stream has been synchronised.
void collect_timing(aao_plan* p) {
  for (auto& t : p->pending) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) p->stats.ms[t.cls] += ms;
    p->pool.push_back(t.a);
    p->pool.push_back(t.b);
  }
  p->pending.clear();
}

// ------------------------------------------------------------------ tables
// alpha-dependent tables for the primal (adj = 0) or transposed (adj = 1)
// sweep: scale before/after the DFT over l, the node transforms of each
// frequency and the shifts dT d_jm of the inner systems.
// Build the tables of alpha into slot `slot` (host, pinned) and enqueue their
// upload into the same device slot.  The host copy of a slot is rewritten
// only after the stream has been synchronised since its last upload.
// tau_w of the absolute inner floor: the caller's (aao_set_inner_floor), else
// min(tau, tol / 100) with tol the stop tolerance of the current solve (the
// error the floor leaves behind stays two decades under the stop rule).
double floor_tau(const aao_plan* p) {
  if (p->floor_tol >= 0) return p->floor_tol / p->floor_div;
  return std::min(p->inner_tol, 0.01 * p->solve_tol) / p->floor_div;
}

aao_status build_tables(aao_plan* p, double alpha, int adj, int slot) {
  if (!(alpha > 0.0 && alpha < 1.0))
    return fail(AAO_EINVAL, "alpha must lie in (0, 1), got " + std::to_string(alpha));
  const int M = p->M, L = p->L, Lh = p->Lh;
  if (!p->slot_ev[slot]) HIPCHK(hipEventCreateWithFlags(&p->slot_ev[slot], hipEventDisableTiming));
  else HIPCHK(hipEventSynchronize(p->slot_ev[slot]));  // the slot's previous upload has been read
  char* h = p->htab + (size_t)slot * p->atab_stride;
  double* sf = reinterpret_cast<double*>(h + (p->off_sf - p->off_sf));
  double* sb = reinterpret_cast<double*>(h + (p->off_sb - p->off_sf));
  cd* m1 = reinterpret_cast<cd*>(h + (p->off_m1 - p->off_sf));
  cd* m2 = reinterpret_cast<cd*>(h + (p->off_m2 - p->off_sf));
  cd* sh = reinterpret_cast<cd*>(h + (p->off_sh - p->off_sf));
  double* bf = reinterpret_cast<double*>(h + (p->off_bf - p->off_sf));
  const double tw_used = p->floor_on ? floor_tau(p) : 0.0;
  p->slot_alpha[slot] = -1;
  // Lemma 1: J^{-1} = diag(alpha^{(l-1)/L}) before the DFT, J and the 1/L of the
  // inverse DFT after it.  Transposed (V^T = (1/L) F J, V^{-T} = J^{-1} F^*):
  // J and 1/L before an inverse DFT, J^{-1} after a forward DFT.
  for (int l = 0; l < L; ++l) {
    const double up = std::pow(alpha, (double)l / L);
    const double dn = std::pow(alpha, -(double)l / L);
    sf[l] = adj ? dn / L : up;
    sb[l] = adj ? up : dn / L;
  }
  for (int j = 0; j < Lh; ++j) {
    aao::FreqTable ft;
    std::string why = aao::freq_table(p->t, p->Q, alpha, L, j, ft);
    if (!why.empty())
      return fail(AAO_ENODIAG, "alpha=" + std::to_string(alpha) + ", frequency " + std::to_string(j) +
                                   ": " + why);
    cd* A1 = m1 + (size_t)j * M * M;
    cd* A2 = m2 + (size_t)j * M * M;
    for (int m = 0; m < M; ++m)
      for (int k = 0; k < M; ++k) {
        if (!adj) {
          // x1 = S^{-1} x (eq. (innerdiag)); y = G^{-1} S x2 with G^{-1} = I - r H_M (eq. (QGL))
          A1[m * M + k] = ft.Sinv[m * M + k];
          A2[m * M + k] = ft.S[m * M + k] - ft.r * ft.S[(M - 1) * M + k];
        } else {
          // transposed: x1 = S^T G^{-T} x, (G^{-T})[i][k] = delta_ik - r delta_{i,M-1}
          // (G^{-T} = I - r H_M^T), so (S^T G^{-T})[m][k] = S[k][m] - r S[M-1][m];
          // y = S^{-T} x2
          A1[m * M + k] = ft.S[k * M + m] - ft.r * ft.S[(M - 1) * M + m];
          A2[m * M + k] = ft.Sinv[k * M + m];
        }
      }
    for (int b = 0; b < p->B; ++b)
      for (int m = 0; m < M; ++m) sh[((size_t)b * Lh + j) * M + m] = p->dt * ft.lam[m];
    // Absolute floor of the inner stop: the paper's right-hand-side form of
    // eq. (Riteration) hands each shifted system the transform of w + (C_alpha
    // - C) u^k, which is w-sized, and stops it at tau relative to that; in the
    // defect-correction form the right-hand side is the residual instead, and
    // the same absolute accuracy is tau_w times the norm of the transform of
    // w.  Without a source, w is 1_M (x) u0 in step 1 only (g_last at the last
    // node of step L for the adjoint), so frequency j holds it unchanged (times
    // the scaling of that step) and system (j, m) gets row m of the node
    // transform applied to it.  With a source only the u0 part is counted (a
    // smaller floor: the inner solves are then at least as accurate).
    const double tw = tw_used;
    const std::vector<double>& n2 = p->n2[adj];
    for (int m = 0; m < M; ++m) {
      double g2 = 0;
      if (!adj) {
        cd s = 0;
        for (int k = 0; k < M; ++k) s += A1[m * M + k];
        g2 = std::norm(s);
      } else {
        g2 = std::norm(A1[m * M + (M - 1)]) * sf[L - 1] * sf[L - 1];
      }
      const double ratio = tw > 0 ? tw / p->inner_tol : 0.0;
      for (int b = 0; b < p->B; ++b)
        bf[((size_t)b * Lh + j) * M + m] = ((size_t)b < n2.size()) ? ratio * ratio * g2 * n2[b] : 0.0;
    }
  }
  close_run(p);
  HIPCHK(hipMemcpyAsync(p->dtab + p->off_sf + (size_t)slot * p->atab_stride, h, p->atab_stride,
                        hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipEventRecord(p->slot_ev[slot], p->stream));
  p->slot_alpha[slot] = alpha;
  p->slot_adj[slot] = adj;
  p->slot_tw[slot] = tw_used;
  return AAO_OK;
}

int slot_of(const aao_plan* p, double alpha, int adj) {
  for (int i = 0; i < 2; ++i)
    if (p->slot_alpha[i] == alpha && p->slot_adj[i] == adj && p->slot_tw[i] == (p->floor_on ? floor_tau(p) : 0.0))
      return i;
  return -1;
}

// Make the tables of alpha current (built into the other slot if neither
// holds them).
aao_status upload_tables(aao_plan* p, double alpha, int adj) {
  int i = slot_of(p, alpha, adj);
  if (i < 0) {
    i = p->cur_slot ^ 1;
    aao_status s = build_tables(p, alpha, adj, i);
    if (s != AAO_OK) return s;
  }
  p->cur_slot = i;
  return AAO_OK;
}

// Build the tables of the next sweep's alpha into the idle slot while the
// current sweep runs (failures are left to the sweep that needs them).
void prefetch_tables(aao_plan* p, double alpha, int adj) {
  if (!(alpha > 0.0 && alpha < 1.0) || slot_of(p, alpha, adj) >= 0) return;
  const std::string keep = g_err;
  if (build_tables(p, alpha, adj, p->cur_slot ^ 1) != AAO_OK) g_err = keep;
}

aao::FwdArgs fwd_args(aao_plan* p, const double* in, int adj) {
  aao::FwdArgs a{};
  a.u = in;
  a.w0 = p->u0;
  a.frc = adj ? nullptr : p->frc;
  a.out = p->vec(1);  // the Krylov right-hand side / residual buffer R
  a.scale = p->d_sf();
  a.tw = p->d_tw();
  a.mix = p->d_m1();
  a.part = p->fb();
  a.g = {p->nx, p->ny, p->N};
  a.taps = adj ? p->tapsT : p->taps;
  const std::vector<double>& q = adj ? p->QT : p->Q;
  for (int i = 0; i < p->M * p->M; ++i) a.q[i] = q[i];
  a.dt = p->dt;
  a.L = p->L;
  a.logL = p->logL;
  a.Lh = p->Lh;
  a.TN = p->TN;
  a.logTN = p->logTN;
  return a;
}

aao::BwdArgs bwd_args(aao_plan* p, double* u) {
  aao::BwdArgs a{};
  a.in = p->vec(0);  // Krylov solution X
  a.u = u;
  a.scale = p->d_sb();
  a.tw = p->d_tw();
  a.mix = p->d_m2();
  a.part = p->fb() + p->fb_slots;
  a.g = {p->nx, p->ny, p->N};
  a.L = p->L;
  a.logL = p->logL;
  a.Lh = p->Lh;
  a.TN = p->TN;
  a.logTN = p->logTN;
  return a;
}

// BiCGStab chunking for nact active systems: as many workgroups in all as the
// plan uses with every system active (wps per system), spread over the
// systems still active (at most wps_max per system).
void krylov_chunks(const aao_plan* p, int nact, aao::KrylovArgs& a) {
  const int64_t total = (int64_t)p->wps * p->S;
  const int na = std::max(nact, 1);
  int want = (int)std::min<int64_t>(p->wps_max, std::max<int64_t>(p->wps, (total + na - 1) / na));
  int chunk = (p->N + want - 1) / want;
  chunk = ((chunk + aao::kBlock - 1) / aao::kBlock) * aao::kBlock;
  a.chunk = chunk;
  a.wps = (p->N + chunk - 1) / chunk;
}

aao::KrylovArgs krylov_args(aao_plan* p, int adj, int nsys) {
  aao::KrylovArgs a{};
  a.X = p->vec(0);
  a.R = p->vec(1);
  a.P[0] = p->vec(2);
  a.P[1] = p->vec(3);
  a.V[0] = p->vec(4);
  a.V[1] = p->nvec > 5 ? p->vec(5) : nullptr;
  a.Rh = p->nvec > 6 ? p->vec(6) : nullptr;
  a.S = p->nvec > 7 ? p->vec(7) : nullptr;
  a.T = p->nvec > 8 ? p->vec(8) : nullptr;
  a.shift = p->d_sh();
  a.st = p->st();
  a.part = p->part();
  a.work = p->work();
  a.sys_list = p->dlist();
  a.g = {p->nx, p->ny, p->N};
  a.taps = adj ? p->tapsT : p->taps;
  a.num_sys = nsys;
  krylov_chunks(p, nsys, a);
  a.wps_stride = p->wps_max;
  a.wps_rho = a.wps;
  a.wps_bb = a.wps;
  a.tol2 = p->inner_tol * p->inner_tol;
  a.bbfloor = p->floor_on ? p->d_bf() : nullptr;
  a.maxit = p->inner_maxit;
  return a;
}

// Tile fields of the COCG arguments: the large tiling, or the small one.
void cg_tiling(aao::CgArgs& a, const aao_plan* p, bool small) {
  a.TX = small ? p->cgTXs : p->cgTX;
  a.TY = small ? p->cgTYs : p->cgTY;
  a.ntx = small ? p->cg_ntxs : p->cg_ntx;
  a.ntiles = small ? p->cg_ntiles_s : p->cg_ntiles;
  a.nty = a.ntiles / a.ntx;
  auto magic = [](int d) { return ((1ull << 40) + (unsigned long long)d - 1) / (unsigned long long)d; };
  a.m_ntx = magic(a.ntx);
  a.m_tx = magic(a.TX);
  a.m_pw = magic(a.TX + 4 * a.Rx);
  a.m_hw = a.Rx > 0 ? magic(4 * a.Rx) : 0;
  a.xcd_band = (AAO_XCD_BANDS && a.ntiles % 8 == 0 && a.ntiles >= 16) ? a.ntiles / 8 : 0;
}

aao::CgArgs cg_args(aao_plan* p, int adj, int nsys) {
  aao::CgArgs a{};
  a.snap_row = -1;  // no snapshot row unless a pass is given one
  a.X = p->vec(0);
  a.R[0] = p->vec(1);
  a.R[1] = p->vec(2);
  a.P[0] = p->vec(3);
  a.P[1] = p->vec(4);
  a.shift = p->d_sh();
  a.st = p->st();
  a.part = p->part();
  a.sys_list = p->dlist();
  a.work = p->work();
  a.g = {p->nx, p->ny, p->N};
  a.taps = adj ? p->tapsT : p->taps;
  a.num_sys = nsys;
  a.Rx = p->Rx;
  a.Ry = p->Ry;
  cg_tiling(a, p, false);
  a.fused = a.ntiles <= 256 ? 1 : 0;
  a.ntiles_prev = a.ntiles;
  a.part_stride = (size_t)5 * nsys * std::max(p->cg_ntiles, p->cg_ntiles_s);
  a.tol2 = p->inner_tol * p->inner_tol;
  a.bbfloor = p->floor_on ? p->d_bf() : nullptr;
  a.maxit = p->inner_maxit;
  return a;
}

// Lagged convergence checks: every few iterations a one-workgroup kernel
// lists the still-active systems into one of two device buffers and writes
// their count, then a tag, to pinned host memory (a system-scope fence between
// the two).  At the next check the host waits for that tag (one interval
// late, so the launch queue never drains on a host round trip), switches the
// launches to that list and sizes their grids by its count.  No event is
// recorded: a marker in the queue would hold back the next pass.  Passes
// launched after a system converged exit at once (its state says inactive).
struct LagCheck {
  aao_plan* p;
  int nsys;
  int tag[2] = {0, 0};
  int pending = -1, cur = 0;
  int deferred = -1;  // slot of a snapshot that the next fused COCG pass takes (-1: none)
};

// Start a new snapshot; if an earlier one is outstanding, wait for it first
// and make its list current (n_out = its count, else -1).  defer: the next
// fused COCG pass takes the snapshot (one extra workgroup) instead of a
// kernel of its own.
aao_status lag_check(LagCheck& c, int& nact, const int*& list, int& n_out, bool final_check, bool defer = false) {
  aao_plan* p = c.p;
  n_out = -1;
  if (c.pending >= 0) {
    // the kernel's own fence orders count before tag: wait (bounded) for
    // this snapshot's tag
    volatile int* ct = p->hlist + 2 * c.pending;
    const auto t0 = std::chrono::steady_clock::now();
    while (ct[1] != c.tag[c.pending]) {
      if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(5))
        return fail(AAO_EHIP, "active-system snapshot did not reach host memory");
    }
    const int n = ct[0];
    n_out = n;
    if (n > 0) {
      list = p->dlist(c.pending);
      nact = n;
    }
    c.pending = -1;
    if (n == 0 || final_check) return AAO_OK;
  }
  c.tag[c.cur] = ++p->snap_tag;
  if (defer) {
    c.deferred = c.cur;
  } else {
    close_run(p);
    HIPCHK(aao::launch_compact_active(p->st(), c.nsys, p->dlist(c.cur), p->hlist + 2 * c.cur, c.tag[c.cur],
                                      p->stream));
  }
  c.pending = c.cur;
  c.cur ^= 1;
  return AAO_OK;
}

aao_status lag_begin(aao_plan* p, LagCheck& c, int nsys) {
  c.p = p;
  c.nsys = nsys;
  return AAO_OK;
}

// Complex words per element that the COCG passes of one system move when it
// made ks iterations: pass k reads r (and p_{k-1} after the first) and writes
// r and p; odd passes also write x (and read it after pass 1); if the last
// pass was even, its x update is applied afterwards (in the stopping pass when
// fused, else in the closing kernel: reads p, writes x, reads x after pass 1).
double cocg_words(int ks) {
  double w = 0;
  for (int k = 0; k < ks; ++k) {
    w += (k > 0) ? 4 : 3;
    if (k & 1) w += (k >= 3) ? 2 : 1;
  }
  if (ks & 1) w += (ks >= 3) ? 3 : 2;
  return w;
}

// Single-pass COCG over all nsys systems.
aao_status inner_solve_cg(aao_plan* p, int adj, int nsys) {
  aao::CgArgs a = cg_args(p, adj, nsys);
  aao::KrylovArgs ka = krylov_args(p, adj, nsys);
  int nact = nsys;  // all active: the initial list is 0 .. nsys - 1
  if (a.fused) {
    a.init_list = p->dlist(2);  // the init pass writes the fresh states and the list
  } else {
    close_run(p);
    HIPCHK(aao::launch_krylov_init(ka, p->stream, p->dlist(2)));
  }
  HIPCHK(timed(p, aao::KC_COCG_B, [&] { return aao::launch_cg_init(p->f32, a, nact, p->stream); }));
  a.init_list = nullptr;
  if (!a.fused) HIPCHK(timed(p, aao::KC_MISC, [&] { return aao::launch_cg_scalars(a, -1, nact, p->stream); }));
  LagCheck c;
  aao_status ls = lag_begin(p, c, nsys);
  if (ls != AAO_OK) return ls;
  int next_check = AAO_CG_CHECK_EARLY;
  bool small = false;
  // fused: pass k advances the scalars from pass k-1's sums (pass inner_maxit
  // only records the iteration cap); else a scalar kernel follows each pass
  const int last = a.fused ? p->inner_maxit : p->inner_maxit - 1;
  for (int k = 0; k <= last; ++k) {
    a.snap_row = -1;
    if (c.deferred >= 0) {  // this pass also lists the systems still iterating after pass k - 1
      a.snap_row = nact;
      a.snap_k = k - 1;
      a.snap_n = nsys;
      a.snap_tag = c.tag[c.deferred];
      a.snap_list = p->dlist(c.deferred);
      a.snap_host = p->hlist + 2 * c.deferred;
      c.deferred = -1;
    }
    HIPCHK(timed(p, aao::KC_COCG_A, [&] { return aao::launch_cg_pass(p->f32, a, k, nact, p->stream); }));
    a.snap_row = -1;
    a.ntiles_prev = a.ntiles;
    if (!a.fused)
      HIPCHK(timed(p, aao::KC_MISC, [&] { return aao::launch_cg_scalars(a, k, nact, p->stream); }));
    if (k + 1 == next_check) {
      int n;
      aao_status s = lag_check(c, nact, a.sys_list, n, false, a.fused != 0);
      if (s != AAO_OK) return s;
      if (n == 0) break;
      // few systems left: the passes are bound by latency, and small tiles
      // spread each system over more CUs
      if (!small && a.fused && p->cg_ntiles_s > 0 && (long)nact * p->cg_ntiles <= AAO_CG_SMALL_WG) {
        cg_tiling(a, p, true);
        small = true;
      }
      next_check += small ? AAO_CG_CHECK_SMALL : (k < AAO_CG_CHECK_SWITCH ? AAO_CG_CHECK_EARLY : AAO_CG_CHECK_LATE);
    }
  }
  if (c.deferred >= 0) {  // requested after the last pass: no pass takes it
    c.deferred = -1;
    c.pending = -1;
  }
  if (c.pending >= 0) {  // drain the last outstanding snapshot
    int n;
    aao_status s = lag_check(c, nact, a.sys_list, n, true);
    if (s != AAO_OK) return s;
  }
  if (!a.fused) {  // x updates left pending by a last even pass
    close_run(p);
    HIPCHK(timed(p, aao::KC_MISC, [&] { return aao::launch_cg_xfix(p->f32, a, nsys, p->stream); }));
  }
  return AAO_OK;
}

// Solve the nsys shifted systems held in R into X.  Fills the per-system
// iteration counts into p->hread (as SysState) after the final check.
// Spatial-FFT direct solve of all nsys systems (exact; no iteration).
aao_status inner_solve_fft(aao_plan* p, int adj, int nsys) {
  aao::KrylovArgs ka = krylov_args(p, adj, nsys);
  close_run(p);
  HIPCHK(aao::launch_krylov_init(ka, p->stream));  // iteration counts read back as 0
  aao::FftArgs f{};
  f.R = p->vec(1);
  f.X = p->vec(0);
  f.shift = p->d_sh();
  f.Wx = p->d_wx();
  f.Wy = p->d_wy();
  f.taps = adj ? p->tapsT : p->taps;
  f.nx = p->nx;
  f.ny = p->ny;
  f.N = p->N;
  f.lognx = ilog2(p->nx);
  f.logny = ilog2(p->ny);
  f.px2 = is_pow2(p->nx) ? 1 : 0;
  f.py2 = is_pow2(p->ny) ? 1 : 0;
  f.diag = 0;
  for (int t = 0; t < f.taps.n; ++t)
    if (f.taps.dx[t] != 0 && f.taps.dy[t] != 0) f.diag = 1;
  f.rows = p->fft_rows;
  f.cols = p->fft_cols;
  f.norm = (double)p->N;
  auto blue = [&](int n, int P, size_t off) {
    aao::BlueDim d{};
    if (!P) return d;
    const double2* base = reinterpret_cast<const double2*>(p->dtab + off);
    d.P = P;
    d.logP = ilog2(P);
    d.W = base;
    d.ch = base + P;
    d.Bf = base + P + n;
    d.Bi = base + 2 * P + n;
    return d;
  };
  f.bx = blue(p->nx, p->Px, p->off_bx);
  f.by = blue(p->ny, p->Py, p->off_by);
  HIPCHK(timed(p, aao::KC_FFT_INNER, [&] { return aao::launch_fft_solve(p->f32, f, nsys, p->stream); }));
  p->work_later[aao::KC_FFT_INNER] += (double)nsys * p->N;
  return AAO_OK;
}

aao_status inner_solve(aao_plan* p, int adj, int nsys) {
  if (p->inner == AAO_INNER_COCG) return inner_solve_cg(p, adj, nsys);
  if (p->inner == AAO_INNER_FFT) return inner_solve_fft(p, adj, nsys);
  aao::KrylovArgs a = krylov_args(p, adj, nsys);
  if (aao::bicg_wg_fits(p->N)) {  // one workgroup runs every iteration of one system
    HIPCHK(timed(p, aao::KC_BICG_WG, [&] { return aao::launch_bicg_wg(p->f32, a, nsys, p->stream); }));
    return AAO_OK;
  }
  // tiled: phases 1 and 2 on the COCG tiles, one chunk per tile throughout
  const bool tiled = p->bicg_tiled;
  aao::CgArgs g{};
  if (tiled) {
    g = cg_args(p, adj, nsys);
    a.wps = g.ntiles;
    a.chunk = (p->N + g.ntiles - 1) / g.ntiles;
    a.wps_rho = a.wps;
    a.wps_bb = a.wps;
  }
  auto phase = [&](int ph, int k, int nact) {
    return (tiled && ph < 3) ? aao::launch_bicg_tiled(ph, p->f32, g, a, k, nact, p->stream)
                             : aao::launch_bicg(ph, p->f32, a, k, nact, p->stream);
  };
  close_run(p);
  HIPCHK(aao::launch_krylov_init(a, p->stream, p->dlist(2)));  // all active: the list is 0 .. nsys - 1
  int nact = nsys;
  LagCheck c;
  aao_status ls = lag_begin(p, c, nsys);
  if (ls != AAO_OK) return ls;
  int next_check = AAO_BICG_CHECK_EARLY;
  for (int k = 0; k <= p->inner_maxit; ++k) {
    HIPCHK(timed(p, aao::KC_BICG_1, [&] { return phase(1, k, nact); }));
    if (k < p->inner_maxit) {
      HIPCHK(timed(p, aao::KC_BICG_2, [&] { return phase(2, k, nact); }));
      HIPCHK(timed(p, aao::KC_BICG_3, [&] { return phase(3, k, nact); }));
      a.wps_rho = a.wps;  // rho_{k+1} and ||r_{k+1}||^2 were written by a.wps chunks
    }
    if (k + 1 == next_check) {
      next_check += (k < AAO_CG_CHECK_SWITCH) ? AAO_BICG_CHECK_EARLY : AAO_BICG_CHECK_LATE;
      int n;
      aao_status s = lag_check(c, nact, a.sys_list, n, false);
      if (s != AAO_OK) return s;
      if (n == 0) break;
      if (!tiled) krylov_chunks(p, nact, a);  // wider launches once fewer systems remain
    }
  }
  if (c.pending >= 0) {
    int n;
    aao_status s = lag_check(c, nact, a.sys_list, n, true);
    if (s != AAO_OK) return s;
  }
  return AAO_OK;
}

struct SweepOut {
  double res2 = 0, dmax = 0;
  double inner_mean = 0;
  int inner_max = 0, inner_fail = 0;
};

// Work of the inner solves of one sweep: sum and sum of max(iters - 1, 0)
// over the systems, and (COCG) the words of cocg_words summed.
void account_inner(aao_plan* p, int nsys, double sum, double later, double words) {
  if (nsys <= 0) return;
  const double n = (double)p->N;
  if (p->inner == AAO_INNER_FFT) {
    // counted in inner_solve_fft
  } else if (p->inner == AAO_INNER_COCG) {
    p->work_first[aao::KC_COCG_B] += n * nsys;  // init pass
    p->bytes_direct[aao::KC_COCG_A] += n * words * (double)p->csize;
    p->elems_direct[aao::KC_COCG_A] += n * sum;
  } else if (aao::bicg_wg_fits(p->N)) {  // reads b, writes x and the last residual
    p->bytes_direct[aao::KC_BICG_WG] += 3.0 * n * nsys * (double)p->csize;
    p->elems_direct[aao::KC_BICG_WG] += n * sum;
  } else {
    for (int c : {aao::KC_BICG_1, aao::KC_BICG_2, aao::KC_BICG_3}) {
      p->work_first[c] += n * nsys;
      p->work_later[c] += n * later;
    }
  }
}

// Read norms and per-system Krylov statistics (synchronises the stream).
aao_status read_back(aao_plan* p, int nsys, bool want_norms, SweepOut& o) {
  close_run(p);
  double* hn = reinterpret_cast<double*>(p->hread + 64);
  aao::SysState* hs = reinterpret_cast<aao::SysState*>(p->hread + 128);
  if (want_norms) HIPCHK(hipMemcpyAsync(hn, p->norms(), 2 * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  if (nsys > 0) {
    close_run(p);
    HIPCHK(hipMemcpyAsync(hs, p->st(), (size_t)nsys * sizeof(aao::SysState), hipMemcpyDeviceToHost, p->stream));
  }
  close_run(p);
  HIPCHK(hipStreamSynchronize(p->stream));
  collect_timing(p);
  if (want_norms) {
    o.res2 = hn[0];
    o.dmax = hn[1];
  }
  double sum = 0, later = 0;
  for (int s = 0; s < nsys; ++s) {
    sum += hs[s].iters;
    later += std::max(hs[s].iters - 1, 0);
    o.inner_max = std::max(o.inner_max, hs[s].iters);
    if (hs[s].flag != 0) o.inner_fail += 1;
  }
  o.inner_mean = nsys ? sum / nsys : 0;
  double words = 0;  // x moves every other pass
  if (p->inner == AAO_INNER_COCG)
    for (int s = 0; s < nsys; ++s) words += cocg_words(hs[s].iters);
  account_inner(p, nsys, sum, later, words);
  return AAO_OK;
}

// Wait for the end-of-sweep report tag (spin briefly, then block on the
// stream) and take the norms and iteration statistics from it.
aao_status read_report(aao_plan* p, int nsys, int tag, SweepOut& o) {
  close_run(p);
  const double* hr = reinterpret_cast<const double*>(reinterpret_cast<char*>(p->hlist) + 64);
  volatile const int* ht = reinterpret_cast<volatile const int*>(hr + 8);
  const auto t0 = std::chrono::steady_clock::now();
  while (*ht != tag) {
    if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2)) {
      HIPCHK(hipStreamSynchronize(p->stream));
      if (*ht != tag) return fail(AAO_EHIP, "end-of-sweep report did not reach host memory");
      break;
    }
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  o.res2 = hr[0];
  o.dmax = hr[1];
  const double sum = hr[2], later = hr[3];
  o.inner_max = (int)hr[4];
  o.inner_fail = (int)hr[5];
  o.inner_mean = nsys ? sum / nsys : 0;
  account_inner(p, nsys, sum, later, hr[6]);
  return AAO_OK;
}

// Device table block, pinned staging and the static tables (twiddles, Q); done
// once, on the first aao_set_workspace, so that aao_setup stays host-only.
aao_status alloc_tables(aao_plan* p) {
  if (p->dtab) return AAO_OK;
  HIPCHK(hipMalloc(&p->dtab, p->tab_bytes));
  HIPCHK(hipHostMalloc(&p->htab, 2 * p->atab_stride, hipHostMallocDefault));
  HIPCHK(hipHostMalloc(&p->hread, p->hread_bytes, hipHostMallocDefault));
  HIPCHK(hipHostMalloc(&p->hlist, 256, hipHostMallocDefault));
  // Pinned memory may come back from an earlier allocation with its old
  // contents: a snapshot or report tag left there by a destroyed plan would
  // match this plan's first tags (both count from 1), so every byte starts at 0.
  std::memset(p->hlist, 0, 256);
  std::memset(p->htab, 0, 2 * p->atab_stride);
  std::memset(p->hread, 0, p->hread_bytes);
  std::vector<double2> tw(p->L / 2 + 1);
  for (int k = 0; k < (int)tw.size(); ++k) {
    const double ang = -2.0 * M_PI * (double)k / (double)p->L;
    tw[k].x = std::cos(ang);
    tw[k].y = std::sin(ang);
  }
  close_run(p);
  HIPCHK(hipMemcpyAsync(p->dtab + p->off_tw, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice,
                        p->stream));
  close_run(p);
  HIPCHK(hipMemcpyAsync(p->dtab + p->off_q, p->Q.data(), p->Q.size() * sizeof(double), hipMemcpyHostToDevice,
                        p->stream));
  // e^{+2 pi i k / n} for the spatial transforms of the FFT inner solve
  std::vector<double2> wx(p->nx), wy(p->ny);
  for (int k = 0; k < p->nx; ++k) {
    wx[k].x = std::cos(2.0 * M_PI * k / p->nx);
    wx[k].y = std::sin(2.0 * M_PI * k / p->nx);
  }
  for (int k = 0; k < p->ny; ++k) {
    wy[k].x = std::cos(2.0 * M_PI * k / p->ny);
    wy[k].y = std::sin(2.0 * M_PI * k / p->ny);
  }
  close_run(p);
  HIPCHK(hipMemcpyAsync(p->dtab + p->off_wx, wx.data(), wx.size() * sizeof(double2), hipMemcpyHostToDevice, p->stream));
  close_run(p);
  HIPCHK(hipMemcpyAsync(p->dtab + p->off_wy, wy.data(), wy.size() * sizeof(double2), hipMemcpyHostToDevice, p->stream));
  // Bluestein tables of the dimensions that are not powers of two
  std::vector<double2> bt[2];
  for (int dim = 0; dim < 2; ++dim) {
    const int n = dim == 0 ? p->nx : p->ny, P = dim == 0 ? p->Px : p->Py;
    if (!P) continue;
    std::vector<aao::cd> W, ch, Bf, Bi;
    aao::bluestein_tables(n, P, W, ch, Bf, Bi);
    std::vector<double2>& b = bt[dim];
    for (const auto* v : {&W, &ch, &Bf, &Bi})
      for (const aao::cd& z : *v) b.push_back(make_double2(z.real(), z.imag()));
    close_run(p);
    HIPCHK(hipMemcpyAsync(p->dtab + (dim == 0 ? p->off_bx : p->off_by), b.data(), b.size() * sizeof(double2),
                          hipMemcpyHostToDevice, p->stream));
  }
  close_run(p);
  HIPCHK(hipStreamSynchronize(p->stream));
  p->slot_alpha[0] = p->slot_alpha[1] = -1;
  return AAO_OK;
}

aao_status need_ready(aao_plan* p, bool need_u0) {
  if (!p) return fail(AAO_EINVAL, "null plan");
  if (!p->ws || p->ws_bytes < p->ws_need) return fail(AAO_EWORKSPACE, "workspace not set or too small");
  if (need_u0 && !p->u0) return fail(AAO_ESTATE, "aao_set_u0 has not been called");
  return AAO_OK;
}

// One sweep; res_stop > 0 stops before the update if ||r||/||w|| <= res_stop.
// One sweep with alpha; next_alpha > 0: the tables of the next sweep are
// built while this one runs.
aao_status do_sweep(aao_plan* p, double* u, double alpha, int adj, double res_stop, double next_alpha,
                    SweepOut& o, bool& stopped) {
  stopped = false;
  aao_status s = upload_tables(p, alpha, adj);
  if (s != AAO_OK) return s;
  aao::FwdArgs fa = fwd_args(p, u, adj);
  const bool f32 = p->f32;
  HIPCHK(timed(p, aao::KC_FWD, [&] { return aao::launch_fwd(p->M, adj, false, f32, fa, p->B, p->stream); }));
  const int nt = p->ntiles * p->B;
  if (res_stop > 0) {
    HIPCHK(timed(p, aao::KC_MISC, [&] { return aao::launch_finalize(p->fb(), nt, p->fb(), 0, p->norms(), p->stream); }));
    SweepOut pre;
    s = read_back(p, 0, true, pre);
    if (s != AAO_OK) return s;
    o.res2 = pre.res2;
    if (!std::isfinite(pre.res2)) return fail(AAO_ENAN, "residual norm is not finite");
    if (std::sqrt(pre.res2) <= res_stop * std::sqrt(adj ? 0.0 : p->w2)) {
      stopped = true;
      return AAO_OK;
    }
  }
  s = inner_solve(p, adj, p->S);
  if (s != AAO_OK) return s;
  aao::BwdArgs ba = bwd_args(p, u);
  HIPCHK(timed(p, aao::KC_BWD, [&] { return aao::launch_bwd(p->M, adj, false, f32, ba, p->B, p->stream); }));
  const int tag = ++p->rep_tag;
  double* hr = reinterpret_cast<double*>(reinterpret_cast<char*>(p->hlist) + 64);
  HIPCHK(timed(p, aao::KC_MISC, [&] {
    return aao::launch_sweep_report(p->fb(), nt, p->fb() + p->fb_slots, nt, p->norms(), p->st(), p->S,
                                    p->inner == AAO_INNER_COCG, hr, tag, p->stream);
  }));
  if (next_alpha > 0) prefetch_tables(p, next_alpha, adj);
  double keep = o.res2;
  s = read_report(p, p->S, tag, o);
  if (s != AAO_OK) return s;
  if (res_stop > 0) o.res2 = keep;
  if (!std::isfinite(o.res2) || !std::isfinite(o.dmax)) return fail(AAO_ENAN, "sweep produced a non-finite norm");
  return AAO_OK;
}

// A = A^T for a periodic stencil: the weight at offset d equals the weight at
// -d (needed by COCG, where I - c A must be complex-symmetric).
bool symmetric_taps(const aao::Taps& t) {
  for (int i = 0; i < t.n; ++i) {
    double c = 0, ci = 0;
    for (int k = 0; k < t.n; ++k) {
      if (t.dx[k] == -t.dx[i] && t.dy[k] == -t.dy[i]) c += t.c[k];
      if (t.dx[k] == t.dx[i] && t.dy[k] == t.dy[i]) ci += t.c[k];
    }
    if (std::abs(c - ci) > 1e-14 * std::max(1.0, std::abs(ci))) return false;
  }
  return true;
}

aao_status fill_taps(aao::Taps& t, int n, const int32_t* dx, const int32_t* dy, const double* c, int ndim) {
  t.n = n;
  for (int i = 0; i < n; ++i) {
    t.dx[i] = dx[i];
    t.dy[i] = (ndim == 2 && dy) ? dy[i] : 0;
    t.c[i] = c[i];
  }
  return AAO_OK;
}

}  // namespace

extern "C" {

const char* aao_last_error(void) { return g_err.c_str(); }

const char* aao_kernel_name(int c) {
  static const char* names[AAO_NUM_KERNELS] = {
      "fwd_residual_dft_l", "bwd_idft_l_update", "cocg_pass", "cocg_init",
      "bicgstab_p_matvec", "bicgstab_s_matvec", "bicgstab_update", "fft_inner",
      "residual", "misc", "init", "grad", "gmres_orth", "bicgstab_wg"};
  return (c >= 0 && c < AAO_NUM_KERNELS) ? names[c] : "";
}

aao_status aao_setup(const aao_stencil* A, const aao_config* cfg, void* hip_stream, aao_plan_t* out) {
  if (!A || !cfg || !out) return fail(AAO_EINVAL, "null argument");
  *out = nullptr;
  if (A->ndim != 1 && A->ndim != 2) return fail(AAO_EINVAL, "ndim must be 1 or 2");
  const int64_t nx = A->nx, ny = (A->ndim == 1) ? 1 : A->ny;
  if (nx < 2 || ny < 1 || (A->ndim == 2 && ny < 2)) return fail(AAO_EINVAL, "grid too small");
  if (nx * ny > (int64_t(1) << 28)) return fail(AAO_EINVAL, "grid too large (N <= 2^28)");
  if (A->ntaps < 1 || A->ntaps > aao::kMaxTaps) return fail(AAO_EINVAL, "ntaps must be in 1..32");
  if (!A->dx || !A->coef || (A->ndim == 2 && !A->dy)) return fail(AAO_EINVAL, "null stencil array");
  for (int i = 0; i < A->ntaps; ++i) {
    const int dxv = A->dx[i], dyv = A->ndim == 2 ? A->dy[i] : 0;
    if (std::abs(dxv) > 4 || std::abs(dyv) > 4 || std::abs(dxv) >= nx || (A->ndim == 2 && std::abs(dyv) >= ny))
      return fail(AAO_EINVAL, "tap offsets must satisfy |d| <= 4 and |d| < grid size");
    if (!std::isfinite(A->coef[i])) return fail(AAO_EINVAL, "non-finite stencil coefficient");
  }
  if (cfg->M < 1 || cfg->M > aao::kMaxM) return fail(AAO_EINVAL, "M must be in 1..8");
  if (!is_pow2(cfg->L) || cfg->L > 1024) return fail(AAO_EINVAL, "L must be a power of two in 1..1024");
  if ((int64_t)cfg->L * cfg->M > 2048) return fail(AAO_EINVAL, "L*M must not exceed 2048");
  if (!(cfg->dt > 0) || !std::isfinite(cfg->dt)) return fail(AAO_EINVAL, "dt must be positive");
  if (cfg->batch < 1) return fail(AAO_EINVAL, "batch must be >= 1");
  if (cfg->precision != AAO_FP64 && cfg->precision != AAO_MIXED) return fail(AAO_EINVAL, "bad precision");
  if (cfg->inner != AAO_INNER_COCG && cfg->inner != AAO_INNER_BICGSTAB && cfg->inner != AAO_INNER_FFT)
    return fail(AAO_EINVAL, "unknown inner solver");
  if (cfg->inner == AAO_INNER_FFT) {
    // one transform line (n, or the Bluestein length P >= 2n - 1) must fit 64 KiB of LDS
    const int64_t cs = cfg->precision == AAO_MIXED ? 8 : 16;
    if (fft_line(nx) * cs > 65536 || fft_line(ny) * cs > 65536)
      return fail(AAO_EINVAL, "FFT inner solve: a transform line (n if a power of two, else the Bluestein "
                              "length P >= 2n - 1) times sizeof(complex) must not exceed 64 KiB");
  }
  if (!(cfg->inner_tol > 0) || cfg->inner_maxit < 1) return fail(AAO_EINVAL, "bad inner tolerance / iteration cap");

  aao_plan* p = new aao_plan();
  p->ndim = A->ndim;
  p->nx = (int)nx;
  p->ny = (int)ny;
  p->N = (int)(nx * ny);
  p->M = cfg->M;
  p->L = cfg->L;
  p->logL = ilog2(cfg->L);
  p->Lh = cfg->L / 2 + 1;
  p->B = cfg->batch;
  p->dt = cfg->dt;
  p->precision = cfg->precision;
  p->inner = cfg->inner;
  p->inner_tol = cfg->inner_tol;
  p->inner_maxit = cfg->inner_maxit;
  p->stream = reinterpret_cast<hipStream_t>(hip_stream);
  p->f32 = (cfg->precision == AAO_MIXED);
  p->csize = p->f32 ? 8 : 16;

  // nodes and Q (Sec. 2.1, eq. (collocation))
  if (cfg->nodes) {
    p->t.assign(cfg->nodes, cfg->nodes + cfg->M);
    for (int m = 0; m < cfg->M; ++m)
      if (!(p->t[m] > (m ? p->t[m - 1] : 0.0)) || p->t[m] > 1.0) {
        delete p;
        return fail(AAO_EINVAL, "nodes must increase in (0, 1]");
      }
    if (p->t[cfg->M - 1] != 1.0) {
      delete p;
      return fail(AAO_EINVAL, "the last node must be 1 (H_M copies the last node)");
    }
  } else if (!aao::radau_right_nodes(cfg->M, p->t)) {
    delete p;
    return fail(AAO_EINVAL, "Radau node computation failed");
  }
  aao::collocation_matrix(p->t, p->Q);
  p->QT.assign(p->M * p->M, 0.0);
  for (int m = 0; m < p->M; ++m)
    for (int k = 0; k < p->M; ++k) p->QT[m * p->M + k] = p->Q[k * p->M + m];

  fill_taps(p->taps, A->ntaps, A->dx, A->dy, A->coef, A->ndim);
  std::vector<int32_t> rdx(A->ntaps), rdy(A->ntaps);
  for (int i = 0; i < A->ntaps; ++i) {
    rdx[i] = -A->dx[i];
    rdy[i] = A->ndim == 2 ? -A->dy[i] : 0;
  }
  fill_taps(p->tapsT, A->ntaps, rdx.data(), rdy.data(), A->coef, A->ndim);
  p->has_dnu = A->dcoef_dnu != nullptr;
  if (p->has_dnu) fill_taps(p->dtaps, A->ntaps, A->dx, A->dy, A->dcoef_dnu, A->ndim);
  p->symmetric = symmetric_taps(p->taps);
  if (p->inner == AAO_INNER_COCG && !p->symmetric) {
    delete p;
    return fail(AAO_EINVAL, "COCG needs a symmetric stencil (A = A^T); use BiCGStab");
  }
  for (int i = 0; i < A->ntaps; ++i) p->Anorm_inf += std::abs(A->coef[i]);

  // tiling of the DFT over l: TN spatial points per workgroup, LDS planes <= AAO_XFORM_LDS_KB
  int TN = 64;
  while (TN > 2 && (size_t)p->L * p->M * TN * 8 > AAO_XFORM_LDS_KB * 1024) TN >>= 1;
  p->TN = TN;
  p->logTN = ilog2(TN);
  p->ntiles = (p->N + TN - 1) / TN;

  // batched inner solves: S systems, wps workgroups per system
  p->S = p->B * p->Lh * p->M;
  p->nvec = (p->inner == AAO_INNER_COCG) ? 5 : (p->inner == AAO_INNER_FFT ? 2 : 9);
  if (p->inner == AAO_INNER_FFT) {
    p->Px = (int)blue_len(p->nx);
    p->Py = p->ny > 1 ? (int)blue_len(p->ny) : 0;
  }
  if (p->inner == AAO_INNER_FFT && p->ny > 1) {
    // rows (columns) per workgroup: a divisor of ny (nx) within the LDS budget
    const int cs = (int)p->csize;
    const int lx = aao::fft_pad_line((int)fft_line(p->nx)), ly = aao::fft_pad_line((int)fft_line(p->ny));
    p->fft_rows = largest_divisor(p->ny, AAO_FFT_ROW_LDS_KB * 1024 / (lx * cs));
    // columns: 128 bytes of consecutive elements per row where such a tile
    // fits the smaller budget (more workgroups per CU), else 64 bytes within
    // the larger one
    int ccap = std::min(128 / cs, AAO_FFT_COL_LDS_SMALL_KB * 1024 / (ly * cs));
    if (ccap * cs < 64) ccap = std::min(64 / cs, AAO_FFT_COL_LDS_KB * 1024 / (ly * cs));
    p->fft_cols = largest_divisor(p->nx, ccap);
  }
  {
    const int target = 4096;
    int wps = (target + p->S - 1) / p->S;
    wps = std::max(1, std::min(wps, (p->N + 1023) / 1024));
    int chunk = (p->N + wps - 1) / wps;
    chunk = ((chunk + aao::kBlock - 1) / aao::kBlock) * aao::kBlock;
    p->chunk = chunk;
    p->wps = (p->N + chunk - 1) / chunk;
    // as systems converge the grid would shrink to (active) x wps workgroups;
    // the launches widen back towards wps x S workgroups, down to one point
    // per thread, at most 256 chunks (one partial per thread in a reduction)
    p->wps_max = std::max(p->wps, std::min(256, (p->N + aao::kBlock - 1) / aao::kBlock));
  }
  // COCG tiles: TX x TY points per workgroup; Rx, Ry: stencil reach
  for (int i = 0; i < A->ntaps; ++i) {
    p->Rx = std::max(p->Rx, std::abs(p->taps.dx[i]));
    p->Ry = std::max(p->Ry, std::abs(p->taps.dy[i]));
  }
  if (p->ny == 1) {
    p->cgTX = std::min(p->nx, 1024);
    p->cgTY = 1;
  } else {
    p->cgTX = std::min(p->nx, AAO_CG_TX2D);
    p->cgTY = std::min(p->ny, AAO_CG_TY2D);
  }
  // at most `per` tile points per thread, and the two-hop region within 8 per
  // thread (LDS <= 32 KB); halves TY, then TX, until both hold
  auto fit_tile = [&](int& tx, int& ty, int per) {
    auto pts = [&](int x, int y) { return (x + 4 * p->Rx) * (y + 4 * p->Ry); };
    auto bad = [&] { return pts(tx, ty) > 8 * aao::kBlock || tx * ty > per * aao::kBlock; };
    while (bad() && ty > 1) ty = (ty + 1) / 2;
    while (bad() && tx > 8) tx = (tx + 1) / 2;
    return !bad();
  };
  if (!fit_tile(p->cgTX, p->cgTY, 4)) {
    delete p;
    return fail(AAO_EINVAL, "stencil reach too large for the COCG tile");
  }
  p->cg_ntx = (p->nx + p->cgTX - 1) / p->cgTX;
  p->cg_nty = (p->ny + p->cgTY - 1) / p->cgTY;
  p->cg_ntiles = p->cg_ntx * p->cg_nty;
  {  // small tiling (one point per thread) for the passes where few systems remain
    int tx = (p->ny == 1) ? std::min(p->nx, 256) : std::min(p->nx, 32);
    int ty = (p->ny == 1) ? 1 : std::min(p->ny, 8);
    if (fit_tile(tx, ty, 1)) {
      const int ntx = (p->nx + tx - 1) / tx, nts = ntx * ((p->ny + ty - 1) / ty);
      if (nts > p->cg_ntiles && nts <= aao::kBlock && p->cg_ntiles <= aao::kBlock) {
        p->cgTXs = tx;
        p->cgTYs = ty;
        p->cg_ntxs = ntx;
        p->cg_ntiles_s = nts;
      }
    }
  }
  if (p->inner == AAO_INNER_COCG && p->cg_ntiles >= (1 << 16)) {  // tile indices use 16-bit exact division
    delete p;
    return fail(AAO_EINVAL, "grid too large for the COCG tiling (at most 65535 tiles per system)");
  }
  // BiCGStab on the COCG tiles: 2D grids beyond the one-workgroup size with
  // at most 256 tiles per system (the update phase then uses one flat chunk
  // of ceil(N / tiles) points per tile)
  if (p->inner == AAO_INNER_BICGSTAB && p->ny > 1 && !aao::bicg_wg_fits(p->N)) {
    aao::CgArgs g{};
    g.TX = p->cgTX;
    g.TY = p->cgTY;
    g.Rx = p->Rx;
    g.Ry = p->Ry;
    g.ntiles = p->cg_ntiles;
    const int64_t nt = p->cg_ntiles;
    p->bicg_tiled = aao::bicg_tiled_fits(g) && nt * (nt - 1) < p->N;
    if (p->bicg_tiled) p->wps_max = std::max(p->wps_max, p->cg_ntiles);
  }
  p->fb_slots = std::max(p->ntiles * p->B, 1024);
  p->grad_blocks = std::max(1, std::min(256, (p->N + aao::kBlock - 1) / aao::kBlock));

  // workspace layout
  size_t off = 0;
  p->off_vec = off;
  off = align256(off + (size_t)p->nvec * p->S * p->N * p->csize);
  p->off_part = off;
  off = align256(off + std::max((size_t)aao::QP_COUNT * p->S * p->wps_max, (size_t)2 * 5 * p->S * std::max(p->cg_ntiles, p->cg_ntiles_s)) *
                           sizeof(double));
  p->off_list = off;  // three lists of active systems (two alternating snapshots, the initial one)
  off = align256(off + (size_t)3 * p->S * sizeof(int));
  p->off_st = off;
  off = align256(off + (size_t)p->S * sizeof(aao::SysState));
  p->off_fb = off;
  off = align256(off + 2 * (size_t)p->fb_slots * sizeof(double));
  p->off_norms = off;
  off = align256(off + 8 * sizeof(double));
  p->off_cnt = off;
  off = align256(off + 16 * sizeof(int));
  p->off_work = off;
  off = align256(off + kWorkSlots * sizeof(unsigned long long));
  p->off_gpart = off;
  off = align256(off + (size_t)p->B * p->grad_blocks * sizeof(double));
  p->off_npart = off;  // norms over all instances, then per instance
  off = align256(off + 2 * kNormBlocks * (size_t)(p->B + 1) * sizeof(double));
  p->off_win = off;
  off = align256(off + (size_t)p->B * p->N * sizeof(double));
  p->ws_need = off;

  // library-owned tables
  size_t t = 0;
  p->off_tw = t;
  t = align256(t + (size_t)(p->L / 2 + 1) * sizeof(double2));
  p->off_q = t;
  t = align256(t + (size_t)p->M * p->M * sizeof(double));
  p->off_wx = t;
  t = align256(t + (size_t)p->nx * sizeof(double2));
  p->off_wy = t;
  t = align256(t + (size_t)p->ny * sizeof(double2));
  // Bluestein blocks: W (P), ch (n), Bf (P), Bi (P)
  p->off_bx = t;
  t = align256(t + (p->Px ? (size_t)(3 * p->Px + p->nx) * sizeof(double2) : 0));
  p->off_by = t;
  t = align256(t + (p->Py ? (size_t)(3 * p->Py + p->ny) * sizeof(double2) : 0));
  p->off_sf = t;
  t = align256(t + (size_t)p->L * sizeof(double));
  p->off_sb = t;
  t = align256(t + (size_t)p->L * sizeof(double));
  p->off_m1 = t;
  t = align256(t + (size_t)p->Lh * p->M * p->M * sizeof(double2));
  p->off_m2 = t;
  t = align256(t + (size_t)p->Lh * p->M * p->M * sizeof(double2));
  p->off_sh = t;
  t = align256(t + (size_t)p->S * sizeof(double2));
  p->off_bf = t;
  t = align256(t + (size_t)p->S * sizeof(double));
  p->off_hostend = t;
  p->atab_stride = p->off_hostend - p->off_sf;
  p->tab_bytes = t + p->atab_stride;  // second slot of the alpha-dependent tables
  p->hread_bytes = 128 + (size_t)p->S * sizeof(aao::SysState) + 64;
  *out = p;
  return AAO_OK;
}

aao_status aao_set_inner_floor(aao_plan_t p, double tau_w) {
  if (!p) return fail(AAO_EINVAL, "null plan");
  if (!std::isfinite(tau_w)) return fail(AAO_EINVAL, "tau_w must be finite");
  p->floor_tol = tau_w < 0 ? -1.0 : tau_w;
  return AAO_OK;
}

aao_status aao_set_stream(aao_plan_t p, void* s) {
  if (!p) return fail(AAO_EINVAL, "null plan");
  p->stream = reinterpret_cast<hipStream_t>(s);
  return AAO_OK;
}

aao_status aao_set_stencil_coef(aao_plan_t p, const double* coef, const double* dcoef_dnu) {
  if (!p || !coef) return fail(AAO_EINVAL, "null argument");
  aao::Taps t = p->taps;
  double an = 0;
  for (int i = 0; i < t.n; ++i) {
    if (!std::isfinite(coef[i]) || (dcoef_dnu && !std::isfinite(dcoef_dnu[i])))
      return fail(AAO_EINVAL, "stencil coefficients must be finite");
    t.c[i] = coef[i];
    an += std::abs(coef[i]);
  }
  const bool sym = symmetric_taps(t);
  if (p->inner == AAO_INNER_COCG && !sym)
    return fail(AAO_EINVAL, "COCG needs a symmetric stencil (A = A^T); use BiCGStab");
  // kernels take the taps by value: launches enqueued earlier keep the old ones
  p->taps = t;
  for (int i = 0; i < t.n; ++i) p->tapsT.c[i] = coef[i];
  p->symmetric = sym;
  p->Anorm_inf = an;
  if (dcoef_dnu) {
    for (int i = 0; i < t.n; ++i) {
      p->dtaps.dx[i] = t.dx[i];
      p->dtaps.dy[i] = t.dy[i];
      p->dtaps.c[i] = dcoef_dnu[i];
    }
    p->dtaps.n = t.n;
    p->has_dnu = true;
  }
  return AAO_OK;
}

aao_status aao_workspace_size(aao_plan_t p, size_t* bytes) {
  if (!p || !bytes) return fail(AAO_EINVAL, "null argument");
  *bytes = p->ws_need;
  return AAO_OK;
}

aao_status aao_set_workspace(aao_plan_t p, void* dev, size_t bytes) {
  if (!p || !dev) return fail(AAO_EINVAL, "null argument");
  if ((reinterpret_cast<uintptr_t>(dev) & 255) != 0) return fail(AAO_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < p->ws_need)
    return fail(AAO_EWORKSPACE, "workspace of " + std::to_string(bytes) + " bytes < required " +
                                    std::to_string(p->ws_need));
  aao_status st = alloc_tables(p);
  if (st != AAO_OK) return st;
  p->ws = reinterpret_cast<char*>(dev);
  p->ws_bytes = bytes;
  return AAO_OK;
}

// ||w||_2^2 and ||w||_inf of the all-at-once right-hand side (Alg. 2 uses
// ||w||_inf, the residual stop ||w||_2); w = (1_M (x) u0 + dT Q b_1, dT Q b_2, ...).
// Per instance ||v_b||_2^2 of v [B][N] into n2, the slots of the alpha tables
// of direction adj marked stale (their inner floors scale with these norms).
// Enqueued only; the caller reads npart after synchronising.
static aao_status enqueue_norms_b(aao_plan* p, const double* v) {
  close_run(p);
  HIPCHK(aao::launch_norms_per_b(v, p->B, p->N, p->npart() + 2 * kNormBlocks, kNormBlocks, p->stream));
  return AAO_OK;
}
static void take_norms_b(aao_plan* p, const std::vector<double>& h, int adj) {
  std::vector<double>& n2 = p->n2[adj];
  n2.assign(p->B, 0.0);
  for (int b = 0; b < p->B; ++b)
    for (int i = 0; i < kNormBlocks; ++i) n2[b] += h[2 * kNormBlocks * (b + 1) + 2 * i];
  for (int i = 0; i < 2; ++i)
    if (p->slot_adj[i] == adj) p->slot_alpha[i] = -1;
}

static aao_status update_wnorms(aao_plan* p, const double* u0) {
  close_run(p);
  if (p->frc) {
    aao::FwdArgs fa = fwd_args(p, nullptr, 0);
    fa.w0 = u0;
    HIPCHK(aao::launch_wnorms(p->M, fa, p->B, p->npart(), kNormBlocks, p->stream));
  } else {
    HIPCHK(aao::launch_norms_bn(u0, p->B, p->N, p->npart(), kNormBlocks, p->stream));
  }
  aao_status st = enqueue_norms_b(p, u0);
  if (st != AAO_OK) return st;
  std::vector<double> h(2 * kNormBlocks * (size_t)(p->B + 1));
  HIPCHK(hipMemcpyAsync(h.data(), p->npart(), h.size() * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  double s2 = 0, mx = 0;
  for (int i = 0; i < kNormBlocks; ++i) {
    s2 += h[2 * i];
    mx = std::max(mx, h[2 * i + 1]);
  }
  if (!std::isfinite(s2)) return fail(AAO_ENAN, p->frc ? "u0 or the source contains NaN or Inf"
                                                       : "u0 contains NaN or Inf");
  p->w2 = p->frc ? s2 : p->M * s2;  // without a source ||w||_2^2 = M ||u0||^2
  p->winf = mx;
  take_norms_b(p, h, 0);
  return AAO_OK;
}

aao_status aao_set_u0(aao_plan_t p, const double* u0) {
  aao_status s = need_ready(p, false);
  if (s != AAO_OK) return s;
  if (!u0) return fail(AAO_EINVAL, "null u0");
  s = update_wnorms(p, u0);
  if (s != AAO_OK) return s;
  p->u0 = u0;
  return AAO_OK;
}

aao_status aao_set_forcing(aao_plan_t p, const double* b) {
  aao_status s = need_ready(p, false);
  if (s != AAO_OK) return s;
  const double* keep = p->frc;
  p->frc = b;
  if (p->u0) {
    s = update_wnorms(p, p->u0);
    if (s != AAO_OK) {
      p->frc = keep;
      return s;
    }
  }
  return AAO_OK;
}

aao_status aao_residual(aao_plan_t p, const double* u, double* r, double* res_norm) {
  aao_status s = need_ready(p, true);
  if (s != AAO_OK) return s;
  if (!u || !r) return fail(AAO_EINVAL, "null array");
  aao::FwdArgs fa = fwd_args(p, u, 0);
  const int nblk = std::min(1024, std::max(1, (int)(((int64_t)p->B * p->L * p->N + 255) / 256)));
  HIPCHK(timed(p, aao::KC_RESIDUAL, [&] { return aao::launch_residual(p->M, false, fa, r, p->B, p->stream); }));
  close_run(p);
  HIPCHK(aao::launch_finalize(p->fb(), nblk, p->fb(), 0, p->norms(), p->stream));
  SweepOut o;
  s = read_back(p, 0, true, o);
  if (s != AAO_OK) return s;
  if (res_norm) *res_norm = std::sqrt(o.res2) / std::sqrt(p->w2);
  return AAO_OK;
}

// aao_residual with its partial sums in the library's fixed device scratch
// (aao_noalloc.hip) instead of the plan's workspace: no workspace, no
// aao_set_u0, no allocation.  The kernels and the order of every reduction are
// those of aao_residual and aao_set_u0, so r and the norm come out the same
// bit for bit.
aao_status aao_residual_noalloc(aao_plan_t p, const double* u0, const double* u, double* r, double* res_norm) {
  if (!p) return fail(AAO_EINVAL, "null plan");
  if (!u0 || !u || !r) return fail(AAO_EINVAL, "null array");
  const int nblk = std::min(1024, std::max(1, (int)(((int64_t)p->B * p->L * p->N + 255) / 256)));
  if (nblk > aao::kScratchResParts || kNormBlocks != aao::kScratchWBlocks)
    return fail(AAO_EINVAL, "residual partial sums exceed the fixed scratch (" +
                                std::to_string(aao::kScratchResParts) + " blocks)");
  double* sc = nullptr;
  HIPCHK(aao::noalloc_scratch(&sc));
  aao::FwdArgs fa{};
  fa.u = u;
  fa.w0 = u0;
  fa.frc = p->frc;
  fa.part = sc;
  fa.g = {p->nx, p->ny, p->N};
  fa.taps = p->taps;
  for (int i = 0; i < p->M * p->M; ++i) fa.q[i] = p->Q[i];
  fa.dt = p->dt;
  fa.L = p->L;
  fa.logL = p->logL;
  fa.Lh = p->Lh;
  fa.TN = p->TN;
  fa.logTN = p->logTN;
  // ||w||: the kernels of aao_set_u0 into the scratch's w-norm slots
  if (p->frc) {
    aao::FwdArgs fw = fa;
    fw.part = nullptr;
    HIPCHK(aao::launch_wnorms(p->M, fw, p->B, sc + aao::kScratchWParts, kNormBlocks, p->stream));
  } else {
    HIPCHK(aao::launch_norms_bn(u0, p->B, p->N, sc + aao::kScratchWParts, kNormBlocks, p->stream));
  }
  HIPCHK(aao::launch_residual(p->M, false, fa, r, p->B, p->stream));
  HIPCHK(aao::launch_finalize(sc, nblk, sc, 0, sc + aao::kScratchOut, p->stream));
  double hn[2];
  double hw[2 * aao::kScratchWBlocks];
  HIPCHK(hipMemcpyAsync(hn, sc + aao::kScratchOut, sizeof hn, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipMemcpyAsync(hw, sc + aao::kScratchWParts, sizeof hw, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  double s2 = 0;
  for (int i = 0; i < kNormBlocks; ++i) s2 += hw[2 * i];
  if (!std::isfinite(s2)) return fail(AAO_ENAN, "u0 or the source contains NaN or Inf");
  const double w2 = p->frc ? s2 : p->M * s2;
  if (res_norm) *res_norm = std::sqrt(hn[0]) / std::sqrt(w2);
  return AAO_OK;
}

aao_status aao_precond(aao_plan_t p, const double* r, double* delta, double alpha) {
  aao_status s = need_ready(p, false);
  if (s != AAO_OK) return s;
  if (!r || !delta) return fail(AAO_EINVAL, "null array");
  s = upload_tables(p, alpha, 0);
  if (s != AAO_OK) return s;
  aao::FwdArgs fa = fwd_args(p, r, 0);
  HIPCHK(timed(p, aao::KC_FWD, [&] { return aao::launch_fwd(p->M, false, true, p->f32, fa, p->B, p->stream); }));
  s = inner_solve(p, 0, p->S);
  if (s != AAO_OK) return s;
  aao::BwdArgs ba = bwd_args(p, delta);
  HIPCHK(timed(p, aao::KC_BWD, [&] { return aao::launch_bwd(p->M, false, true, p->f32, ba, p->B, p->stream); }));
  SweepOut o;
  return read_back(p, p->S, false, o);
}

aao_status aao_sweep(aao_plan_t p, double* u, double alpha, double* res_rel, double* dlast_inf) {
  aao_status s = need_ready(p, true);
  if (s != AAO_OK) return s;
  if (!u) return fail(AAO_EINVAL, "null u");
  SweepOut o;
  bool stopped;
  s = do_sweep(p, u, alpha, 0, 0.0, 0.0, o, stopped);
  close_run(p);
  const hipError_t e = hipStreamSynchronize(p->stream);
  collect_timing(p);
  if (s != AAO_OK) return s;
  if (e != hipSuccess) return fail(AAO_EHIP, std::string("HIP: ") + hipGetErrorString(e));
  if (res_rel) *res_rel = std::sqrt(o.res2) / std::sqrt(p->w2);
  if (dlast_inf) *dlast_inf = o.dmax;
  return AAO_OK;
}

static aao_status run_solve_sweeps(aao_plan_t p, double* u, const double* alphas, int n_alphas, double m0,
                                   double tol, int stop_rule, int max_iter, aao_solve_info* info, int adj,
                                   double gnorm_inf);

// The sweeps read their reports without synchronising the stream; the timing
// events of the solve are collected once at its end.
static aao_status run_solve(aao_plan_t p, double* u, const double* alphas, int n_alphas, double m0,
                            double tol, int stop_rule, int max_iter, aao_solve_info* info, int adj,
                            double gnorm_inf) {
  p->solve_tol = tol;
  p->floor_div = 1;
  // a floor far below tau never binds (the relative stop is met first)
  p->floor_on = floor_tau(p) > 1e-8 * p->inner_tol;
  aao_status s = run_solve_sweeps(p, u, alphas, n_alphas, m0, tol, stop_rule, max_iter, info, adj, gnorm_inf);
  p->floor_on = false;
  close_run(p);
  hipError_t e = hipStreamSynchronize(p->stream);
  collect_timing(p);
  if (s == AAO_OK && e != hipSuccess) return fail(AAO_EHIP, std::string("HIP: ") + hipGetErrorString(e));
  return s;
}

static aao_status run_solve_sweeps(aao_plan_t p, double* u, const double* alphas, int n_alphas, double m0,
                                   double tol, int stop_rule, int max_iter, aao_solve_info* info, int adj,
                                   double gnorm_inf) {
  if (!info) return fail(AAO_EINVAL, "null info");
  if (max_iter < 1) return fail(AAO_EINVAL, "max_iter must be >= 1");
  if (alphas && n_alphas < 1) return fail(AAO_EINVAL, "n_alphas must be >= 1");
  if (stop_rule != AAO_STOP_LASTSTEP && stop_rule != AAO_STOP_RESIDUAL) return fail(AAO_EINVAL, "bad stop rule");
  if (adj && stop_rule != AAO_STOP_LASTSTEP) return fail(AAO_EINVAL, "adjoint supports the last-step rule only");
  std::memset(info, 0, sizeof(*info));
  // Alg. 2 (Sec. 3.3): gamma = L (3 eps + tau) ||w||_inf; eps is the unit
  // roundoff of the inner-solve precision.
  const double eps = p->f32 ? std::ldexp(1.0, -24) : std::ldexp(1.0, -53);
  const double wi = adj ? gnorm_inf : p->winf;
  const double gamma = p->L * (3 * eps + p->inner_tol) * wi;
  double m = m0 > 0 ? m0 : (adj ? wi : p->L * p->dt * p->Anorm_inf * p->winf);
  info->gamma = gamma;
  info->m0 = m;
  // alpha of sweep k and the error model after it (mm updated); the sequence
  // depends on gamma and m0 only, so the next sweep's alpha is known while
  // the current one runs.  done: Alg. 2's loop condition ended the iteration
  // (only when allow_exit).
  auto alpha_at = [&](int k, double& mm, bool allow_exit, bool& done) {
    done = false;
    if (alphas) return alphas[std::min(k, n_alphas - 1)];
    if (p->f32) {
      // Complex64 inner solves: in the defect-correction form the error of a
      // sweep is relative to the current residual, m_{k+1} = alpha m_k +
      // (gamma_r / alpha) m_k with gamma_r = L (3 eps + tau); minimising over
      // alpha as in eq. (minimeq) gives the constant alpha = sqrt(gamma_r).
      const double gr = p->L * (3 * eps + p->inner_tol);
      const double a = std::min(std::sqrt(gr), 0.5);
      mm = mm * (a + gr / a);
      return a;
    }
    if (allow_exit && mm <= tol) {  // Alg. 2 loop condition: the error model is below tol
      done = true;
      return 0.0;
    }
    const double a = std::min(std::sqrt(gamma / mm), 0.5);
    mm = 2 * std::sqrt(mm * gamma);
    return a;
  };
  // Sec. 3.3: the error model m_k overestimates the error and the difference
  // of consecutive iterates alone can take stagnation for convergence.  The
  // model's exit rests on gamma, which assumes every shifted system met tau,
  // so it is honoured only after a sweep without inner failures; and the
  // monitored quantity must keep improving: when kStallSweeps sweeps in a row
  // leave it above tol without a new best (below kStallGain times the best so
  // far), the call returns ESTAGNATE.  A slow but steady contraction (alpha
  // near 1/2 late in Alg. 2 contracts the lowest modes by about
  // alpha / (1 - alpha) per sweep) sets a new best every sweep; round-off
  // plateaus do not.  While the absolute inner floor is on, its error (of the
  // order of tau_w ||w||) is the first suspect: after kFloorStall sweeps
  // without a new best the floor is tightened a hundredfold (at most three
  // times, then switched off), and only a stall without it counts.
  constexpr int kStallSweeps = 4;
  constexpr int kFloorStall = 2;
  constexpr double kStallGain = 0.99;
  int last_fail = 0, stall = 0;
  double best_mon = 0.0;
  for (int k = 0; k < max_iter; ++k) {
    bool done;
    double alpha = alpha_at(k, m, last_fail == 0, done);
    if (done) {
      info->converged = 1;
      return AAO_OK;
    }
    double m_next = m, next_alpha = 0.0;
    if (k + 1 < max_iter) {
      next_alpha = alpha_at(k + 1, m_next, true, done);
      if (done) next_alpha = 0.0;
    }
    SweepOut o;
    bool stopped = false;
    aao_status s = AAO_ENODIAG;
    for (int tries = 0; tries < 6 && s == AAO_ENODIAG; ++tries) {
      s = do_sweep(p, u, alpha, adj, stop_rule == AAO_STOP_RESIDUAL ? tol : 0.0, next_alpha, o, stopped);
      if (s == AAO_ENODIAG && alphas) return s;
      if (s == AAO_ENODIAG) alpha = std::min(alpha * 1.05, 0.5);  // step off a non-diagonalisable alpha
    }
    if (s != AAO_OK) return s;
    const double wn = std::sqrt(adj ? 1.0 : p->w2);
    const double res_rel = std::sqrt(o.res2) / wn;
    if (k < AAO_MAX_HIST) {
      info->alpha[k] = alpha;
      info->m[k] = m;
      info->res_rel[k] = res_rel;
      info->dlast_inf[k] = stopped ? 0.0 : o.dmax;
      info->inner_mean[k] = stopped ? 0.0 : o.inner_mean;
      info->inner_max[k] = stopped ? 0 : o.inner_max;
      info->inner_fail[k] = stopped ? 0 : o.inner_fail;
    }
    if (stopped) {
      info->iterations = k;
      info->converged = 1;
      return AAO_OK;
    }
    info->inner_fail_total += o.inner_fail;
    last_fail = o.inner_fail;
    info->iterations = k + 1;
    if (stop_rule == AAO_STOP_LASTSTEP && o.dmax <= tol) {
      info->converged = 1;
      return AAO_OK;
    }
    // the residual rule monitors the residual before the sweep, the last-step
    // rule the difference the sweep made
    const double mon = stop_rule == AAO_STOP_RESIDUAL ? res_rel : o.dmax;
    if (k > 0 && mon > tol && !(mon < kStallGain * best_mon)) {
      ++stall;
      if (p->floor_on && stall >= kFloorStall) {
        p->floor_div *= 100;
        if (p->floor_div > 1e6) p->floor_on = false;
        stall = 0;
      } else if (!p->floor_on && stall >= kStallSweeps)
      {
        char msg[160];
        std::snprintf(msg, sizeof msg, "stagnation: %d sweeps in a row above tol without a new best (best %.3e, last %.3e)",
                      kStallSweeps, best_mon, mon);
        return fail(AAO_ESTAGNATE, msg);
      }
    } else {
      stall = 0;
    }
    if (k == 0 || mon < best_mon) best_mon = mon;
  }
  return fail(AAO_ENOCONV, "no convergence within max_iter sweeps");
}

aao_status aao_solve(aao_plan_t p, double* u, const double* alphas, int n_alphas, double m0, double tol,
                     int stop_rule, int max_iter, aao_solve_info* info) {
  aao_status s = need_ready(p, true);
  if (s != AAO_OK) return s;
  if (!u) return fail(AAO_EINVAL, "null u");
  HIPCHK(timed(p, aao::KC_INIT, [&] { return aao::launch_init_u(u, p->u0, p->B, p->L, p->M, p->N, p->stream); }));
  return run_solve(p, u, alphas, n_alphas, m0, tol, stop_rule, max_iter, info, 0, 0.0);
}

// ------------------------------------------------------------ outer GMRES
namespace {

// Scratch of aao_solve_gmres inside the caller's buffer: restart + 1 Arnoldi
// vectors V, restart preconditioned vectors Z (each [B][L][M][N] FP64,
// 256-byte aligned), a zero initial value [B][N] (to apply C alone), block
// partial sums, then coefficients [B][kGmresMax] followed by scales [B] (one
// upload).
struct GmresWs {
  double *V = nullptr, *Z = nullptr, *zero_u0 = nullptr, *part = nullptr, *coef = nullptr, *scl = nullptr;
  size_t stride = 0;  // doubles between basis vectors
  int nblk = 1;
  size_t bytes = 0;
};

GmresWs gmres_layout(const aao_plan* p, int restart, char* base) {
  GmresWs w;
  const int64_t D = (int64_t)p->L * p->M * p->N;
  w.stride = ((size_t)p->B * D + 31) / 32 * 32;
  w.nblk = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (D + 2047) / 2048));
  size_t off = 0;
  auto take = [&](size_t n_doubles) {
    double* q = reinterpret_cast<double*>(base + off);
    off = align256(off + n_doubles * sizeof(double));
    return q;
  };
  w.V = take((size_t)(restart + 1) * w.stride);
  w.Z = take((size_t)restart * w.stride);
  w.zero_u0 = take((size_t)p->B * p->N);
  w.part = take((size_t)p->B * w.nblk * aao::kGmresMax);
  w.coef = take((size_t)p->B * (aao::kGmresMax + 1));
  w.scl = w.coef + (size_t)p->B * aao::kGmresMax;
  w.bytes = off;
  return w;
}

// Pinned staging: [B][nblk][kGmresMax] partial sums, then coefficients and scales.
aao_status gmres_pinned(aao_plan* p, const GmresWs& w) {
  const size_t need = ((size_t)p->B * w.nblk * aao::kGmresMax + (size_t)p->B * (aao::kGmresMax + 1)) * sizeof(double);
  if (p->hgm_bytes >= need) return AAO_OK;
  if (p->hgm) HIPCHK(hipHostFree(p->hgm));
  p->hgm = nullptr;
  p->hgm_bytes = 0;
  HIPCHK(hipHostMalloc(&p->hgm, need, hipHostMallocDefault));
  p->hgm_bytes = need;
  return AAO_OK;
}

// Dot products <V_i[b], t[b]> (i < nvec) into out[b][i], summed on the host in
// a fixed order; synchronises the stream.
aao_status gmres_dots(aao_plan* p, const GmresWs& w, const double* V, int nvec, const double* t, double* out) {
  const int64_t D = (int64_t)p->L * p->M * p->N;
  const int K = aao::gmres_bucket(nvec);
  p->bytes_direct[aao::KC_GMRES] += (double)(nvec + 1) * p->B * D * sizeof(double);
  HIPCHK(timed(p, aao::KC_GMRES,
               [&] { return aao::launch_mdot(V, w.stride, nvec, t, D, p->B, w.part, w.nblk, p->stream); }));
  close_run(p);
  HIPCHK(hipMemcpyAsync(p->hgm, w.part, (size_t)p->B * w.nblk * K * sizeof(double), hipMemcpyDeviceToHost,
                        p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  for (int b = 0; b < p->B; ++b)
    for (int i = 0; i < nvec; ++i) {
      double acc = 0.0;
      for (int k = 0; k < w.nblk; ++k) acc += p->hgm[((size_t)b * w.nblk + k) * K + i];
      out[b * aao::kGmresMax + i] = acc;
    }
  return AAO_OK;
}

// out = s[b] in + sum_{i < nvec} c[b][i] V_i (c: [B][kGmresMax] host); with
// norm2 != null also ||out[b]||^2 (synchronises the stream).
aao_status gmres_axpy(aao_plan* p, const GmresWs& w, double* out, const double* in, const double* s,
                      const double* V, int nvec, const double* c, double* norm2) {
  const int64_t D = (int64_t)p->L * p->M * p->N;
  double* hc = p->hgm + (size_t)p->B * w.nblk * aao::kGmresMax;
  // the staging area is free: every earlier use of it ended in a stream synchronisation
  for (int b = 0; b < p->B; ++b) {
    for (int i = 0; i < aao::kGmresMax; ++i) hc[b * aao::kGmresMax + i] = (c && i < nvec) ? c[b * aao::kGmresMax + i] : 0.0;
    hc[(size_t)p->B * aao::kGmresMax + b] = s[b];
  }
  close_run(p);
  HIPCHK(hipMemcpyAsync(w.coef, hc, (size_t)p->B * (aao::kGmresMax + 1) * sizeof(double), hipMemcpyHostToDevice,
                        p->stream));
  p->bytes_direct[aao::KC_GMRES] += (double)(nvec + 2) * p->B * D * sizeof(double);
  HIPCHK(timed(p, aao::KC_GMRES, [&] {
    return aao::launch_maxpy(out, in, w.scl, V, w.stride, nvec, w.coef, D, p->B, norm2 ? w.part : nullptr, w.nblk,
                             p->stream);
  }));
  close_run(p);
  if (norm2) {
    HIPCHK(hipMemcpyAsync(p->hgm, w.part, (size_t)p->B * w.nblk * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  }
  // the next staging write must not overtake the upload
  HIPCHK(hipStreamSynchronize(p->stream));
  if (norm2)
    for (int b = 0; b < p->B; ++b) {
      double acc = 0.0;
      for (int k = 0; k < w.nblk; ++k) acc += p->hgm[(size_t)b * w.nblk + k];
      norm2[b] = acc;
    }
  return AAO_OK;
}

// r = w - C v with the plan's w (zero_w: w = 0 and no source, so r = -C v).
aao_status gmres_residual(aao_plan* p, const GmresWs& w, const double* v, double* r, bool zero_w) {
  aao::FwdArgs fa = fwd_args(p, v, 0);
  if (zero_w) {
    fa.w0 = w.zero_u0;
    fa.frc = nullptr;
  }
  HIPCHK(timed(p, aao::KC_RESIDUAL, [&] { return aao::launch_residual(p->M, false, fa, r, p->B, p->stream); }));
  return AAO_OK;
}

// z = C_alpha^{-1} v (rows a2 - a4); inner statistics into o.
aao_status gmres_precond(aao_plan* p, const double* v, double* z, double alpha, SweepOut& o) {
  aao_status s = upload_tables(p, alpha, 0);
  if (s != AAO_OK) return s;
  aao::FwdArgs fa = fwd_args(p, v, 0);
  HIPCHK(timed(p, aao::KC_FWD, [&] { return aao::launch_fwd(p->M, false, true, p->f32, fa, p->B, p->stream); }));
  s = inner_solve(p, 0, p->S);
  if (s != AAO_OK) return s;
  aao::BwdArgs ba = bwd_args(p, z);
  HIPCHK(timed(p, aao::KC_BWD, [&] { return aao::launch_bwd(p->M, false, true, p->f32, ba, p->B, p->stream); }));
  return read_back(p, p->S, false, o);
}

}  // namespace

aao_status aao_gmres_workspace_size(aao_plan_t p, int restart, size_t* bytes) {
  if (!p || !bytes) return fail(AAO_EINVAL, "null argument");
  if (restart < 1 || restart >= aao::kGmresMax) return fail(AAO_EINVAL, "restart must lie in 1..31");
  *bytes = gmres_layout(p, restart, nullptr).bytes;
  return AAO_OK;
}

aao_status aao_solve_gmres(aao_plan_t p, double* u, int restart, const double* alphas, int n_alphas, double tol,
                           int max_steps, void* work, size_t work_bytes, aao_gmres_info* info) {
  aao_status s = need_ready(p, true);
  if (s != AAO_OK) return s;
  if (!u || !work) return fail(AAO_EINVAL, "null array");
  if (restart < 1 || restart >= aao::kGmresMax) return fail(AAO_EINVAL, "restart must lie in 1..31");
  if (!(tol >= 0.0) || max_steps < 1) return fail(AAO_EINVAL, "tol must be >= 0 and max_steps >= 1");
  if ((reinterpret_cast<uintptr_t>(work) & 255) != 0) return fail(AAO_EINVAL, "GMRES workspace must be 256-byte aligned");
  if (alphas) {
    if (n_alphas < 1) return fail(AAO_EINVAL, "n_alphas must be >= 1");
    for (int i = 0; i < n_alphas; ++i)
      if (!(alphas[i] > 0.0 && alphas[i] < 1.0)) return fail(AAO_EINVAL, "alpha must lie in (0, 1)");
  }
  const GmresWs w = gmres_layout(p, restart, reinterpret_cast<char*>(work));
  if (work_bytes < w.bytes)
    return fail(AAO_EWORKSPACE, "GMRES workspace of " + std::to_string(work_bytes) + " bytes < required " +
                                    std::to_string(w.bytes));
  s = gmres_pinned(p, w);
  if (s != AAO_OK) return s;
  aao_gmres_info loc{};
  aao_gmres_info& o = info ? *info : loc;
  std::memset(&o, 0, sizeof(o));
  const int B = p->B, m = restart, KM = aao::kGmresMax;
  const int64_t D = (int64_t)p->L * p->M * p->N;
  const double eps = p->f32 ? std::ldexp(1.0, -24) : std::ldexp(1.0, -53);
  const double a_def = std::min(0.5, std::max(1e-8, std::sqrt(p->L * (3.0 * eps + p->inner_tol))));
  auto Vi = [&](int i) { return w.V + (size_t)i * w.stride; };
  auto Zi = [&](int i) { return w.Z + (size_t)i * w.stride; };

  close_run(p);
  HIPCHK(aao::launch_fill(w.zero_u0, 0.0, (int64_t)B * p->N, p->stream));
  // ||w_b||: the residual of a zero vector is w
  HIPCHK(aao::launch_fill(Zi(0), 0.0, (int64_t)B * D, p->stream));
  s = gmres_residual(p, w, Zi(0), Vi(0), false);
  if (s != AAO_OK) return s;
  std::vector<double> wn(B), dot((size_t)B * KM), h1((size_t)B * KM), h2((size_t)B * KM), nrm(B), scl(B);
  s = gmres_dots(p, w, Vi(0), 1, Vi(0), dot.data());
  if (s != AAO_OK) return s;
  for (int b = 0; b < B; ++b) wn[b] = std::sqrt(dot[(size_t)b * KM]);
  close_run(p);
  HIPCHK(aao::launch_init_u(u, p->u0, B, p->L, p->M, p->N, p->stream));

  // H[b][i][j] (i <= j + 1), Givens (c, s) per column, g the rotated right-hand side
  std::vector<double> H((size_t)B * (m + 1) * m), cs((size_t)B * m), sn((size_t)B * m), g((size_t)B * (m + 1)),
      y((size_t)B * KM);
  auto h = [&](int b, int i, int j) -> double& { return H[((size_t)b * (m + 1) + i) * m + j]; };
  auto rel = [&](int b, double r) { return wn[b] > 0.0 ? r / wn[b] : r; };
  bool conv = false;
  while (true) {
    // true residual r0 = w - C u
    s = gmres_residual(p, w, u, Vi(0), false);
    if (s != AAO_OK) return s;
    s = gmres_dots(p, w, Vi(0), 1, Vi(0), dot.data());
    if (s != AAO_OK) return s;
    double worst = 0.0;
    for (int b = 0; b < B; ++b) {
      nrm[b] = std::sqrt(dot[(size_t)b * KM]);
      worst = std::max(worst, rel(b, nrm[b]));
    }
    if (!std::isfinite(worst)) return fail(AAO_ENAN, "GMRES residual is not finite");
    o.res_rel = worst;
    if (worst <= tol) {
      conv = true;
      break;
    }
    if (o.steps >= max_steps) break;
    o.cycles += 1;
    // v_0 = r0 / ||r0|| per instance (an instance already solved keeps v_0 = 0)
    for (int b = 0; b < B; ++b) scl[b] = nrm[b] > 0.0 ? 1.0 / nrm[b] : 0.0;
    s = gmres_axpy(p, w, Vi(0), Vi(0), scl.data(), nullptr, 0, nullptr, nullptr);
    if (s != AAO_OK) return s;
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    for (int b = 0; b < B; ++b) g[(size_t)b * (m + 1)] = nrm[b];
    int jj = 0;
    for (int j = 0; j < m; ++j) {
      const double alpha = alphas ? alphas[std::min(o.steps, n_alphas - 1)] : a_def;
      SweepOut so;
      s = gmres_precond(p, Vi(j), Zi(j), alpha, so);
      if (s != AAO_OK) return s;
      // V_{j+1} <- -C z_j, then Gram-Schmidt twice against V_0 .. V_j
      s = gmres_residual(p, w, Zi(j), Vi(j + 1), true);
      if (s != AAO_OK) return s;
      s = gmres_dots(p, w, w.V, j + 1, Vi(j + 1), h1.data());
      if (s != AAO_OK) return s;
      std::vector<double> m1(B, -1.0), p1(B, 1.0);
      s = gmres_axpy(p, w, Vi(j + 1), Vi(j + 1), m1.data(), w.V, j + 1, h1.data(), nullptr);
      if (s != AAO_OK) return s;
      s = gmres_dots(p, w, w.V, j + 1, Vi(j + 1), h2.data());
      if (s != AAO_OK) return s;
      for (size_t q = 0; q < h2.size(); ++q) h2[q] = -h2[q];
      s = gmres_axpy(p, w, Vi(j + 1), Vi(j + 1), p1.data(), w.V, j + 1, h2.data(), nrm.data());
      if (s != AAO_OK) return s;
      double worst_est = 0.0;
      for (int b = 0; b < B; ++b) {
        for (int i = 0; i <= j; ++i) h(b, i, j) = -h1[(size_t)b * KM + i] - h2[(size_t)b * KM + i];
        const double hn = std::sqrt(nrm[b]);
        h(b, j + 1, j) = hn;
        scl[b] = hn > 0.0 ? 1.0 / hn : 0.0;
        // earlier rotations, then a new one that zeroes h(j + 1, j)
        for (int i = 0; i < j; ++i) {
          const double a0 = h(b, i, j), a1 = h(b, i + 1, j);
          h(b, i, j) = cs[(size_t)b * m + i] * a0 + sn[(size_t)b * m + i] * a1;
          h(b, i + 1, j) = -sn[(size_t)b * m + i] * a0 + cs[(size_t)b * m + i] * a1;
        }
        const double r = std::hypot(h(b, j, j), h(b, j + 1, j));
        const double c = r > 0.0 ? h(b, j, j) / r : 1.0, sj = r > 0.0 ? h(b, j + 1, j) / r : 0.0;
        cs[(size_t)b * m + j] = c;
        sn[(size_t)b * m + j] = sj;
        h(b, j, j) = r;
        h(b, j + 1, j) = 0.0;
        double& gj = g[(size_t)b * (m + 1) + j];
        g[(size_t)b * (m + 1) + j + 1] = -sj * gj;
        gj = c * gj;
        worst_est = std::max(worst_est, rel(b, std::fabs(g[(size_t)b * (m + 1) + j + 1])));
      }
      s = gmres_axpy(p, w, Vi(j + 1), Vi(j + 1), scl.data(), nullptr, 0, nullptr, nullptr);
      if (s != AAO_OK) return s;
      if (o.steps < AAO_MAX_HIST) {
        o.alpha[o.steps] = alpha;
        o.res_est[o.steps] = worst_est;
        o.inner_mean[o.steps] = so.inner_mean;
        o.inner_max[o.steps] = so.inner_max;
      }
      o.steps += 1;
      jj = j + 1;
      if (!std::isfinite(worst_est)) return fail(AAO_ENAN, "GMRES least-squares residual is not finite");
      if (worst_est <= tol || o.steps >= max_steps) break;
    }
    // y = R^{-1} g (upper triangular jj x jj per instance); u += Z y
    for (int b = 0; b < B; ++b) {
      for (int i = jj - 1; i >= 0; --i) {
        double acc = g[(size_t)b * (m + 1) + i];
        for (int k = i + 1; k < jj; ++k) acc -= h(b, i, k) * y[(size_t)b * KM + k];
        y[(size_t)b * KM + i] = h(b, i, i) != 0.0 ? acc / h(b, i, i) : 0.0;
      }
    }
    std::vector<double> one(B, 1.0);
    s = gmres_axpy(p, w, u, u, one.data(), w.Z, jj, y.data(), nullptr);
    if (s != AAO_OK) return s;
  }
  o.converged = conv ? 1 : 0;
  if (!conv) return fail(AAO_ENOCONV, "GMRES: max_steps reached without meeting tol");
  return AAO_OK;
}

aao_status aao_solve_windows(aao_plan_t p, double* u, int n_windows, const double* frc_all, const double* alphas,
                             int n_alphas, double m0, double tol, int stop_rule, int max_iter,
                             aao_solve_info* infos) {
  aao_status s = need_ready(p, true);
  if (s != AAO_OK) return s;
  if (!u || !infos) return fail(AAO_EINVAL, "null argument");
  if (n_windows < 1) return fail(AAO_EINVAL, "n_windows must be >= 1");
  const double* user_u0 = p->u0;
  const double* user_frc = p->frc;
  const size_t dofs = (size_t)p->B * p->L * p->M * p->N;
  aao_status r = AAO_OK;
  for (int k = 0; k < n_windows; ++k) {
    if (frc_all) p->frc = frc_all + (size_t)k * dofs;
    if (k > 0 || frc_all) {  // w changes with the window's initial value and source
      r = update_wnorms(p, p->u0);
      if (r != AAO_OK) break;
    }
    close_run(p);
    HIPCHK(timed(p, aao::KC_INIT, [&] { return aao::launch_init_u(u, p->u0, p->B, p->L, p->M, p->N, p->stream); }));
    r = run_solve(p, u, alphas, n_alphas, m0, tol, stop_rule, max_iter, infos + k, 0, 0.0);
    if (r != AAO_OK) break;
    if (k + 1 < n_windows) {
      // the next window starts from the last node of this one's last step;
      // the buffer is free again: this window's own u0 was last read above
      close_run(p);
      HIPCHK(aao::launch_last_node(u, p->win(), p->B, p->L, p->M, p->N, p->stream));
      p->u0 = p->win();
    }
  }
  p->u0 = user_u0;
  p->frc = user_frc;
  aao_status rs = update_wnorms(p, p->u0);
  return r != AAO_OK ? r : rs;
}

aao_status aao_adjoint_solve(aao_plan_t p, const double* g_last, double* lam, const double* alphas,
                             int n_alphas, double m0, double tol, int max_iter, aao_solve_info* info) {
  aao_status s = need_ready(p, false);
  if (s != AAO_OK) return s;
  if (!g_last || !lam) return fail(AAO_EINVAL, "null array");
  if (!info) return fail(AAO_EINVAL, "null info");
  close_run(p);
  HIPCHK(aao::launch_norms_bn(g_last, p->B, p->N, p->npart(), kNormBlocks, p->stream));
  s = enqueue_norms_b(p, g_last);
  if (s != AAO_OK) return s;
  std::vector<double> h(2 * kNormBlocks * (size_t)(p->B + 1));
  close_run(p);
  HIPCHK(hipMemcpyAsync(h.data(), p->npart(), h.size() * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  close_run(p);
  HIPCHK(hipStreamSynchronize(p->stream));
  double gi = 0, g2 = 0;
  for (int i = 0; i < kNormBlocks; ++i) {
    g2 += h[2 * i];
    gi = std::max(gi, h[2 * i + 1]);
  }
  if (!std::isfinite(g2)) return fail(AAO_ENAN, "g_last contains NaN or Inf");
  take_norms_b(p, h, 1);
  HIPCHK(timed(p, aao::KC_INIT, [&] { return aao::launch_fill(lam, 0.0, (int64_t)p->B * p->L * p->M * p->N, p->stream); }));
  const double* keep_u0 = p->u0;
  p->u0 = g_last;  // w0 of the transposed residual
  aao_status r = (gi == 0.0) ? AAO_OK
                             : run_solve(p, lam, alphas, n_alphas, m0, tol, AAO_STOP_LASTSTEP, max_iter, info, 1, gi);
  if (gi == 0.0) {
    std::memset(info, 0, sizeof(*info));
    info->converged = 1;
  }
  p->u0 = keep_u0;
  return r;
}

aao_status aao_grad(aao_plan_t p, const double* u, const double* lam, double* gu0, double* gnu) {
  aao_status s = need_ready(p, false);
  if (s != AAO_OK) return s;
  if (!u || !lam || !gu0 || !gnu) return fail(AAO_EINVAL, "null array");
  if (!p->has_dnu) return fail(AAO_EINVAL, "stencil has no dcoef_dnu");
  aao::Geo g{p->nx, p->ny, p->N};
  HIPCHK(timed(p, aao::KC_GRAD, [&] {
    return aao::launch_grad(p->M, u, lam, gu0, p->gpart(), p->dtaps, p->d_q(), p->dt, g, p->B, p->L,
                            p->grad_blocks, p->stream);
  }));
  close_run(p);
  HIPCHK(aao::launch_grad_finalize(p->gpart(), p->grad_blocks, p->B, gnu, p->stream));
  close_run(p);
  HIPCHK(hipStreamSynchronize(p->stream));
  collect_timing(p);
  return AAO_OK;
}

aao_status aao_shifted_solve(aao_plan_t p, int S, const double* shifts, const double* b, double* x, int* iters) {
  aao_status s = need_ready(p, false);
  if (s != AAO_OK) return s;
  if (S < 1 || S > p->S) return fail(AAO_EINVAL, "S must be in 1..B*(L/2+1)*M");
  if (!shifts || !b || !x) return fail(AAO_EINVAL, "null argument");
  close_run(p);
  HIPCHK(hipStreamSynchronize(p->stream));  // the host slot may still be in an upload
  cd* sh = reinterpret_cast<cd*>(p->htab + (size_t)p->cur_slot * p->atab_stride + (p->off_sh - p->off_sf));
  for (int i = 0; i < S; ++i) sh[i] = cd(shifts[2 * i], shifts[2 * i + 1]);
  close_run(p);
  HIPCHK(hipMemcpyAsync(p->d_sh(), sh, (size_t)S * sizeof(double2), hipMemcpyHostToDevice, p->stream));
  p->slot_alpha[0] = p->slot_alpha[1] = -1;
  const int64_t n = (int64_t)S * p->N;
  close_run(p);
  HIPCHK(aao::launch_copy_c128_in(p->vec(1), p->f32, b, n, p->stream));
  s = inner_solve(p, 0, S);
  if (s != AAO_OK) return s;
  close_run(p);
  HIPCHK(aao::launch_copy_c128_out(x, p->vec(0), p->f32, n, p->stream));
  SweepOut o;
  s = read_back(p, S, false, o);
  if (s != AAO_OK) return s;
  if (iters) {
    const aao::SysState* hs = reinterpret_cast<const aao::SysState*>(p->hread + 128);
    for (int i = 0; i < S; ++i) iters[i] = hs[i].iters;
  }
  return AAO_OK;
}

aao_status aao_set_timing(aao_plan_t p, int on) {
  if (!p) return fail(AAO_EINVAL, "null plan");
  close_run(p);
  p->timing = on != 0;
  return AAO_OK;
}

aao_status aao_reset_stats(aao_plan_t p) {
  if (!p) return fail(AAO_EINVAL, "null plan");
  std::memset(&p->stats, 0, sizeof(p->stats));
  std::memset(p->work_first, 0, sizeof(p->work_first));
  std::memset(p->work_later, 0, sizeof(p->work_later));
  std::memset(p->bytes_direct, 0, sizeof(p->bytes_direct));
  std::memset(p->elems_direct, 0, sizeof(p->elems_direct));
  return AAO_OK;
}

aao_status aao_get_stats(aao_plan_t p, aao_kernel_stats* out) {
  if (!p || !out) return fail(AAO_EINVAL, "null argument");
  *out = p->stats;
  const double cs = (double)p->csize;
  const double dof = (double)p->B * p->L * p->M * p->N;
  const double freq = (double)p->B * p->Lh * p->M * p->N;
  // fwd: read u (8 B/DOF), write x1; bwd: read x2, read and write u.
  out->elements[aao::KC_FWD] = dof * out->launches[aao::KC_FWD];
  out->bytes[aao::KC_FWD] = (8.0 * dof + cs * freq) * out->launches[aao::KC_FWD];
  out->elements[aao::KC_BWD] = dof * out->launches[aao::KC_BWD];
  out->bytes[aao::KC_BWD] = (16.0 * dof + cs * freq) * out->launches[aao::KC_BWD];
  // Krylov kernels: complex words read + written per element processed in
  // iterations after the first / in the first iteration (COCG passes: per
  // system, counted directly, see cocg_words).
  // FFT inner solve: read and write the vector once per pass (1 pass in 1D, 3 in 2D)
  const double fftw = p->ny > 1 ? 6.0 : 2.0;
  out->elements[aao::KC_COCG_A] = 0;
  out->bytes[aao::KC_COCG_A] = 0;
  struct { int c; double later, first; } kw[] = {
      {aao::KC_COCG_B, 1, 1}, {aao::KC_BICG_1, 6, 4},
      {aao::KC_BICG_2, 4, 4}, {aao::KC_BICG_3, 7, 6}, {aao::KC_FFT_INNER, fftw, fftw}};
  for (auto& k : kw) {
    out->elements[k.c] = p->work_first[k.c] + p->work_later[k.c];
    out->bytes[k.c] = cs * (k.later * p->work_later[k.c] + k.first * p->work_first[k.c]);
  }
  for (int c = 0; c < AAO_NUM_KERNELS; ++c) {
    out->bytes[c] += p->bytes_direct[c];
    out->elements[c] += p->elems_direct[c];
  }
  return AAO_OK;
}

aao_status aao_tables(aao_plan_t p, double alpha, double* d, double* r, double* djm, double* cond_max) {
  if (!p) return fail(AAO_EINVAL, "null plan");
  if (!(alpha > 0.0 && alpha < 1.0)) return fail(AAO_EINVAL, "alpha must lie in (0, 1)");
  double cm = 0;
  for (int j = 0; j < p->Lh; ++j) {
    aao::FreqTable ft;
    std::string why = aao::freq_table(p->t, p->Q, alpha, p->L, j, ft);
    if (d) { d[2 * j] = ft.d.real(); d[2 * j + 1] = ft.d.imag(); }
    if (r) { r[2 * j] = ft.r.real(); r[2 * j + 1] = ft.r.imag(); }
    if (djm)
      for (int m = 0; m < p->M; ++m) {
        djm[2 * (j * p->M + m)] = ft.lam[m].real();
        djm[2 * (j * p->M + m) + 1] = ft.lam[m].imag();
      }
    cm = std::max(cm, ft.cond);
    if (!why.empty()) {
      if (cond_max) *cond_max = cm;
      return fail(AAO_ENODIAG, why);
    }
  }
  if (cond_max) *cond_max = cm;
  return AAO_OK;
}

aao_status aao_collocation(aao_plan_t p, double* nodes, double* Q) {
  if (!p) return fail(AAO_EINVAL, "null plan");
  if (nodes) std::copy(p->t.begin(), p->t.end(), nodes);
  if (Q) std::copy(p->Q.begin(), p->Q.end(), Q);
  return AAO_OK;
}

void aao_destroy(aao_plan_t p) {
  if (!p) return;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  for (auto& t : p->pending) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (auto e : p->pool) (void)hipEventDestroy(e);
  if (p->run_a) (void)hipEventDestroy(p->run_a);
  if (p->dtab) (void)hipFree(p->dtab);
  if (p->htab) (void)hipHostFree(p->htab);
  if (p->hread) (void)hipHostFree(p->hread);
  if (p->hlist) (void)hipHostFree(p->hlist);
  if (p->hgm) (void)hipHostFree(p->hgm);
  for (auto e : p->slot_ev)
    if (e) (void)hipEventDestroy(e);
  delete p;
}

}  // extern "C"
