// Kernel-side interface of the alpha-circulant sweep (internal to libaao.so).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace aao {

constexpr int kMaxTaps = 32;
constexpr int kMaxM = 8;
constexpr int kBlock = 256;

// Periodic grid: n = y * nx + x, N = nx * ny.
struct Geo {
  int nx, ny, N;
};

// Stencil taps: (A v)[n] = sum_t c[t] v[wrap(x + dx[t], y + dy[t])].
struct Taps {
  int n;
  int dx[kMaxTaps];
  int dy[kMaxTaps];
  double c[kMaxTaps];
};

// Per shifted system state of the batched Krylov solvers.
struct SysState {
  int active;     // 1 while iterating
  int iters;      // iterations done when it stopped
  int flag;       // 0 converged, 1 hit the iteration cap, 2 breakdown
  int breakdown;  // set by an update kernel, consumed by the next matvec kernel
  int stop_pass;  // fused COCG: the pass that stopped the system (INT_MAX while active)
  double2 rho;    // BiCGStab: rho_k
  double2 alpha;  // BiCGStab, COCG: alpha_k
  double2 omega;  // BiCGStab: omega_k
  double2 beta;   // COCG: beta_k
  double2 gamma;  // COCG: gamma_k = r_k^T r_k
  double2 alpha_prev;  // COCG, scalar kernel between passes: alpha_{k-1}
  double bb;      // ||b||^2
  double rr;      // ||r_k||^2
  double2 gamma2[2];  // COCG, fused scalar update: gamma_k and alpha_k by parity of k
  double2 alpha2[2];
};

// State of a system before its first Krylov iteration.
__host__ __device__ inline SysState fresh_state() {
  SysState z{};
  z.active = 1;
  z.iters = 0;
  z.flag = 0;
  z.breakdown = 0;
  z.stop_pass = 0x7fffffff;
  z.rho = double2{1.0, 0.0};
  z.alpha = double2{1.0, 0.0};
  z.omega = double2{1.0, 0.0};
  return z;
}

// Single-pass COCG over 2D tiles (row a3).  Pass k reads R[k&1], P[(k+1)&1]
// and X, writes R[(k+1)&1], P[k&1] and X; the LDS tile holds p on a two-hop
// halo and r_{k+1} on a one-hop halo so that s = (I - cA) p and
// w = (I - cA) r_{k+1} need no extra global vector.
struct CgArgs {
  void* X;
  void* R[2];
  void* P[2];
  const double2* shift;
  SysState* st;
  double* part;             // [5][num_sys][ntiles]
  const int* sys_list;      // active systems of this launch
  unsigned long long* work;
  Geo g;
  Taps taps;
  int num_sys;
  int TX, TY, ntx, nty, ntiles, Rx, Ry;
  // ceil(2^40 / d) for exact division by ntx, TX, the two-hop width
  // TX + 4 Rx and the side-ring width 4 Rx (0 when Rx = 0)
  unsigned long long m_ntx, m_tx, m_pw, m_hw;
  int xcd_band;  // ntiles / 8 when tiles are banded per XCD, else 0
  int fused;     // 1: each pass advances the scalars itself (partials double-buffered)
  // fused: tile count of the pass that wrote the partials this pass reduces
  // (the tiling may change between passes) and the offset between the two
  // partial buffers (5 num_sys times the larger tile count)
  int ntiles_prev;
  size_t part_stride;
  // first init pass of a solve: workgroup row y is system y (every system
  // active), and tile 0 writes its fresh state and init_list[y] = y
  int* init_list;
  double tol2;
  // nullable, [num_sys]: a system stops once ||r||^2 <= tol2 max(||b||^2,
  // bbfloor[s]), i.e. at the relative tolerance or an absolute floor
  const double* bbfloor;
  int maxit;
  // fused passes: when snap_row >= 0 the launch has one more row of
  // workgroups (row snap_row == the active count); its first workgroup lists
  // the systems with stop_pass > snap_k (still iterating after pass snap_k)
  // into snap_list, then writes their count and snap_tag to snap_host
  int snap_row, snap_k, snap_n, snap_tag;
  int* snap_list;
  int* snap_host;
};

// Forward transform + fused residual (rows a1, a2).
struct FwdArgs {
  const double* u;      // u (or lambda) [B][L][M][N], or r when the input is a residual
  const double* w0;     // u0 [B][N] (primal) or g_last [B][N] (adjoint)
  const double* frc;    // source b at the collocation times [B][L][M][N] or null (primal only)
  void* out;            // x1 [B][Lh][M][N] complex (double2 or float2)
  const double* scale;  // [L] scaling applied before the DFT over l
  const double2* tw;    // [L/2] e^{-2 pi i k / L}
  const double2* mix;   // [Lh][M][M] per-frequency node transform
  double* part;         // per-workgroup sum of r^2
  Geo g;
  Taps taps;            // A (primal) or A^T (adjoint)
  double q[kMaxM * kMaxM];  // Q (primal) or Q^T (adjoint), row-major
  double dt;
  int L, logL, Lh, TN, logTN;
  int hx;               // halo width of the staged residual (set by the launcher)
  int mixo;             // LDS offset (doubles) of the staged node transforms, -1: read
                        // from global memory (set by the launcher)
};

// Inverse transform + update (row a4).
struct BwdArgs {
  const void* in;       // x2 [B][Lh][M][N] complex (double2 or float2)
  double* u;            // updated in place, or receives delta
  const double* scale;  // [L] scaling applied after the inverse DFT
  const double2* tw;
  const double2* mix;   // [Lh][M][M]
  double* part;         // per-workgroup max |delta| over the monitored step
  Geo g;
  int L, logL, Lh, TN, logTN;
};

// Batched Krylov solvers (row a3).
struct KrylovArgs {
  void* X;       // solution
  void* R;       // residual (holds the right-hand side on entry)
  void* P[2];    // search directions (double-buffered: the matvec reads halos)
  void* V[2];    // BiCGStab: A p (double-buffered), COCG: V[0] = A p
  void* Rh;      // BiCGStab: shadow residual
  void* S;       // BiCGStab: s
  void* T;       // BiCGStab: A s
  const double2* shift;  // [num_sys] shifted operator is I - shift * A
  SysState* st;
  double* part;  // [quantity][num_sys][wps_stride]
  unsigned long long* work;  // element counters per kernel class
  const int* sys_list;       // systems of this launch (grid.y entries)
  Geo g;
  Taps taps;
  // BiCGStab: wps workgroups per system, each over chunk points; wps may grow
  // between iterations as systems drop out.  Partial sums have a fixed
  // stride; wps_rho is the count that wrote rho and ||r||^2 (the previous
  // iteration's last kernel), wps_bb the count of the first iteration.
  int num_sys, wps, chunk, wps_stride, wps_rho, wps_bb;
  double tol2;
  const double* bbfloor;  // nullable, [num_sys]: as in CgArgs
  int maxit;
};

// A spatial dimension of length n that is not a power of two is transformed
// by Bluestein's chirp-z algorithm: cyclic convolutions of length P (a power
// of two, P >= 2n - 1).  W[k] = e^{+2 pi i k / P} (k < P); ch[j] = e^{-i pi
// j^2 / n} (j < n); Bf, Bi: length-P DFTs of the forward filter (conj(ch) at
// m and P - m) and of the inverse filter (ch).  P = 0: radix-2 directly.
struct BlueDim {
  int P, logP;
  const double2 *W, *ch, *Bf, *Bi;
};

// Spatial-FFT direct solve (row a3 for periodic constant-coefficient A).
struct FftArgs {
  void* R;                // right-hand sides, overwritten (2D)
  void* X;                // solutions
  const double2* shift;   // [num_sys]
  const double2* Wx;      // e^{+2 pi i k / nx}, k < nx
  const double2* Wy;      // e^{+2 pi i k / ny}, k < ny
  Taps taps;
  int nx, ny, N, lognx, logny;
  int px2, py2;           // nx / ny is a power of two
  int diag;               // some tap has both offsets nonzero
  int rows, cols;         // rows / columns per workgroup in the 2D passes (divide ny / nx)
  double norm;            // nx * ny
  BlueDim bx, by;         // Bluestein data of x / y (P = 0 where n is a power of two)
};

// Partial-sum quantities of the Krylov kernels: part[q][system][chunk].
enum PartialQ {
  QP_RHO0_RE = 0, QP_RHO0_IM, QP_RHO1_RE, QP_RHO1_IM, QP_RR0, QP_RR1, QP_A_RE, QP_A_IM,
  QP_B_RE, QP_B_IM, QP_TT, QP_BB, QP_COUNT
};

enum KernelClass {
  KC_FWD = 0, KC_BWD, KC_COCG_A, KC_COCG_B, KC_BICG_1, KC_BICG_2, KC_BICG_3,
  KC_FFT_INNER, KC_RESIDUAL, KC_MISC, KC_INIT, KC_GRAD, KC_GMRES, KC_BICG_WG
};

// Launchers (return hipSuccess or the launch error).
hipError_t launch_fwd(int M, bool adj, bool from_r, bool out_f32, const FwdArgs& a, int B,
                      hipStream_t st);
hipError_t launch_bwd(int M, bool adj, bool to_delta, bool in_f32, const BwdArgs& a, int B,
                      hipStream_t st);
hipError_t launch_residual(int M, bool adj, const FwdArgs& a, double* r_out, int B, hipStream_t st);
hipError_t launch_finalize(const double* part_sum, int n_sum, const double* part_max, int n_max,
                           double* out, hipStream_t st);
hipError_t launch_init_u(double* u, const double* u0, int B, int L, int M, int N, hipStream_t st);
// launch_finalize plus the sweep's iteration statistics, all also written to
// pinned host memory rep[0..6], then tag to rep[8] (as an int).
hipError_t launch_sweep_report(const double* ps, int ns, const double* pm, int nm, double* out, const SysState* sst,
                               int nsys, bool cocg, double* rep, int tag, hipStream_t st);
hipError_t launch_last_node(const double* u, double* out, int B, int L, int M, int N, hipStream_t st);
hipError_t launch_fill(double* p, double v, int64_t n, hipStream_t st);
hipError_t launch_norms_bn(const double* v, int B, int N, double* part, int nparts,
                           hipStream_t st);
// The same per instance: part[2 (b nparts + blk) + {0, 1}] for v + b N.
hipError_t launch_norms_per_b(const double* v, int B, int N, double* part, int nparts, hipStream_t st);
hipError_t launch_wnorms(int M, const FwdArgs& a, int B, double* part, int nparts, hipStream_t st);
hipError_t launch_cg_init(bool f32, const CgArgs& a, int nact, hipStream_t st);
hipError_t launch_cg_pass(bool f32, const CgArgs& a, int k, int nact, hipStream_t st);

// Outer flexible GMRES (Gram-Schmidt over [B][D] FP64 vectors, basis vector i
// at i * stride): part[(b nblk + blk) K + i] with K = gmres_bucket(nvec) holds
// block shares of <V_i[b], t[b]>; out = s[b] in + sum_i c[b][i] V_i with
// block shares of ||out[b]||^2 in part[b nblk + blk] (part may be null).
constexpr int kGmresMax = 32;
int gmres_bucket(int nvec);
hipError_t launch_mdot(const double* V, size_t stride, int nvec, const double* t, int64_t D, int B, double* part,
                       int nblk, hipStream_t st);
hipError_t launch_maxpy(double* out, const double* in, const double* s, const double* V, size_t stride, int nvec,
                        const double* c, int64_t D, int B, double* part, int nblk, hipStream_t st);
hipError_t launch_cg_scalars(const CgArgs& a, int k, int nact, hipStream_t st);
// After the last pass of a solve with a scalar kernel between passes: x of the
// systems (all nsys) whose last pass left x alone gets that pass's update.
hipError_t launch_cg_xfix(bool f32, const CgArgs& a, int nsys, hipStream_t st);
size_t cg_lds_bytes(bool f32, const CgArgs& a);
int cg_ring_slots(const CgArgs& a);
hipError_t launch_bicg(int phase, bool f32, const KrylovArgs& a, int k, int nact, hipStream_t st);
// Phases 1 and 2 of the batched BiCGStab on the COCG tiles of g (2D; every
// tile one chunk: a.wps == g.ntiles); bicg_tiled_fits says whether g allows it.
bool bicg_tiled_fits(const CgArgs& g);
hipError_t launch_bicg_tiled(int phase, bool f32, const CgArgs& g, const KrylovArgs& a, int k, int nact,
                             hipStream_t st);
// Fresh state for systems 0 .. num_sys - 1, and list[i] = i when list is given
// (every system starts active).
hipError_t launch_krylov_init(const KrylovArgs& a, hipStream_t st, int* list = nullptr);
// BiCGStab with one workgroup per system (all nsys systems, every iteration in
// one launch) for systems small enough to sit in one workgroup's registers.
bool bicg_wg_fits(int N);
hipError_t launch_bicg_wg(bool f32, const KrylovArgs& a, int nsys, hipStream_t st);
hipError_t launch_fft_solve(bool f32, const FftArgs& a, int nsys, hipStream_t st);
// LDS slots of one transform line of n elements (one pad slot per eight).
inline int fft_pad_line(int n) { return n + (n >> 3); }
hipError_t launch_compact_active(const SysState* st, int n, int* list, int* count_tag, int tag, hipStream_t s);
hipError_t launch_copy_c128_in(void* dst, bool f32, const double* src, int64_t n, hipStream_t st);
hipError_t launch_copy_c128_out(double* dst, const void* src, bool f32, int64_t n,
                                hipStream_t st);
hipError_t launch_grad(int M, const double* u, const double* lam, double* gu0, double* part,
                       const Taps& dtaps, const double* q, double dt, const Geo& g, int B,
                       int L, int nblk, hipStream_t st);
hipError_t launch_grad_finalize(const double* part, int nblk, int B, double* gnu,
                                hipStream_t st);

}  // namespace aao
