// HIP kernels of the alpha-circulant preconditioned Richardson sweep (gfx950).
//
// Layouts (all C order): u, r [B][L][M][N] FP64; frequency data x1, x2 and the
// Krylov vectors [B][Lh][M][N] complex (double2 or float2), Lh = L/2 + 1 (only
// the non-redundant half of the DFT over l is kept: the time data is real, so
// frequency L-j is the conjugate of frequency j).
//
// The DFT over l runs in LDS on a tile of TN consecutive spatial points: two
// real columns (n, n+1) are packed into one complex column, transformed by an
// in-place radix-2 FFT (bit-reversed load, natural-order result) and separated
// again; the M x M node transform of each frequency is applied on the way out.
#include <algorithm>
#include <cstdlib>

#include "aao_kernels.hpp"
#include "aao_device.hpp"

namespace aao {

namespace {

using namespace dev;

// ----------------------------------------------------------------------------
// Staged all-at-once residual of one tile (TN points of one grid row, N a
// multiple of TN) for k_fwd: r_{l,m} = w - C u at every (l, m) of the tile,
// scaled and left in the LDS planes (bit-reversed rows, the layout of the DFT
// over l).  Phase 1 copies u of the tile into the planes and the hx points on
// either side of the tile (periodic) into hal [lr][M][2 hx]; phase 2 forms the
// residual rows of this thread in registers (stencil taps with dy = 0, the
// node's own value and the coupling u_{l-1,M} (lambda_{l+1,.} for C^T) from
// LDS, other taps and the source from global memory); phase 3 overwrites the
// planes with the scaled rows.  The arithmetic is that of the unstaged loop,
// operation for operation.
constexpr int kStageRows = 4;  // rows l per thread: L TN <= kStageRows kBlock
#ifndef AAO_FWD_STG_WAVES
#define AAO_FWD_STG_WAVES 5  // waves per SIMD asked for the staged forward transform
#endif

// The per-frequency node transforms [Lh][M][M] are copied to LDS (at double
// offset mixo, real and imaginary parts side by side) where they fit
// kMixLdsBytes: read from global memory, the M^2 coefficients of every
// output item miss L1 once the tile data streams through it.
constexpr size_t kMixLdsBytes = 8192;
template <int M>
__device__ __forceinline__ void stage_mix(const double2* mix, int Lh, int mixo) {
  extern __shared__ double lds[];
  if (mixo < 0) return;
  for (int i = threadIdx.x; i < Lh * M * M; i += kBlock) {
    const double2 v = mix[i];
    lds[mixo + 2 * i] = v.x;
    lds[mixo + 2 * i + 1] = v.y;
  }
}
__device__ __forceinline__ double2 mix_lds(int mixo, int i) {
  extern __shared__ double lds[];
  return mk(lds[mixo + 2 * i], lds[mixo + 2 * i + 1]);
}

template <int M, bool ADJ, int NT>
__device__ __forceinline__ void stage_residual(const FwdArgs& a, int b, int n0, int nl, int x, int y,
                                               const int* nbs, int cim_off, int hal_off, double& res2) {
  extern __shared__ double lds[];  // the transform's dynamic LDS (planes, twiddles, halo)
  const int TN = a.TN, P = TN >> 1, L = a.L, N = a.g.N, nx = a.g.nx, hx = a.hx;
  const int n = n0 + nl;
  const int x0 = n0 % nx, row0 = n0 - x0;
  const int step = kBlock >> a.logTN;
  const int l0 = threadIdx.x >> a.logTN;
  // every LDS access is lds[offset]: the planes start at 0 and cim_off, the
  // halo at hal_off; own = this thread's point in its plane
  const int own = ((nl & 1) ? cim_off : 0) + (nl >> 1);
  const double* ub = a.u + (size_t)b * L * M * N;

  // phase 1: the tile and its halo (the tile's loads all issued before the
  // first LDS store: row by row each row's loads waited for the previous
  // row's stores)
  double cv[kStageRows][M];
#pragma unroll
  for (int i = 0; i < kStageRows; ++i) {
    const int l = l0 + i * step;
#pragma unroll
    for (int m = 0; m < M; ++m) cv[i][m] = (l < L) ? ub[((size_t)l * M + m) * N + n] : 0.0;
  }
#pragma unroll
  for (int i = 0; i < kStageRows; ++i) {
    const int l = l0 + i * step;
    if (l < L) {
      const int lr = bitrev(l, a.logL);
#pragma unroll
      for (int m = 0; m < M; ++m) lds[own + (lr * M + m) * P] = cv[i][m];
    }
  }
  const int hw = 2 * hx;
  for (int i = threadIdx.x; i < L * M * hw; i += kBlock) {
    const int k = i % hw, lm = i / hw;
    const int l = lm / M, m = lm - l * M;
    int xx = (k < hx) ? x0 - hx + k : x0 + TN + (k - hx);
    xx += (xx < 0) ? nx : 0;
    xx -= (xx >= nx) ? nx : 0;
    lds[hal_off + (bitrev(l, a.logL) * M + m) * hw + k] = ub[((size_t)l * M + m) * N + row0 + xx];
  }
  __syncthreads();

  // a tap along the row reads plane (q & 1) at q / 2 for a tile point q, or a
  // halo slot: offset and row stride (P in the planes, 2 hx in the halo);
  // stride 0 marks a tap read from global memory
  auto row_src = [&](int dx, int& off, int& stride) {
    int q = nl + dx;
    if (TN == nx) {  // the tile is the whole row: the periodic wrap stays inside
      q += (q < 0) ? TN : 0;
      q -= (q >= TN) ? TN : 0;
    }
    if (q >= 0 && q < TN) {
      off = ((q & 1) ? cim_off : 0) + (q >> 1);
      stride = P;
    } else {
      off = hal_off + ((q < 0) ? q + hx : hx + (q - TN));
      stride = hw;
    }
  };
  int toff[NT > 0 ? NT : 1];
  int tstr[NT > 0 ? NT : 1];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    toff[t] = 0;
    tstr[t] = 0;
    if (a.taps.dy[t] == 0) row_src(a.taps.dx[t], toff[t], tstr[t]);
  }

  // phase 2: residual rows in registers
  double rr[kStageRows][M];
#pragma unroll
  for (int i = 0; i < kStageRows; ++i) {
    const int l = l0 + i * step;
#pragma unroll
    for (int m = 0; m < M; ++m) rr[i][m] = 0.0;
    if (l < L) {
      const int lr = bitrev(l, a.logL);
      const size_t base = ((size_t)b * L + l) * M * (size_t)N;
      const double* ul = a.u + base;
      double v[M];
#pragma unroll
      for (int m = 0; m < M; ++m) v[m] = 0.0;
      auto tap = [&](double ct, int off, int str, int nb) {
        if (str) {
#pragma unroll
          for (int m = 0; m < M; ++m) v[m] = fma(ct, lds[off + (lr * M + m) * str], v[m]);
        } else {
#pragma unroll
          for (int m = 0; m < M; ++m) v[m] = fma(ct, ul[(size_t)m * N + nb], v[m]);
        }
      };
      if (NT > 0) {
#pragma unroll
        for (int t = 0; t < NT; ++t) tap(a.taps.c[t], toff[t], tstr[t], nbs[t]);
      } else {
        for (int t = 0; t < a.taps.n; ++t) {
          int off = 0, str = 0, nb = 0;
          if (a.taps.dy[t] == 0) row_src(a.taps.dx[t], off, str);
          else nb = wrap_index(x, y, a.taps.dx[t], a.taps.dy[t], a.g);
          tap(a.taps.c[t], off, str, nb);
        }
      }
      double f[M];  // source at the collocation times (eq. (collocation): dT Q b_l)
#pragma unroll
      for (int m = 0; m < M; ++m) f[m] = (!ADJ && a.frc) ? a.frc[base + (size_t)m * N + n] : 0.0;
#pragma unroll
      for (int m = 0; m < M; ++m) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < M; ++k) s = fma(a.q[m * M + k], v[k] + f[k], s);
        rr[i][m] = fma(a.dt, s, -lds[own + (lr * M + m) * P]);
      }
      if (!ADJ) {
        const double add = (l == 0) ? a.w0[(size_t)b * N + n]
                                    : lds[own + (bitrev(l - 1, a.logL) * M + (M - 1)) * P];  // u_{l-1, M}
#pragma unroll
        for (int m = 0; m < M; ++m) rr[i][m] += add;
      } else {
        if (l == L - 1) {
          rr[i][M - 1] += a.w0[(size_t)b * N + n];
        } else {
          const int ln = bitrev(l + 1, a.logL) * M;  // lambda_{l+1, .}
          double s = 0.0;
#pragma unroll
          for (int m = 0; m < M; ++m) s += lds[own + (ln + m) * P];
          rr[i][M - 1] += s;
        }
      }
#pragma unroll
      for (int m = 0; m < M; ++m) res2 = fma(rr[i][m], rr[i][m], res2);
    }
  }
  __syncthreads();

  // phase 3: the scaled residual replaces u in the planes
#pragma unroll
  for (int i = 0; i < kStageRows; ++i) {
    const int l = l0 + i * step;
    if (l < L) {
      const double sc = a.scale[l];
      const int lr = bitrev(l, a.logL);
#pragma unroll
      for (int m = 0; m < M; ++m) lds[own + (lr * M + m) * P] = rr[i][m] * sc;
    }
  }
}

// ----------------------------------------------------------------------------
// Forward transform with the fused all-at-once residual.
// MODE 0: r = w - C u computed on the fly; MODE 1: r read from memory.
// ADJ: residual of C^T (coupling from step l+1 into the last node, Q^T, A^T).
// NT > 0: the stencil has NT taps (unrolled, so all neighbour loads of a
// point are in flight together).
// STG (MODE 0, tiles inside one grid row): the tile's u for every (l, m) is
// staged in the LDS planes, with a halo of a.hx points on each side of the
// tile; taps along the row and the coupling between steps read LDS, taps into
// other rows read global memory (L2: the neighbouring rows' tiles run on the
// same XCD just before and after).
template <int M, bool ADJ, int MODE, typename OutV, int NT, bool STG>
// The staged form asks for five waves per SIMD (at most 96 VGPRs; the
// unstaged form is left to the compiler, which takes about 100).
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(STG ? AAO_FWD_STG_WAVES : 1)))
void k_fwd(FwdArgs a) {
  extern __shared__ double lds[];
  const int TN = a.TN, P = TN >> 1, L = a.L, N = a.g.N;
  const int b = blockIdx.y;
  // XCD-banded tile order (workgroup slot b runs on XCD b % 8): a contiguous
  // range of tiles per XCD keeps the stencil's neighbouring rows in its L2.
  int tile = blockIdx.x;
  if ((gridDim.x & 7) == 0) tile = (tile & 7) * (gridDim.x >> 3) + (tile >> 3);
  const int n0 = tile * TN;
  // planes: real columns n0 + 2p in cre, n0 + 2p + 1 in cim ([L][M][P] each,
  // l in bit-reversed order), then the twiddles
  const int plane = L * M * P + kPlanePad;
  double* cre = lds;
  double* cim = lds + plane;
  double* twr = lds + 2 * plane;
  double* twi = twr + (L >> 1);
  __shared__ double sh[4];
  for (int i = threadIdx.x; i < (L >> 1); i += kBlock) {
    twr[i] = a.tw[i].x;
    twi[i] = a.tw[i].y;
  }
  stage_mix<M>(a.mix, a.Lh, a.mixo);

  // TN divides kBlock, so the spatial point of a thread is the same in every
  // row l it visits: its coordinates and the unrolled taps' neighbour offsets
  // are computed once.  Two rows per loop trip (their loads in flight together)
  // also keep the register count below that of the per-row form.
  const int nl = threadIdx.x & (TN - 1);
  const int n = n0 + nl;
  const int x = n % a.g.nx, y = n / a.g.nx;
  int nbs[NT > 0 ? NT : 1];
#pragma unroll
  for (int t = 0; t < NT; ++t) nbs[t] = wrap_index(x, y, a.taps.dx[t], a.taps.dy[t], a.g);
  double* dst = ((nl & 1) ? cim : cre) + (nl >> 1);

  double res2 = 0.0;
  if constexpr (MODE == 0 && STG) {
    stage_residual<M, ADJ, NT>(a, b, n0, nl, x, y, nbs, plane, 2 * plane + L, res2);
  } else {
#ifndef AAO_FWD_ROW_UNROLL
#define AAO_FWD_ROW_UNROLL 2
#endif
#pragma unroll AAO_FWD_ROW_UNROLL
  for (int l = threadIdx.x >> a.logTN; l < L; l += (kBlock >> a.logTN)) {
    double rv[M];
#pragma unroll
    for (int m = 0; m < M; ++m) rv[m] = 0.0;
    if (n < N) {
      const size_t base = ((size_t)b * L + l) * M * (size_t)N;
      if (MODE == 1) {
#pragma unroll
        for (int m = 0; m < M; ++m) rv[m] = a.u[base + (size_t)m * N + n];
      } else {
        const double* ul = a.u + base;
        double v[M];
#pragma unroll
        for (int m = 0; m < M; ++m) v[m] = 0.0;
        auto tap = [&](int t, int nb) {
          const double ct = a.taps.c[t];
#pragma unroll
          for (int m = 0; m < M; ++m) v[m] = fma(ct, ul[(size_t)m * N + nb], v[m]);
        };
        if (NT > 0) {
#pragma unroll
          for (int t = 0; t < NT; ++t) tap(t, nbs[t]);
        } else {
          for (int t = 0; t < a.taps.n; ++t) tap(t, wrap_index(x, y, a.taps.dx[t], a.taps.dy[t], a.g));
        }
        double f[M];  // source at the collocation times (eq. (collocation): dT Q b_l)
#pragma unroll
        for (int m = 0; m < M; ++m) f[m] = (!ADJ && a.frc) ? a.frc[base + (size_t)m * N + n] : 0.0;
#pragma unroll
        for (int m = 0; m < M; ++m) {
          double s = 0.0;
#pragma unroll
          for (int k = 0; k < M; ++k) s = fma(a.q[m * M + k], v[k] + f[k], s);
          rv[m] = fma(a.dt, s, -ul[(size_t)m * N + n]);
        }
        if (!ADJ) {
          if (l == 0) {
            const double w0 = a.w0[(size_t)b * N + n];
#pragma unroll
            for (int m = 0; m < M; ++m) rv[m] += w0;
          } else {
            const double up = a.u[base - (size_t)N + n];  // u_{l-1, M}
#pragma unroll
            for (int m = 0; m < M; ++m) rv[m] += up;
          }
        } else {
          if (l == L - 1) {
            rv[M - 1] += a.w0[(size_t)b * N + n];
          } else {
            const double* un = ul + (size_t)M * N;  // lambda_{l+1, .}
            double s = 0.0;
#pragma unroll
            for (int m = 0; m < M; ++m) s += un[(size_t)m * N + n];
            rv[M - 1] += s;
          }
        }
#pragma unroll
        for (int m = 0; m < M; ++m) res2 = fma(rv[m], rv[m], res2);
      }
    }
    const double sc = a.scale[l];
    const int lr = bitrev(l, a.logL);
#pragma unroll
    for (int m = 0; m < M; ++m) dst[((size_t)lr * M + m) * P] = rv[m] * sc;
  }
  }

  const int ncol = M * P;
  lds_fft<false>(cre, cim, twr, twi, L, a.logL, ncol);

  OutV* out = reinterpret_cast<OutV*>(a.out);
  const int logP = a.logTN - 1;
  // frequencies 0 and L/2 (both self-conjugate) share an item, so that the
  // (L/2) P items fill the block once (L TN = 1024 within the LDS budget)
  auto emit = [&](int j, int p, auto&& mixw) __attribute__((always_inline)) {
    const int jm = (L - j) & (L - 1);
    double2 A[M], Bv[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int oz = j * ncol + m * P + p, ozc = jm * ncol + m * P + p;
      const double2 Z = mk(cre[oz], cim[oz]);
      const double2 Zc = mk(cre[ozc], cim[ozc]);
      A[m] = mk(0.5 * (Z.x + Zc.x), 0.5 * (Z.y - Zc.y));
      Bv[m] = mk(0.5 * (Z.y + Zc.y), -0.5 * (Z.x - Zc.x));
      if (ADJ) {
        A[m].y = -A[m].y;
        Bv[m].y = -Bv[m].y;
      }
    }
    const int n = n0 + 2 * p;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      double2 xa = mk(0, 0), xb = mk(0, 0);
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const double2 w = mixw(j, m * M + k);
        xa = cadd(xa, cmul(w, A[k]));
        xb = cadd(xb, cmul(w, Bv[k]));
      }
      const size_t o = (((size_t)b * a.Lh + j) * M + m) * (size_t)N + n;
      if (n < N) out[o] = from_d2<OutV>(xa);
      if (n + 1 < N) out[o + 1] = from_d2<OutV>(xb);
    }
  };
  auto emit_all = [&](auto&& mixw) __attribute__((always_inline)) {
    for (int idx = threadIdx.x; idx < max(L >> 1, 1) * P; idx += kBlock) {
      const int j = idx >> logP;
      const int p = idx & (P - 1);
      emit(j, p, mixw);
      if (j == 0 && L > 1) emit(L >> 1, p, mixw);
    }
  };
  if (a.mixo >= 0) emit_all([&](int j, int i) { return mix_lds(a.mixo + 2 * j * M * M, i); });
  else emit_all([&](int j, int i) { return (a.mix + (size_t)j * M * M)[i]; });
  if (MODE == 0) {
    double v[1] = {res2};
    block_sum<1>(v, sh);
    if (threadIdx.x == 0) a.part[(size_t)blockIdx.y * gridDim.x + tile] = v[0];
  }
}

// Residual only (row a1 on its own): r = w - C u written to memory.
template <int M, bool ADJ>
__global__ __launch_bounds__(kBlock) void k_residual(FwdArgs a, double* r_out, int B) {
  __shared__ double sh[4];
  const int L = a.L, N = a.g.N;
  const size_t total = (size_t)B * L * N;
  double res2 = 0.0;
  for (size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * kBlock) {
    const int n = (int)(idx % N);
    const size_t bl = idx / N;
    const int l = (int)(bl % L);
    const int b = (int)(bl / L);
    const size_t base = ((size_t)b * L + l) * M * (size_t)N;
    const double* ul = a.u + base;
    const int x = n % a.g.nx, y = n / a.g.nx;
    double v[M], rv[M];
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] = 0.0;
    for (int t = 0; t < a.taps.n; ++t) {
      const int nb = wrap_index(x, y, a.taps.dx[t], a.taps.dy[t], a.g);
#pragma unroll
      for (int m = 0; m < M; ++m) v[m] = fma(a.taps.c[t], ul[(size_t)m * N + nb], v[m]);
    }
    double f[M];
#pragma unroll
    for (int m = 0; m < M; ++m) f[m] = (!ADJ && a.frc) ? a.frc[base + (size_t)m * N + n] : 0.0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < M; ++k) s = fma(a.q[m * M + k], v[k] + f[k], s);
      rv[m] = fma(a.dt, s, -ul[(size_t)m * N + n]);
    }
    if (!ADJ) {
      const double add = (l == 0) ? a.w0[(size_t)b * N + n] : a.u[base - (size_t)N + n];
#pragma unroll
      for (int m = 0; m < M; ++m) rv[m] += add;
    } else {
      if (l == L - 1) {
        rv[M - 1] += a.w0[(size_t)b * N + n];
      } else {
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < M; ++m) s += ul[(size_t)(M + m) * N + n];
        rv[M - 1] += s;
      }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
      r_out[base + (size_t)m * N + n] = rv[m];
      res2 = fma(rv[m], rv[m], res2);
    }
  }
  double v[1] = {res2};
  block_sum<1>(v, sh);
  if (threadIdx.x == 0) a.part[blockIdx.x] = v[0];
}

// ----------------------------------------------------------------------------
// Inverse transform and update.  MODE 0: u += delta; MODE 1: u = delta.
template <int M, bool ADJ, int MODE, typename InV>
__global__ __launch_bounds__(kBlock) void k_bwd(BwdArgs a) {
  extern __shared__ double lds[];
  const int TN = a.TN, P = TN >> 1, L = a.L, N = a.g.N;
  const int b = blockIdx.y;
  // XCD-banded tile order (workgroup slot b runs on XCD b % 8): a contiguous
  // range of tiles per XCD keeps the stencil's neighbouring rows in its L2.
  int tile = blockIdx.x;
  if ((gridDim.x & 7) == 0) tile = (tile & 7) * (gridDim.x >> 3) + (tile >> 3);
  const int n0 = tile * TN;
  const int plane = L * M * P + kPlanePad;  // as in k_fwd
  double* cre = lds;
  double* cim = lds + plane;
  double* twr = lds + 2 * plane;
  double* twi = twr + (L >> 1);
  __shared__ double sh[4];
  for (int i = threadIdx.x; i < (L >> 1); i += kBlock) {
    twr[i] = a.tw[i].x;
    twi[i] = a.tw[i].y;
  }
  const int ncol = M * P;
  const InV* in = reinterpret_cast<const InV*>(a.in);

  const int logP = a.logTN - 1;
  // as in k_fwd, frequencies 0 and L/2 share an item
  auto take = [&](int j, int p) {
    const int n = n0 + 2 * p;
    const InV* ij = in + ((size_t)b * a.Lh + j) * M * N + n;
    double2 xa[M], xb[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      xa[m] = (n < N) ? to_d2(ij[m * N]) : mk(0, 0);
      xb[m] = (n + 1 < N) ? to_d2(ij[m * N + 1]) : mk(0, 0);
    }
    const double2* mx = a.mix + (size_t)j * M * M;
    const bool selfconj = (j == 0) || (2 * j == L);
    const int jr = bitrev(j, a.logL);
    const int jmr = bitrev((L - j) & (L - 1), a.logL);
#pragma unroll
    for (int m = 0; m < M; ++m) {
      double2 ya = mk(0, 0), yb = mk(0, 0);
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const double2 w = mx[m * M + k];
        ya = cadd(ya, cmul(w, xa[k]));
        yb = cadd(yb, cmul(w, xb[k]));
      }
      if (ADJ) {
        ya.y = -ya.y;
        yb.y = -yb.y;
      }
      if (selfconj) {
        ya.y = 0.0;
        yb.y = 0.0;
      }
      const int o = jr * ncol + m * P + p;
      cre[o] = ya.x - yb.y;
      cim[o] = ya.y + yb.x;
      if (!selfconj) {
        const int oc = jmr * ncol + m * P + p;
        cre[oc] = ya.x + yb.y;
        cim[oc] = yb.x - ya.y;
      }
    }
  };
  for (int idx = threadIdx.x; idx < max(L >> 1, 1) * P; idx += kBlock) {
    const int j = idx >> logP;
    const int p = idx & (P - 1);
    take(j, p);
    if (j == 0 && L > 1) take(L >> 1, p);
  }
  lds_fft<true>(cre, cim, twr, twi, L, a.logL, ncol);

  // as in k_fwd every row lm this thread visits is at the same spatial point.
  // Its rows are taken in batches of kUpdRows, each read whole before any of
  // it is written: row by row, each load of u would wait for the previous
  // row's store (the compiler cannot tell the rows apart), one memory round
  // trip per row.  (A thread has at most 12 rows, L M TN <= 3072, unless TN
  // is at its minimum of 2; eight rows per batch keep the register count of
  // the transform.)
  const int lmon = ADJ ? 0 : L - 1;
  double dmax = 0.0;
  const int nl = threadIdx.x & (TN - 1);
  const int n = n0 + nl;
  if (n < N) {
    const double* src = ((nl & 1) ? cim : cre) + (nl >> 1);
    double* ub = a.u + (size_t)b * L * M * N + n;  // this instance's u at point n
    const int step = kBlock >> a.logTN;
    constexpr int kUpdRows = 8;
    for (int lm0 = threadIdx.x >> a.logTN; lm0 < L * M; lm0 += kUpdRows * step) {
      // the scales first, then u (loads complete in order: waiting for a
      // scale then leaves every u load in flight)
      double d[kUpdRows], uo[kUpdRows];
#pragma unroll
      for (int i = 0; i < kUpdRows; ++i) {
        const int lm = lm0 + i * step;
        d[i] = (lm < L * M) ? a.scale[lm / M] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < kUpdRows; ++i) {
        const int lm = lm0 + i * step;
        uo[i] = (MODE == 0 && lm < L * M) ? ub[(size_t)lm * N] : 0.0;
      }
      // all results before the first store (each guarded store would
      // otherwise wait for every memory operation issued before it)
#pragma unroll
      for (int i = 0; i < kUpdRows; ++i) {
        const int lm = lm0 + i * step;
        const double sv = (lm < L * M) ? src[lm * P] : 0.0;
        const double dd = sv * d[i];  // delta (d holds the scale here)
        if (lm < L * M && lm / M == lmon) dmax = fmax(dmax, fabs(dd));
        uo[i] = (MODE == 0) ? fma(sv, d[i], uo[i]) : dd;  // u + delta in one rounding
      }
#pragma unroll
      for (int i = 0; i < kUpdRows; ++i) {
        const int lm = lm0 + i * step;
        if (lm < L * M) ub[(size_t)lm * N] = uo[i];
      }
    }
  }
  dmax = block_max(dmax, sh);
  if (threadIdx.x == 0) a.part[(size_t)blockIdx.y * gridDim.x + tile] = dmax;
}

// ----------------------------------------------------------------------------
// This thread's share (indices threadIdx.x + kBlock j) of the sum / max of
// x[0 .. n): eight independent accumulators, so eight loads are in flight per
// step instead of one chain of dependent adds (tens of thousands of
// per-workgroup partials otherwise take 0.1-0.4 ms to add up); the order is
// fixed by n.
__device__ __forceinline__ double strided_sum(const double* x, int n) {
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int i = threadIdx.x;
  for (; i + 7 * kBlock < n; i += 8 * kBlock) {
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] += x[i + q * kBlock];
  }
  for (; i < n; i += kBlock) a[0] += x[i];
  return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

__device__ __forceinline__ double strided_max(const double* x, int n) {
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int i = threadIdx.x;
  for (; i + 7 * kBlock < n; i += 8 * kBlock) {
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] = fmax(a[q], x[i + q * kBlock]);
  }
  for (; i < n; i += kBlock) a[0] = fmax(a[0], x[i]);
  return fmax(fmax(fmax(a[0], a[1]), fmax(a[2], a[3])), fmax(fmax(a[4], a[5]), fmax(a[6], a[7])));
}

__global__ __launch_bounds__(kBlock) void k_finalize(const double* ps, int ns, const double* pm,
                                                     int nm, double* out) {
  __shared__ double sh[4];
  const double s = strided_sum(ps, ns);
  double mx = strided_max(pm, nm);
  double v[1] = {s};
  block_sum<1>(v, sh);
  mx = block_max(mx, sh);
  if (threadIdx.x == 0) {
    out[0] = v[0];
    out[1] = mx;
  }
}

// Complex words per element that the COCG passes of a system with ks
// iterations moved (x moves every other pass; see the pass kernel).
__device__ __forceinline__ double cocg_words_dev(int ks) {
  double w = 0;
  for (int k = 0; k < ks; ++k) {
    w += (k > 0) ? 4 : 3;
    if (k & 1) w += (k >= 3) ? 2 : 1;
  }
  if (ks & 1) w += (ks >= 3) ? 3 : 2;
  return w;
}

// End of a sweep: the norms of k_finalize, and the per-system iteration
// statistics (sum, sum of max(iters - 1, 0), max, count with flag != 0, and
// with cocg the bytes words), written to out and then to pinned host memory
// rep[0 .. 6] followed, after a system-scope fence, by the tag in rep[8].
__global__ __launch_bounds__(kBlock) void k_sweep_report(const double* ps, int ns, const double* pm, int nm,
                                                         double* out, const SysState* st, int nsys, int cocg,
                                                         double* rep, int tag) {
  __shared__ double sh[4 * 8];
  const double s = strided_sum(ps, ns);
  double mx = strided_max(pm, nm);
  double v[5] = {s, 0.0, 0.0, 0.0, 0.0};
  double imax = 0.0;
  for (int i = threadIdx.x; i < nsys; i += kBlock) {
    const int it = st[i].iters;
    v[1] += it;
    v[2] += it > 1 ? it - 1 : 0;
    v[3] += st[i].flag != 0 ? 1.0 : 0.0;
    if (cocg) v[4] += cocg_words_dev(it);
    imax = fmax(imax, (double)it);
  }
  block_sum<5>(v, sh);
  mx = block_max(mx, sh);
  imax = block_max(imax, sh);
  if (threadIdx.x == 0) {
    out[0] = v[0];
    out[1] = mx;
    rep[0] = v[0];
    rep[1] = mx;
    rep[2] = v[1];
    rep[3] = v[2];
    rep[4] = imax;
    rep[5] = v[3];
    rep[6] = v[4];
    __threadfence_system();
    reinterpret_cast<volatile int*>(rep + 8)[0] = tag;
  }
}

__global__ void k_init_u(double* u, const double* u0, int B, int L, int M, int N) {
  const size_t total = (size_t)B * L * M * N;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int n = (int)(i % N);
    const int b = (int)(i / ((size_t)L * M * N));
    u[i] = u0[(size_t)b * N + n];
  }
}

// out[b][n] = u[b][L-1][M-1][n]: the last node of the last step (the next
// window's initial value).
__global__ void k_last_node(const double* u, double* out, int B, int L, int M, int N) {
  const size_t total = (size_t)B * N;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const size_t b = i / N, n = i % N;
    out[i] = u[((b * L + (L - 1)) * M + (M - 1)) * (size_t)N + n];
  }
}

__global__ void k_fill(double* p, double v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// part[2*blk] = sum v^2, part[2*blk+1] = max |v| over a grid-stride share;
// grid row y covers v + y n into part + 2 y gridDim.x.
__global__ __launch_bounds__(kBlock) void k_norms(const double* v, int64_t n, double* part) {
  __shared__ double sh[4];
  v += (int64_t)blockIdx.y * n;
  part += 2 * (size_t)gridDim.x * blockIdx.y;
  double s = 0.0, mx = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    s = fma(v[i], v[i], s);
    mx = fmax(mx, fabs(v[i]));
  }
  double t[1] = {s};
  block_sum<1>(t, sh);
  mx = block_max(mx, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = t[0];
    part[2 * blockIdx.x + 1] = mx;
  }
}

// ||w||^2 and max |w| of the all-at-once right-hand side w_{l,m} = [l = 0] u0 +
// dT sum_k Q_mk b_{l,k} (eq. (collocation)) over a grid-stride share of
// (b, l, n): part[2 blk], part[2 blk + 1].
template <int M>
__global__ __launch_bounds__(kBlock) void k_wnorms(FwdArgs a, int B, double* part) {
  __shared__ double sh[4];
  const int L = a.L, N = a.g.N;
  const size_t total = (size_t)B * L * N;
  double s2 = 0.0, mx = 0.0;
  for (size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x; idx < total; idx += (size_t)gridDim.x * kBlock) {
    const int n = (int)(idx % N);
    const size_t bl = idx / N;
    const int l = (int)(bl % L);
    const int b = (int)(bl / L);
    const size_t base = ((size_t)b * L + l) * M * (size_t)N;
    const double u0 = (l == 0) ? a.w0[(size_t)b * N + n] : 0.0;
    double f[M];
#pragma unroll
    for (int m = 0; m < M; ++m) f[m] = a.frc ? a.frc[base + (size_t)m * N + n] : 0.0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < M; ++k) s = fma(a.q[m * M + k], f[k], s);
      const double w = fma(a.dt, s, u0);
      s2 = fma(w, w, s2);
      mx = fmax(mx, fabs(w));
    }
  }
  double v[1] = {s2};
  block_sum<1>(v, sh);
  mx = block_max(mx, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = v[0];
    part[2 * blockIdx.x + 1] = mx;
  }
}

// ----------------------------------------------------------------------------
// Batched Krylov solvers for (I - c_s A) x_s = b_s.  Grid (wps, num_sys); each
// workgroup owns one chunk of one system.  Scalars are reduced from per-chunk
// partial sums by every workgroup in the same fixed order (bitwise identical),
// so no grid-wide synchronisation and no host round trip is needed.
// (qpart, reduce_parts and write_parts: aao_device.hpp)


// Shifted operator at point n on a vector given through an accessor.
template <typename V, typename F>
__device__ __forceinline__ V shifted_apply(const KrylovArgs& a, int n, V center, V shift, F get) {
  const int x = n % a.g.nx, y = n / a.g.nx;
  V acc = vzero<V>();
  for (int t = 0; t < a.taps.n; ++t) {
    const int nb = wrap_index(x, y, a.taps.dx[t], a.taps.dy[t], a.g);
    acc = vadd(acc, vscale(get(nb), (decltype(center.x))a.taps.c[t]));
  }
  return vsub(center, vmul(shift, acc));
}

// BiCGStab (Hermitian inner products <a, b> = sum conj(a) b), r_hat = r_0.
// Phase 1: convergence test, beta = (rho_k / rho_{k-1}) (alpha / omega),
// p = r + beta (p_old - omega v_old), v = (I - cA) p, partial <r_hat, v>.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bicg1(KrylovArgs a, int k) {
  using V = typename cvec<T>::type;
  __shared__ double sh[4 * 8];
  const int s = a.sys_list[blockIdx.y];
  SysState* st = a.st + s;
  // One read of the flag per workgroup: kernel A may clear it concurrently
  // (workgroup 0, on convergence), and every thread must take the same path.
  __shared__ int act;
  if (threadIdx.x == 0) act = st->active;
  __syncthreads();
  if (!act) return;
  const int cur = k & 1;
  const size_t off = (size_t)s * a.g.N;
  const V* R = reinterpret_cast<const V*>(a.R) + off;
  V* Rh = reinterpret_cast<V*>(a.Rh) + off;
  V* Pn = reinterpret_cast<V*>(a.P[k & 1]) + off;
  const V* Po = reinterpret_cast<const V*>(a.P[(k + 1) & 1]) + off;
  V* Vn = reinterpret_cast<V*>(a.V[k & 1]) + off;
  const V* Vo = reinterpret_cast<const V*>(a.V[(k + 1) & 1]) + off;
  const V sft = from_d2<V>(a.shift[s]);
  const int n0 = blockIdx.x * a.chunk;
  const int n1 = min(a.g.N, n0 + a.chunk);
  double hv_re = 0, hv_im = 0;
  if (k == 0) {
    double bb = 0;
    for (int n = n0 + threadIdx.x; n < n1; n += kBlock) {
      const V r = R[n];
      const V v = shifted_apply(a, n, r, sft, [&](int i) { return R[i]; });
      Rh[n] = r;
      Pn[n] = r;
      Vn[n] = v;
      hv_re += (double)r.x * v.x + (double)r.y * v.y;
      hv_im += (double)r.x * v.y - (double)r.y * v.x;
      bb += (double)r.x * r.x + (double)r.y * r.y;
    }
    // rho_0 = <r_hat, r> = ||b||^2 (real)
    double w[4] = {hv_re, hv_im, bb, bb};
    const int qs[4] = {QP_A_RE, QP_A_IM, QP_BB, QP_RHO0_RE};
    write_parts<4>(a, qs, s, blockIdx.x, w, sh);
    if (threadIdx.x == 0) qpart(a, QP_RHO0_IM, s)[blockIdx.x] = 0.0;
  } else {
    const int qs[4] = {QP_RHO0_RE + 2 * cur, QP_RHO0_IM + 2 * cur, QP_RR0 + cur, QP_BB};
    const int nw[4] = {a.wps_rho, a.wps_rho, a.wps_rho, a.wps_bb};
    double v[4];
    reduce_parts<4>(a, qs, nw, s, v, sh);
    const bool conv = v[2] <= a.tol2 * (a.bbfloor ? fmax(v[3], a.bbfloor[s]) : v[3]);
    if (conv || k >= a.maxit || st->breakdown) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->active = 0;
        st->iters = k;
        st->flag = conv ? 0 : (st->breakdown ? 2 : 1);
      }
      return;
    }
    const double2 rho = mk(v[0], v[1]);
    const double2 beta = cmul(cdiv(rho, st->rho), cdiv(st->alpha, st->omega));
    const V bt = from_d2<V>(beta);
    const V om = from_d2<V>(st->omega);
    auto pnew = [&](int i) { return vadd(R[i], vmul(bt, vsub(Po[i], vmul(om, Vo[i])))); };
    for (int n = n0 + threadIdx.x; n < n1; n += kBlock) {
      const V p = pnew(n);
      const V v = shifted_apply(a, n, p, sft, pnew);
      Pn[n] = p;
      Vn[n] = v;
      const V rh = Rh[n];
      hv_re += (double)rh.x * v.x + (double)rh.y * v.y;
      hv_im += (double)rh.x * v.y - (double)rh.y * v.x;
    }
    double w[2] = {hv_re, hv_im};
    const int qw[2] = {QP_A_RE, QP_A_IM};
    write_parts<2>(a, qw, s, blockIdx.x, w, sh);
  }
}

// Phase 2: alpha = rho_k / <r_hat, v>; s = r - alpha v; t = (I - cA) s;
// partials <t, s>, <t, t>.  Workgroup 0 records rho_k and alpha_k.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bicg2(KrylovArgs a, int k) {
  using V = typename cvec<T>::type;
  __shared__ double sh[4 * 8];
  const int s = a.sys_list[blockIdx.y];
  SysState* st = a.st + s;
  // One read of the flag per workgroup: kernel A may clear it concurrently
  // (workgroup 0, on convergence), and every thread must take the same path.
  __shared__ int act;
  if (threadIdx.x == 0) act = st->active;
  __syncthreads();
  if (!act) return;
  const int cur = k & 1;
  double v[4];
  {
    const int qs[4] = {QP_RHO0_RE + 2 * cur, QP_RHO0_IM + 2 * cur, QP_A_RE, QP_A_IM};
    const int nw[4] = {a.wps_rho, a.wps_rho, a.wps, a.wps};  // rho: the previous iteration (k = 0: this one)
    reduce_parts<4>(a, qs, nw, s, v, sh);
  }
  const double2 rho = mk(v[0], v[1]);
  const double2 hv = mk(v[2], v[3]);
  double2 al = mk(0, 0);
  if (hv.x * hv.x + hv.y * hv.y > 0.0) al = cdiv(rho, hv);
  else if (blockIdx.x == 0 && threadIdx.x == 0 && (rho.x != 0.0 || rho.y != 0.0)) st->breakdown = 1;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->rho = rho;
    st->alpha = al;
  }
  const size_t off = (size_t)s * a.g.N;
  const V* R = reinterpret_cast<const V*>(a.R) + off;
  const V* Vc = reinterpret_cast<const V*>(a.V[k & 1]) + off;
  V* Sv = reinterpret_cast<V*>(a.S) + off;
  V* Tv = reinterpret_cast<V*>(a.T) + off;
  const V sft = from_d2<V>(a.shift[s]);
  const V av = from_d2<V>(al);
  const int n0 = blockIdx.x * a.chunk;
  const int n1 = min(a.g.N, n0 + a.chunk);
  auto sval = [&](int i) { return vsub(R[i], vmul(av, Vc[i])); };
  double ts_re = 0, ts_im = 0, tt = 0;
  for (int n = n0 + threadIdx.x; n < n1; n += kBlock) {
    const V sv = sval(n);
    const V t = shifted_apply(a, n, sv, sft, sval);
    Sv[n] = sv;
    Tv[n] = t;
    ts_re += (double)t.x * sv.x + (double)t.y * sv.y;
    ts_im += (double)t.x * sv.y - (double)t.y * sv.x;
    tt += (double)t.x * t.x + (double)t.y * t.y;
  }
  double w[3] = {ts_re, ts_im, tt};
  const int qs[3] = {QP_B_RE, QP_B_IM, QP_TT};
  write_parts<3>(a, qs, s, blockIdx.x, w, sh);
}

// Phase 3: omega = <t, s> / <t, t>; x += alpha p + omega s; r = s - omega t;
// partials rho_{k+1} = <r_hat, r>, ||r||^2.  Workgroup 0 records omega_k.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bicg3(KrylovArgs a, int k) {
  using V = typename cvec<T>::type;
  __shared__ double sh[4 * 8];
  const int s = a.sys_list[blockIdx.y];
  SysState* st = a.st + s;
  // One read of the flag per workgroup: kernel A may clear it concurrently
  // (workgroup 0, on convergence), and every thread must take the same path.
  __shared__ int act;
  if (threadIdx.x == 0) act = st->active;
  __syncthreads();
  if (!act) return;
  const int nxt = (k & 1) ^ 1;
  double v[3];
  {
    const int qs[3] = {QP_B_RE, QP_B_IM, QP_TT};
    const int nw[3] = {a.wps, a.wps, a.wps};
    reduce_parts<3>(a, qs, nw, s, v, sh);
  }
  double2 om = mk(0, 0);
  if (v[2] > 0.0) om = mk(v[0] / v[2], v[1] / v[2]);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->omega = om;
    if (v[2] > 0.0 && om.x == 0.0 && om.y == 0.0) st->breakdown = 1;
  }
  const size_t off = (size_t)s * a.g.N;
  V* X = reinterpret_cast<V*>(a.X) + off;
  V* R = reinterpret_cast<V*>(a.R) + off;
  const V* Rh = reinterpret_cast<const V*>(a.Rh) + off;
  const V* Pc = reinterpret_cast<const V*>(a.P[k & 1]) + off;
  const V* Sv = reinterpret_cast<const V*>(a.S) + off;
  const V* Tv = reinterpret_cast<const V*>(a.T) + off;
  const V av = from_d2<V>(st->alpha);
  const V ov = from_d2<V>(om);
  const int n0 = blockIdx.x * a.chunk;
  const int n1 = min(a.g.N, n0 + a.chunk);
  double hr_re = 0, hr_im = 0, rr = 0;
  for (int n = n0 + threadIdx.x; n < n1; n += kBlock) {
    const V sv = Sv[n];
    const V inc = vadd(vmul(av, Pc[n]), vmul(ov, sv));
    const V x = (k == 0) ? inc : vadd(X[n], inc);
    const V r = vsub(sv, vmul(ov, Tv[n]));
    X[n] = x;
    R[n] = r;
    const V rh = Rh[n];
    hr_re += (double)rh.x * r.x + (double)rh.y * r.y;
    hr_im += (double)rh.x * r.y - (double)rh.y * r.x;
    rr += (double)r.x * r.x + (double)r.y * r.y;
  }
  double w[3] = {hr_re, hr_im, rr};
  const int qs[3] = {QP_RHO0_RE + 2 * nxt, QP_RHO0_IM + 2 * nxt, QP_RR0 + nxt};
  write_parts<3>(a, qs, s, blockIdx.x, w, sh);
}

// BiCGStab for a whole system in one workgroup, for systems of at most
// kWgCap points: the iteration of k_bicg1..3 (same scalars, same
// stopping test at the start of each iteration k >= 1, same breakdown flags),
// with thread t of BLK owning the points t + BLK j (j < kWgCap / BLK), the
// vectors r, p, v, t, x of
// its points in registers, the vector that the stencil reads in LDS, and
// block-wide sums in place of the chunk partial sums.  One launch runs every
// iteration of every system, one workgroup each; nothing is shared between
// workgroups, and each loop ends at the iteration cap at the latest.
// complex128 takes 512 threads (eight points each), accumulates x in memory
// (read and written once per iteration by its owner thread) and keeps v in a
// second LDS array (each thread touches only its own points there); with
// half the waves of a 1024 x 4 shape the block sums cost half the
// instructions per point (the kernel is bound by instruction issue).
// complex64 takes 512 threads too (x and v in registers, no spills).
constexpr int kWgCap = 4096;
#ifndef AAO_BICG_WG_F64_BLK
#define AAO_BICG_WG_F64_BLK 512
#endif
#ifndef AAO_BICG_WG_F64_XMEM
#define AAO_BICG_WG_F64_XMEM 1
#endif
template <typename T> struct WgShape { static constexpr int BLK = AAO_BICG_WG_F64_BLK; };
template <> struct WgShape<float> { static constexpr int BLK = 512; };

// Sum of K values over the BLK threads in a fixed order; every thread gets
// the same bits.  The wave sums go through sh ((BLK / 64) * K doubles), and
// each wave then adds them up with one lane per wave (one LDS read per value
// and lane, so the reduction holds K values per lane, not BLK / 64 * K).
// Consecutive sums must use different sh buffers: the one barrier between
// the writes and the reads of a sum keeps every wave from writing sum i + 1
// before all have read sum i - 1, not sum i.
template <int BLK, int K>
__device__ __forceinline__ void wg_sum(double (&v)[K], double* sh) {
  constexpr int NW = BLK / 64;
#pragma unroll
  for (int i = 0; i < K; ++i) v[i] = wave_sum(v[i]);
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < K; ++i) sh[wid * K + i] = v[i];
  }
  __syncthreads();
  if constexpr (NW <= 8) {  // few wave sums: every lane adds them in order (broadcast reads)
#pragma unroll
    for (int i = 0; i < K; ++i) {
      double acc = sh[i];
#pragma unroll
      for (int w = 1; w < NW; ++w) acc += sh[w * K + i];
      v[i] = acc;
    }
  } else {
#pragma unroll
    for (int i = 0; i < K; ++i) v[i] = wave_sum(lane < NW ? sh[lane * K + i] : 0.0);
  }
}

// FAST: a 1D system of exactly kWgCap points (every owned point exists and a
// neighbour index is one add and one mask).
template <typename T, bool FAST>
__global__ __launch_bounds__(WgShape<T>::BLK) void k_bicg_wg(KrylovArgs a) {
  using V = typename cvec<T>::type;
  constexpr int kWgBlock = WgShape<T>::BLK;
  constexpr int kWgPts = kWgCap / kWgBlock;
  extern __shared__ double wg_lds[];
  __shared__ double sh2[2][(kWgBlock / 64) * 4];  // two buffers, used in turn by the block sums
  int sb = 0;
  auto sh = [&]() {
    sb ^= 1;
    return sh2[sb];
  };
  const int N = a.g.N;
  const int s = blockIdx.x;
  const size_t off = (size_t)s * N;
  const V* B = reinterpret_cast<const V*>(a.R) + off;  // b = r_0 = r_hat
  V* Rout = reinterpret_cast<V*>(a.R) + off;
  V* X = reinterpret_cast<V*>(a.X) + off;
  const LdsCplx<V> W(wg_lds, N);
  const V sft = from_d2<V>(a.shift[s]);
  const int t0 = threadIdx.x;
  // (x, y) of each owned point, packed (N <= 4096, so both fit 16 bits)
  int xy[kWgPts];
#pragma unroll
  for (int j = 0; j < kWgPts; ++j) {
    const int n = t0 + j * kWgBlock;
    xy[j] = (n % a.g.nx) | ((n / a.g.nx) << 16);
  }
  // out = (I - c A) in at the owned points, the neighbours read from LDS.
  // Between two applies there is always a block sum, whose barrier follows
  // every wave's reads of the previous copy, so the copy is written at once.
  auto apply = [&](const V (&in)[kWgPts], V (&out)[kWgPts]) {
#pragma unroll
    for (int j = 0; j < kWgPts; ++j) {
      const int n = t0 + j * kWgBlock;
      if (FAST || n < N) W.st(n, in[j]);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kWgPts; ++j) out[j] = vzero<V>();
#pragma unroll 1
    for (int q = 0; q < a.taps.n; ++q) {
      const int dx = a.taps.dx[q], dy = a.taps.dy[q];
      const T c = (T)a.taps.c[q];
#pragma unroll
      for (int j = 0; j < kWgPts; ++j) {
        const int n = t0 + j * kWgBlock;
        const int nb = FAST ? ((n + dx) & (kWgCap - 1)) : wrap_index(xy[j] & 0xffff, xy[j] >> 16, dx, dy, a.g);
        if (FAST || n < N) out[j] = vadd(out[j], vscale(W.ld(nb), c));
      }
    }
#pragma unroll
    for (int j = 0; j < kWgPts; ++j) out[j] = vsub(in[j], vmul(sft, out[j]));
  };
  auto dot = [](V u, V w, double& re, double& im) {  // conj(u) w
    re += (double)u.x * w.x + (double)u.y * w.y;
    im += (double)u.x * w.y - (double)u.y * w.x;
  };
  auto rhat = [&](int j) {
    const int n = t0 + j * kWgBlock;
    return (FAST || n < N) ? B[n] : vzero<V>();
  };
  constexpr bool kXMem = sizeof(T) == sizeof(double) && AAO_BICG_WG_F64_XMEM;
  V r[kWgPts], p[kWgPts], v[kXMem ? 1 : kWgPts], x[kXMem ? 1 : kWgPts];
  const LdsCplx<V> Vl(reinterpret_cast<char*>(wg_lds) + LdsCplx<V>::bytes(N), N);  // v (complex128)
  auto vget = [&](int j) -> V {
    if constexpr (kXMem) {
      const int n = t0 + j * kWgBlock;
      return (FAST || n < N) ? Vl.ld(n) : vzero<V>();
    } else {
      return v[j];
    }
  };
  auto vput = [&](const V (&o)[kWgPts]) {
#pragma unroll
    for (int j = 0; j < kWgPts; ++j) {
      if constexpr (kXMem) {
        const int n = t0 + j * kWgBlock;
        if (FAST || n < N) Vl.st(n, o[j]);
      } else {
        v[j] = o[j];
      }
    }
  };
#pragma unroll
  for (int j = 0; j < kWgPts; ++j) {
    r[j] = rhat(j);
    p[j] = r[j];
    if (!kXMem) x[j] = vzero<V>();
  }
  // k = 0: r_hat = r_0 = b, p_0 = b, rho_0 = ||b||^2
  {
    V vt[kWgPts];
    apply(p, vt);
    vput(vt);
  }
  double w4[4] = {0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < kWgPts; ++j) {
    dot(r[j], vget(j), w4[0], w4[1]);
    w4[2] += (double)r[j].x * r[j].x + (double)r[j].y * r[j].y;
  }
  wg_sum<kWgBlock, 4>(w4, sh());
  const double bb = w4[2];
  double2 rho = mk(bb, 0.0), hv = mk(w4[0], w4[1]);
  double2 al = mk(1, 0), om = mk(1, 0);
  double rr = bb;
  const double bbstop = a.bbfloor ? fmax(bb, a.bbfloor[s]) : bb;
  bool brk = false;
  int k = 0, flag = 1;
  for (;; ++k) {
    if (k > 0) {
      const bool conv = rr <= a.tol2 * bbstop;
      if (conv || k >= a.maxit || brk) {
        flag = conv ? 0 : (brk ? 2 : 1);
        break;
      }
      // rho_k = <r_hat, r_k> is in w4[0..1] from the end of the last iteration
      const double2 rho_k = mk(w4[0], w4[1]);
      const double2 beta = cmul(cdiv(rho_k, rho), cdiv(al, om));
      rho = rho_k;
      const V bt = from_d2<V>(beta), ov = from_d2<V>(om);
#pragma unroll
      for (int j = 0; j < kWgPts; ++j) p[j] = vadd(r[j], vmul(bt, vsub(p[j], vmul(ov, vget(j)))));
      {
        V vt[kWgPts];
        apply(p, vt);
        vput(vt);
      }
      double w2[2] = {0, 0};
#pragma unroll
      for (int j = 0; j < kWgPts; ++j) dot(rhat(j), vget(j), w2[0], w2[1]);
      wg_sum<kWgBlock, 2>(w2, sh());
      hv = mk(w2[0], w2[1]);
    }
    // alpha = rho_k / <r_hat, v>; s = r - alpha v (kept in r); t = (I - cA) s
    al = mk(0, 0);
    if (hv.x * hv.x + hv.y * hv.y > 0.0) al = cdiv(rho, hv);
    else if (rho.x != 0.0 || rho.y != 0.0) brk = true;
    const V av = from_d2<V>(al);
#pragma unroll
    for (int j = 0; j < kWgPts; ++j) r[j] = vsub(r[j], vmul(av, vget(j)));
    V tv[kWgPts];
    apply(r, tv);
    double w3[3] = {0, 0, 0};
#pragma unroll
    for (int j = 0; j < kWgPts; ++j) {
      dot(tv[j], r[j], w3[0], w3[1]);
      w3[2] += (double)tv[j].x * tv[j].x + (double)tv[j].y * tv[j].y;
    }
    wg_sum<kWgBlock, 3>(w3, sh());
    // omega = <t, s> / <t, t>; x += alpha p + omega s; r = s - omega t
    om = mk(0, 0);
    if (w3[2] > 0.0) om = mk(w3[0] / w3[2], w3[1] / w3[2]);
    if (w3[2] > 0.0 && om.x == 0.0 && om.y == 0.0) brk = true;
    const V ov = from_d2<V>(om);
    w4[0] = w4[1] = w4[2] = w4[3] = 0.0;
#pragma unroll
    for (int j = 0; j < kWgPts; ++j) {
      const V inc = vadd(vmul(av, p[j]), vmul(ov, r[j]));
      if (kXMem) {
        const int n = t0 + j * kWgBlock;
        if (FAST || n < N) X[n] = (k == 0) ? inc : vadd(X[n], inc);
      } else {
        x[j] = (k == 0) ? inc : vadd(x[j], inc);
      }
      r[j] = vsub(r[j], vmul(ov, tv[j]));
      dot(rhat(j), r[j], w4[0], w4[1]);
      w4[2] += (double)r[j].x * r[j].x + (double)r[j].y * r[j].y;
    }
    wg_sum<kWgBlock, 4>(w4, sh());
    rr = w4[2];
  }
#pragma unroll
  for (int j = 0; j < kWgPts; ++j) {
    const int n = t0 + j * kWgBlock;
    if (FAST || n < N) {
      if (!kXMem) X[n] = x[j];
      Rout[n] = r[j];
    }
  }
  if (t0 == 0) {
    SysState* st = a.st + s;
    st->active = 0;
    st->iters = k;
    st->flag = flag;
    st->breakdown = brk ? 1 : 0;
    st->rho = rho;
    st->alpha = al;
    st->omega = om;
    st->rr = rr;
    st->bb = bb;
  }
}

__global__ void k_krylov_init(SysState* st, int n, int* list) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    st[i] = fresh_state();
    if (list) list[i] = i;
  }
}

// List the still-active systems among the first n, in index order (one
// workgroup): in rounds of 256 systems each thread reads one flag, a ballot
// per wavefront and the four wavefront counts give each listed system its
// position.  Each flag is read once, so the list always matches its count.
// If count_tag != nullptr (pinned host memory) the count is stored to
// count_tag[0], then, after a system-scope fence, tag to count_tag[1]: a
// reader that sees the tag sees the count.
__global__ __launch_bounds__(kBlock) void k_compact_active(const SysState* st, int n, int* list, int* count_tag,
                                                           int tag) {
  __shared__ int wcnt[kBlock / 64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int total = 0;
  for (int base = 0; base < n; base += kBlock) {
    const int i = base + t;
    const bool act = i < n && st[i].active != 0;
    const unsigned long long bal = __ballot(act);
    if (lane == 0) wcnt[w] = __popcll(bal);
    __syncthreads();
    int o = total;
    for (int j = 0; j < w; ++j) o += wcnt[j];
    if (act) list[o + __popcll(bal & ((1ull << lane) - 1))] = i;
    total += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    __syncthreads();
  }
  if (t == 0 && count_tag) {
    count_tag[0] = total;
    __threadfence_system();
    count_tag[1] = tag;
  }
}

template <typename V>
__global__ void k_copy_in(V* dst, const double2* src, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = from_d2<V>(src[i]);
}

template <typename V>
__global__ void k_copy_out(double2* dst, const V* src, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = to_d2(src[i]);
}

// grad_u0[b][n] = sum_m lambda[b][0][m][n];
// part[b][blk] = dt sum_{l,m} lambda_{l,m} (sum_k q_mk (dA u_{l,k}))  over a share of n.
template <int M>
__global__ __launch_bounds__(kBlock) void k_grad(const double* u, const double* lam, double* gu0,
                                                 double* part, Taps dt_, const double* __restrict__ q_,
                                                 double dt, Geo g, int L) {
  __shared__ double sh[4];
  __shared__ double q[kMaxM * kMaxM];
  for (int i = threadIdx.x; i < M * M; i += kBlock) q[i] = q_[i];
  __syncthreads();
  const int b = blockIdx.y;
  const int N = g.N;
  double acc = 0.0;
  for (int n = blockIdx.x * kBlock + threadIdx.x; n < N; n += gridDim.x * kBlock) {
    const int x = n % g.nx, y = n / g.nx;
    double s0 = 0.0;
    for (int m = 0; m < M; ++m) s0 += lam[(((size_t)b * L) * M + m) * N + n];
    gu0[(size_t)b * N + n] = s0;
    for (int l = 0; l < L; ++l) {
      const double* ul = u + ((size_t)b * L + l) * M * (size_t)N;
      const double* ll = lam + ((size_t)b * L + l) * M * (size_t)N;
      double v[M];
#pragma unroll
      for (int m = 0; m < M; ++m) v[m] = 0.0;
      for (int t = 0; t < dt_.n; ++t) {
        const int nb = wrap_index(x, y, dt_.dx[t], dt_.dy[t], g);
#pragma unroll
        for (int m = 0; m < M; ++m) v[m] = fma(dt_.c[t], ul[(size_t)m * N + nb], v[m]);
      }
#pragma unroll
      for (int m = 0; m < M; ++m) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < M; ++k) s = fma(q[m * M + k], v[k], s);
        acc = fma(ll[(size_t)m * N + n], s, acc);
      }
    }
  }
  double v[1] = {acc * dt};
  block_sum<1>(v, sh);
  if (threadIdx.x == 0) part[(size_t)b * gridDim.x + blockIdx.x] = v[0];
}

__global__ __launch_bounds__(kBlock) void k_grad_finalize(const double* part, int nblk, double* gnu) {
  __shared__ double sh[4];
  const int b = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk; i += kBlock) s += part[(size_t)b * nblk + i];
  double v[1] = {s};
  block_sum<1>(v, sh);
  if (threadIdx.x == 0) gnu[b] = v[0];
}

int grid_for(int64_t n, int per = kBlock, int cap = 8192) {
  int64_t g = (n + per - 1) / per;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

// two planes of L * M * TN/2 doubles (plus the pad) and the L/2 twiddles
size_t xform_lds_bytes(int M, int L, int TN) {
  return (2 * ((size_t)L * M * (TN / 2) + kPlanePad) + (size_t)L) * sizeof(double);
}

// LDS offset (doubles, even) of the node transforms staged after `used`
// bytes, or -1 where they do not fit kMixLdsBytes or would lower the number of
// workgroups a CU holds (at most five: the transform's register budget);
// *bytes receives the launch's LDS size.
int mix_offset(int M, int Lh, size_t used, size_t* bytes) {
  constexpr size_t kLdsPerCU = 160 * 1024;
  const size_t mb = (size_t)Lh * M * M * sizeof(double2);
  const size_t off = (used + 15) / 16 * 16;
  *bytes = used;
  if (mb > kMixLdsBytes || kLdsPerCU / (off + mb) < std::min<size_t>(kLdsPerCU / used, 5)) return -1;
  *bytes = off + mb;
  return (int)(off / sizeof(double));
}

// Halo width of the staged residual (the largest |dx| of the taps with dy = 0;
// none when a tile is a whole row), or -1 where it is not used: a tile must
// lie inside one grid row, a thread hold at most kStageRows rows l, and the
// halo take at most a quarter of the tile's LDS.  Staging also waits for a
// grid of at least kStageMinGrid workgroups (64 per CU): measured on 1024^2
// (L = 32) and 512^2 x 8 (L = 64) grids it saves 9-11 % of the kernel, on
// 256^2 (L = 64, 4096 workgroups) it costs 8 %.
constexpr int64_t kStageMinGrid = 16384;

int stage_halo(const FwdArgs& a, int B) {
  if ((int64_t)((a.g.N + a.TN - 1) / a.TN) * B < kStageMinGrid) return -1;
  if (a.g.nx % a.TN != 0 || (int64_t)a.L * a.TN > (int64_t)kStageRows * kBlock) return -1;
  if (a.TN == a.g.nx) return 0;
  int hx = 0;
  for (int t = 0; t < a.taps.n; ++t)
    if (a.taps.dy[t] == 0) hx = std::max(hx, std::abs(a.taps.dx[t]));
  return 8 * hx <= a.TN ? hx : -1;
}

template <int M>
hipError_t fwd_m(bool adj, bool from_r, bool out_f32, const FwdArgs& a0, int B, hipStream_t st) {
  dim3 grid((a0.g.N + a0.TN - 1) / a0.TN, B);
  FwdArgs a = a0;
  const int hx = (from_r || M > 4) ? -1 : stage_halo(a0, B);
  a.hx = hx > 0 ? hx : 0;
  size_t lds = xform_lds_bytes(M, a.L, a.TN) + (size_t)a.L * M * 2 * a.hx * sizeof(double);
  a.mixo = mix_offset(M, a.Lh, lds, &lds);
  const int nt = (a.taps.n == 3 || a.taps.n == 5) ? a.taps.n : 0;
#define AAO_FWD(ADJ, MODE, OV, NT, STG) \
  hipLaunchKernelGGL((k_fwd<M, ADJ, MODE, OV, NT, STG>), grid, dim3(kBlock), lds, st, a)
  // residual forms with 5, 3 or any number of taps: staged (M <= 4) or not
#define AAO_FWDT(ADJ, OV, STG)                      \
  do {                                              \
    if (nt == 5) AAO_FWD(ADJ, 0, OV, 5, STG);       \
    else if (nt == 3) AAO_FWD(ADJ, 0, OV, 3, STG);  \
    else AAO_FWD(ADJ, 0, OV, 0, STG);               \
  } while (0)
#define AAO_FWD0(ADJ, OV)                                    \
  do {                                                       \
    if constexpr (M <= 4) {                                  \
      if (hx < 0) AAO_FWDT(ADJ, OV, false);                  \
      else AAO_FWDT(ADJ, OV, true);                          \
    } else {                                                 \
      AAO_FWDT(ADJ, OV, false);                              \
    }                                                        \
  } while (0)
  if (!adj) {
    if (!from_r) { if (out_f32) AAO_FWD0(false, float2); else AAO_FWD0(false, double2); }
    else { if (out_f32) AAO_FWD(false, 1, float2, 0, false); else AAO_FWD(false, 1, double2, 0, false); }
  } else {
    if (!from_r) { if (out_f32) AAO_FWD0(true, float2); else AAO_FWD0(true, double2); }
    else { if (out_f32) AAO_FWD(true, 1, float2, 0, false); else AAO_FWD(true, 1, double2, 0, false); }
  }
#undef AAO_FWD0
#undef AAO_FWDT
#undef AAO_FWD
  return hipGetLastError();
}

template <int M>
hipError_t bwd_m(bool adj, bool to_delta, bool in_f32, const BwdArgs& a, int B, hipStream_t st) {
  dim3 grid((a.g.N + a.TN - 1) / a.TN, B);
  size_t lds = xform_lds_bytes(M, a.L, a.TN);
#define AAO_BWD(ADJ, MODE, IV) hipLaunchKernelGGL((k_bwd<M, ADJ, MODE, IV>), grid, dim3(kBlock), lds, st, a)
  if (!adj) {
    if (!to_delta) { if (in_f32) AAO_BWD(false, 0, float2); else AAO_BWD(false, 0, double2); }
    else { if (in_f32) AAO_BWD(false, 1, float2); else AAO_BWD(false, 1, double2); }
  } else {
    if (!to_delta) { if (in_f32) AAO_BWD(true, 0, float2); else AAO_BWD(true, 0, double2); }
    else { if (in_f32) AAO_BWD(true, 1, float2); else AAO_BWD(true, 1, double2); }
  }
#undef AAO_BWD
  return hipGetLastError();
}

template <int M>
hipError_t res_m(bool adj, const FwdArgs& a, double* r_out, int B, int nblk, hipStream_t st) {
  if (adj) hipLaunchKernelGGL((k_residual<M, true>), dim3(nblk), dim3(kBlock), 0, st, a, r_out, B);
  else hipLaunchKernelGGL((k_residual<M, false>), dim3(nblk), dim3(kBlock), 0, st, a, r_out, B);
  return hipGetLastError();
}

}  // namespace

#define AAO_DISPATCH_M(M_, CALL)                     \
  switch (M_) {                                      \
    case 1: return CALL(1);                          \
    case 2: return CALL(2);                          \
    case 3: return CALL(3);                          \
    case 4: return CALL(4);                          \
    case 5: return CALL(5);                          \
    case 6: return CALL(6);                          \
    case 7: return CALL(7);                          \
    case 8: return CALL(8);                          \
    default: return hipErrorInvalidValue;            \
  }

hipError_t launch_fwd(int M, bool adj, bool from_r, bool out_f32, const FwdArgs& a, int B,
                      hipStream_t st) {
#define C_(m) fwd_m<m>(adj, from_r, out_f32, a, B, st)
  AAO_DISPATCH_M(M, C_)
#undef C_
}

hipError_t launch_bwd(int M, bool adj, bool to_delta, bool in_f32, const BwdArgs& a, int B,
                      hipStream_t st) {
#define C_(m) bwd_m<m>(adj, to_delta, in_f32, a, B, st)
  AAO_DISPATCH_M(M, C_)
#undef C_
}

hipError_t launch_residual(int M, bool adj, const FwdArgs& a, double* r_out, int B, hipStream_t st) {
  const int nblk = grid_for((int64_t)B * a.L * a.g.N, kBlock, 1024);
#define C_(m) res_m<m>(adj, a, r_out, B, nblk, st)
  AAO_DISPATCH_M(M, C_)
#undef C_
}

int residual_blocks(int B, int L, int N) { return grid_for((int64_t)B * L * N, kBlock, 1024); }

hipError_t launch_finalize(const double* ps, int ns, const double* pm, int nm, double* out,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, st, ps, ns, pm, nm, out);
  return hipGetLastError();
}

hipError_t launch_sweep_report(const double* ps, int ns, const double* pm, int nm, double* out, const SysState* sst,
                               int nsys, bool cocg, double* rep, int tag, hipStream_t st) {
  hipLaunchKernelGGL(k_sweep_report, dim3(1), dim3(kBlock), 0, st, ps, ns, pm, nm, out, sst, nsys, cocg ? 1 : 0, rep,
                     tag);
  return hipGetLastError();
}

hipError_t launch_last_node(const double* u, double* out, int B, int L, int M, int N, hipStream_t st) {
  hipLaunchKernelGGL(k_last_node, dim3(grid_for((int64_t)B * N)), dim3(kBlock), 0, st, u, out, B, L, M, N);
  return hipGetLastError();
}

hipError_t launch_init_u(double* u, const double* u0, int B, int L, int M, int N, hipStream_t st) {
  hipLaunchKernelGGL(k_init_u, dim3(grid_for((int64_t)B * L * M * N)), dim3(kBlock), 0, st, u, u0,
                     B, L, M, N);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, double v, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kBlock), 0, st, p, v, n);
  return hipGetLastError();
}

hipError_t launch_norms_bn(const double* v, int B, int N, double* part, int nparts, hipStream_t st) {
  hipLaunchKernelGGL(k_norms, dim3(nparts), dim3(kBlock), 0, st, v, (int64_t)B * N, part);
  return hipGetLastError();
}

hipError_t launch_norms_per_b(const double* v, int B, int N, double* part, int nparts, hipStream_t st) {
  hipLaunchKernelGGL(k_norms, dim3(nparts, B), dim3(kBlock), 0, st, v, (int64_t)N, part);
  return hipGetLastError();
}

template <int M>
hipError_t wnorms_m(const FwdArgs& a, int B, double* part, int nparts, hipStream_t st) {
  hipLaunchKernelGGL((k_wnorms<M>), dim3(nparts), dim3(kBlock), 0, st, a, B, part);
  return hipGetLastError();
}

hipError_t launch_wnorms(int M, const FwdArgs& a, int B, double* part, int nparts, hipStream_t st) {
  switch (M) {
    case 1: return wnorms_m<1>(a, B, part, nparts, st);
    case 2: return wnorms_m<2>(a, B, part, nparts, st);
    case 3: return wnorms_m<3>(a, B, part, nparts, st);
    case 4: return wnorms_m<4>(a, B, part, nparts, st);
    case 5: return wnorms_m<5>(a, B, part, nparts, st);
    case 6: return wnorms_m<6>(a, B, part, nparts, st);
    case 7: return wnorms_m<7>(a, B, part, nparts, st);
    case 8: return wnorms_m<8>(a, B, part, nparts, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_bicg(int phase, bool f32, const KrylovArgs& a, int k, int nact, hipStream_t st) {
  if (a.wps < 1 || a.wps > a.wps_stride || a.wps_rho < 1 || a.wps_rho > a.wps_stride || a.wps_bb < 1 ||
      a.wps_bb > a.wps_stride || (int64_t)a.wps * a.chunk < a.g.N || (int64_t)(a.wps - 1) * a.chunk >= a.g.N)
    return hipErrorInvalidValue;
  dim3 grid(a.wps, nact);
  switch (phase) {
    case 1:
      if (f32) hipLaunchKernelGGL(k_bicg1<float>, grid, dim3(kBlock), 0, st, a, k);
      else hipLaunchKernelGGL(k_bicg1<double>, grid, dim3(kBlock), 0, st, a, k);
      break;
    case 2:
      if (f32) hipLaunchKernelGGL(k_bicg2<float>, grid, dim3(kBlock), 0, st, a, k);
      else hipLaunchKernelGGL(k_bicg2<double>, grid, dim3(kBlock), 0, st, a, k);
      break;
    default:
      if (f32) hipLaunchKernelGGL(k_bicg3<float>, grid, dim3(kBlock), 0, st, a, k);
      else hipLaunchKernelGGL(k_bicg3<double>, grid, dim3(kBlock), 0, st, a, k);
      break;
  }
  return hipGetLastError();
}

bool bicg_wg_fits(int N) { return N >= 1 && N <= kWgCap; }

hipError_t launch_bicg_wg(bool f32, const KrylovArgs& a, int nsys, hipStream_t st) {
  if (!bicg_wg_fits(a.g.N) || nsys < 1) return hipErrorInvalidValue;
  const bool fast = a.g.ny == 1 && a.g.N == kWgCap;
  const size_t l32 = LdsCplx<float2>::bytes(a.g.N), l64 = 2 * LdsCplx<double2>::bytes(a.g.N);  // f64: input, v
  if (f32) {
    if (fast) hipLaunchKernelGGL((k_bicg_wg<float, true>), dim3(nsys), dim3(WgShape<float>::BLK), l32, st, a);
    else hipLaunchKernelGGL((k_bicg_wg<float, false>), dim3(nsys), dim3(WgShape<float>::BLK), l32, st, a);
  } else {
    if (fast) hipLaunchKernelGGL((k_bicg_wg<double, true>), dim3(nsys), dim3(WgShape<double>::BLK), l64, st, a);
    else hipLaunchKernelGGL((k_bicg_wg<double, false>), dim3(nsys), dim3(WgShape<double>::BLK), l64, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_krylov_init(const KrylovArgs& a, hipStream_t st, int* list) {
  hipLaunchKernelGGL(k_krylov_init, dim3(grid_for(a.num_sys)), dim3(kBlock), 0, st, a.st, a.num_sys, list);
  return hipGetLastError();
}

hipError_t launch_compact_active(const SysState* st, int n, int* list, int* count_tag, int tag, hipStream_t s) {
  hipLaunchKernelGGL(k_compact_active, dim3(1), dim3(kBlock), 0, s, st, n, list, count_tag, tag);
  return hipGetLastError();
}

hipError_t launch_copy_c128_in(void* dst, bool f32, const double* src, int64_t n, hipStream_t st) {
  const double2* s2 = reinterpret_cast<const double2*>(src);
  if (f32) hipLaunchKernelGGL(k_copy_in<float2>, dim3(grid_for(n)), dim3(kBlock), 0, st, (float2*)dst, s2, n);
  else hipLaunchKernelGGL(k_copy_in<double2>, dim3(grid_for(n)), dim3(kBlock), 0, st, (double2*)dst, s2, n);
  return hipGetLastError();
}

hipError_t launch_copy_c128_out(double* dst, const void* src, bool f32, int64_t n, hipStream_t st) {
  double2* d2 = reinterpret_cast<double2*>(dst);
  if (f32) hipLaunchKernelGGL(k_copy_out<float2>, dim3(grid_for(n)), dim3(kBlock), 0, st, d2, (const float2*)src, n);
  else hipLaunchKernelGGL(k_copy_out<double2>, dim3(grid_for(n)), dim3(kBlock), 0, st, d2, (const double2*)src, n);
  return hipGetLastError();
}

template <int M>
static hipError_t grad_m(const double* u, const double* lam, double* gu0, double* part,
                         const Taps& dtaps, const double* q, double dt, const Geo& g, int B, int L,
                         int nblk, hipStream_t st) {
  hipLaunchKernelGGL((k_grad<M>), dim3(nblk, B), dim3(kBlock), 0, st, u, lam, gu0, part, dtaps, q,
                     dt, g, L);
  return hipGetLastError();
}

hipError_t launch_grad(int M, const double* u, const double* lam, double* gu0, double* part,
                       const Taps& dtaps, const double* q, double dt, const Geo& g, int B, int L,
                       int nblk, hipStream_t st) {
#define C_(m) grad_m<m>(u, lam, gu0, part, dtaps, q, dt, g, B, L, nblk, st)
  AAO_DISPATCH_M(M, C_)
#undef C_
}

hipError_t launch_grad_finalize(const double* part, int nblk, int B, double* gnu, hipStream_t st) {
  hipLaunchKernelGGL(k_grad_finalize, dim3(B), dim3(kBlock), 0, st, part, nblk, gnu);
  return hipGetLastError();
}

}  // namespace aao
