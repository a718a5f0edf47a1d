// Batched COCG for the complex-symmetric shifted systems (I - c_s A) x_s = b_s
// of the alpha-circulant sweep (row a3), one pass per iteration.
//
// The recurrences are those of CG with the bilinear form x^T y (COCG) in the
// one-reduction arrangement: with gamma_k = r_k^T r_k and delta_k = r_k^T A_s r_k,
//   p_k = r_k + beta_k p_{k-1},  s_k = A_s p_k,
//   x_{k+1} = x_k + alpha_k p_k,  r_{k+1} = r_k - alpha_k s_k,
//   beta_{k+1} = gamma_{k+1} / gamma_k,
//   alpha_{k+1} = gamma_{k+1} / (delta_{k+1} - beta_{k+1} gamma_{k+1} / alpha_k),
// which uses p^T A_s p = r^T A_s r - beta gamma / alpha_prev (A_s-conjugacy of
// p_k, p_{k-1} and orthogonality of r_{k+1}, r_k).  s_k is applied directly
// (not by recurrence): a workgroup owns a TX x TY tile, builds p_k on a two-hop
// halo in LDS, applies A_s on the one-hop halo to get r_{k+1} there, and A_s
// once more at the tile points for delta_{k+1}.  Global traffic per element
// and pass: read r_k, p_{k-1}, x_k and write r_{k+1}, p_k, x_{k+1}.
//
// Scalars live in SysState; a small per-system kernel reduces the tile
// partial sums in a fixed order (bitwise reproducible) between passes.
#include "aao_device.hpp"
#include "aao_kernels.hpp"

namespace aao {

namespace {

using namespace dev;

constexpr int kQ = 5;  // partial quantities: gamma (re, im), delta (re, im), ||r||^2

__device__ __forceinline__ int pmod(int v, int n) {
  if ((n & (n - 1)) == 0) return v & (n - 1);
  v %= n;
  return v < 0 ? v + n : v;
}

// i / d for 0 <= i < 2^16 and 1 <= d < 2^16 with m = ceil(2^40 / d): the error
// term i (m d - 2^40) / (d 2^40) < 2^-24 cannot cross an integer, so it is exact.
__device__ __forceinline__ int fdiv(int i, unsigned long long m) {
  return (int)(((unsigned long long)(unsigned)i * m) >> 40);
}

__device__ __forceinline__ double* cg_part(const CgArgs& a, int q, int s) {
  return a.part + ((size_t)q * a.num_sys + s) * a.ntiles;
}

template <int K>
__device__ __forceinline__ void write_tile_parts(const CgArgs& a, int s, double (&v)[K], double* sh) {
  block_sum<K>(v, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < K; ++q) cg_part(a, q, s)[blockIdx.x] = v[q];
  }
}

// gamma_0 = b^T b, delta_0 = b^T A_s b, ||b||^2 over one tile (neighbours from
// global memory: this pass runs once per solve).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_init(CgArgs a) {
  using V = typename cvec<T>::type;
  __shared__ double sh[4 * kQ];
  const int s = a.sys_list[blockIdx.y];
  const V* Rb = reinterpret_cast<const V*>(a.R[0]) + (size_t)s * a.g.N;
  const V sft = from_d2<V>(a.shift[s]);
  int tile = blockIdx.x;
  if (a.xcd_band > 0) tile = (tile & 7) * a.xcd_band + (tile >> 3);
  const int ty = fdiv(tile, a.m_ntx), tx = tile - ty * a.ntx;
  const int x0 = tx * a.TX, y0 = ty * a.TY;
  double v[kQ] = {0, 0, 0, 0, 0};
  for (int i = threadIdx.x; i < a.TX * a.TY; i += kBlock) {
    const int x = x0 + i % a.TX, y = y0 + i / a.TX;
    if (x >= a.g.nx || y >= a.g.ny) continue;
    const int n = y * a.g.nx + x;
    const V b = Rb[n];
    V acc = vzero<V>();
    for (int t = 0; t < a.taps.n; ++t) {
      const int nb = wrap_index(x, y, a.taps.dx[t], a.taps.dy[t], a.g);
      acc = vadd(acc, vscale(Rb[nb], (T)a.taps.c[t]));
    }
    const V w = vsub(b, vmul(sft, acc));
    v[0] += (double)b.x * b.x - (double)b.y * b.y;
    v[1] += 2.0 * (double)b.x * b.y;
    v[2] += (double)b.x * w.x - (double)b.y * w.y;
    v[3] += (double)b.x * w.y + (double)b.y * w.x;
    v[4] += (double)b.x * b.x + (double)b.y * b.y;
  }
  block_sum<kQ>(v, sh);
  if (threadIdx.x == 0) {
    double* pb = a.part + (a.fused ? (size_t)kQ * a.num_sys * a.ntiles : 0);
#pragma unroll
    for (int q = 0; q < kQ; ++q) pb[((size_t)q * a.num_sys + s) * a.ntiles + tile] = v[q];
  }
}

// Points per thread of the two halo regions; the host keeps
// (TX + 4Rx)(TY + 4Ry) <= kMaxPerThread * kBlock.
constexpr int kMaxPerThread = 8;

// Taps applied to an LDS tile with row pitch W: NT > 0 unrolls a fixed count.
template <int NT, typename T, typename V>
__device__ __forceinline__ V tile_stencil(const CgArgs& a, const V* buf, int c, int W) {
  V acc = vzero<V>();
  if (NT > 0) {
#pragma unroll
    for (int t = 0; t < NT; ++t) acc = vadd(acc, vscale(buf[c + a.taps.dx[t] + a.taps.dy[t] * W], (T)a.taps.c[t]));
  } else {
    for (int t = 0; t < a.taps.n; ++t)
      acc = vadd(acc, vscale(buf[c + a.taps.dx[t] + a.taps.dy[t] * W], (T)a.taps.c[t]));
  }
  return acc;
}

// Advance the COCG scalars of one system from the reduced partial sums of
// r_{k} (gamma_k, delta_k, ||r_k||^2).  Returns 0 to go on, 1 converged, 2
// iteration cap, 3 breakdown.  k == 0: the sums are those of b = r_0.
__device__ __forceinline__ int cg_advance(int k, double2 gam, double2 del, double rr, double bb, double tol2,
                                          int maxit, double2 gam_prev, double2 al_prev, double2& al, double2& be) {
  if (k == 0) {
    const double d2 = del.x * del.x + del.y * del.y;
    al = (rr > 0.0 && d2 > 0.0) ? cdiv(gam, del) : mk(0, 0);  // b = 0: x stays 0
    be = mk(0, 0);
    return 0;
  }
  if (rr <= tol2 * bb) return 1;
  if (k >= maxit) return 2;
  const bool ok0 = (gam_prev.x != 0.0 || gam_prev.y != 0.0) && (al_prev.x != 0.0 || al_prev.y != 0.0);
  be = ok0 ? cdiv(gam, gam_prev) : mk(0, 0);
  const double2 den = ok0 ? csub(del, cdiv(cmul(be, gam), al_prev)) : mk(0, 0);
  if (!ok0 || (den.x == 0.0 && den.y == 0.0) || !isfinite(den.x) || !isfinite(den.y)) return 3;
  al = cdiv(gam, den);
  return 0;
}

// Scalars of pass k for system s (identical in every workgroup of the
// system).  Fused mode: reduce pass k-1's tile sums, advance alpha/beta and
// the convergence decision (tile 0 records it); else read what the scalar
// kernel wrote.  Returns false if the system is done.
template <int BS>
__device__ __forceinline__ bool cg_prologue(const CgArgs& a, int k, int s, int tile, double* sh, int* act,
                                            double2* sc) {
  if (a.fused) {
    // every workgroup of the system reduces the previous pass's tile sums in
    // the same order and takes the same decision; tile 0 records it
    double v[kQ] = {0, 0, 0, 0, 0};
    const double* pp0 = a.part + (size_t)((k + 1) & 1) * kQ * a.num_sys * a.ntiles;
    for (int c = threadIdx.x; c < a.ntiles; c += BS) {
#pragma unroll
      for (int q = 0; q < kQ; ++q) v[q] += pp0[((size_t)q * a.num_sys + s) * a.ntiles + c];
    }
    block_sum_w<kQ, BS / 64>(v, sh);
    if (threadIdx.x == 0) {
      SysState* st = a.st + s;
      const double bb = (k == 0) ? v[4] : st->bb;
      double2 al = mk(0, 0), be = mk(0, 0);
      const int dec = cg_advance(k, mk(v[0], v[1]), mk(v[2], v[3]), v[4], bb, a.tol2, a.maxit,
                                 st->gamma2[(k + 1) & 1], st->alpha2[(k + 1) & 1], al, be);
      sc[0] = al;
      sc[1] = be;
      *act = dec == 0;
      if (tile == 0) {
        if (k == 0) st->bb = bb;
        st->rr = v[4];
        if (dec == 0) {
          st->gamma2[k & 1] = mk(v[0], v[1]);
          st->alpha2[k & 1] = al;
        } else {
          st->active = 0;
          st->iters = k;
          st->flag = dec - 1;
        }
      }
    }
    __syncthreads();
    if (!*act) return false;
  } else {
    if (threadIdx.x == 0) {
      sc[0] = a.st[s].alpha;
      sc[1] = a.st[s].beta;
    }
    __syncthreads();
  }
  return true;
}

#ifndef AAO_CG_MIN_WAVES
#define AAO_CG_MIN_WAVES 1
#endif

template <typename T, int NP, int NT, int BS>
__global__ __launch_bounds__(BS, AAO_CG_MIN_WAVES) void k_cg_pass(CgArgs a, int k) {
  using V = typename cvec<T>::type;
  extern __shared__ char smem[];
  __shared__ double sh[(BS / 64) * kQ];
  __shared__ int act;
  __shared__ double2 sc[2];
  const int s = a.sys_list[blockIdx.y];
  // XCD-aware tile order: workgroups are dealt round-robin to the 8 XCDs
  // (each with its own L2), so slot b goes to XCD b % 8; give each XCD a
  // contiguous band of tiles so that tile halos are read from its own L2.
  int tile = blockIdx.x;
  if (a.xcd_band > 0) tile = (tile & 7) * a.xcd_band + (tile >> 3);
  const int Rx = a.Rx, Ry = a.Ry, TX = a.TX, TY = a.TY;
  const int PW = TX + 4 * Rx, PH = TY + 4 * Ry;
  const int QW = TX + 2 * Rx, QH = TY + 2 * Ry;
  V* Pt = reinterpret_cast<V*>(smem);  // p_k on the two-hop halo, then r_{k+1} on the one-hop halo
  const size_t off = (size_t)s * a.g.N;
  const V* Rin = reinterpret_cast<const V*>(a.R[k & 1]) + off;
  V* Rout = reinterpret_cast<V*>(a.R[(k + 1) & 1]) + off;
  const V* Pold = reinterpret_cast<const V*>(a.P[(k + 1) & 1]) + off;
  V* Pnew = reinterpret_cast<V*>(a.P[k & 1]) + off;
  V* X = reinterpret_cast<V*>(a.X) + off;
  const int nx = a.g.nx, ny = a.g.ny;
  const int ty = fdiv(tile, a.m_ntx);
  const int tx = tile - ty * a.ntx;
  const int x0 = tx * TX, y0 = ty * TY;

  // converged systems leave before touching memory (the host drops them from
  // the launch list at its next, lagged, check)
  if (threadIdx.x == 0) act = a.st[s].active;
  __syncthreads();
  if (!act) return;
  // Each thread owns the same points of the two-hop region in every stage:
  // it loads r_k and p_{k-1} there (and x_k at its tile points), and later
  // computes r_{k+1} at those of its points that lie in the one-hop region,
  // so r_k is read from memory once.  All loads are issued up front; the
  // state read below does not gate them.
  V rp[NP], pp[NP];
  int gq[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    const int i = threadIdx.x + j * BS;
    gq[j] = -1;
    if (i < PW * PH) {
      const int py = fdiv(i, a.m_pw), px = i - py * PW;
      const int ux = x0 - 2 * Rx + px, uy = y0 - 2 * Ry + py;
      const int g = pmod(uy, ny) * nx + pmod(ux, nx);
      rp[j] = Rin[g];
      if (k > 0) pp[j] = Pold[g];
      const bool inside = px >= 2 * Rx && px < 2 * Rx + TX && py >= 2 * Ry && py < 2 * Ry + TY && ux < nx && uy < ny;
      if (inside) gq[j] = g;
    }
  }
  if (!cg_prologue<BS>(a, k, s, tile, sh, &act, sc)) return;
  const V al = from_d2<V>(sc[0]);
  const V be = from_d2<V>(sc[1]);
  const V sft = from_d2<V>(a.shift[s]);
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    const int i = threadIdx.x + j * BS;
    if (i < PW * PH) Pt[i] = (k > 0) ? vadd(rp[j], vmul(be, pp[j])) : rp[j];
  }
  // x_k at this thread's tile points, issued before the barrier
  V xq[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j)
    if (k > 0 && gq[j] >= 0) xq[j] = X[gq[j]];
  __syncthreads();
  // r_{k+1} = r_k - alpha_k A_s p_k on the one-hop halo (kept in registers
  // until every thread has read p_k); tile points store r_{k+1}, p_k, x_{k+1}
  int qi[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    const int i = threadIdx.x + j * BS;
    qi[j] = -1;
    if (i < PW * PH) {
      const int py = fdiv(i, a.m_pw), px = i - py * PW;
      if (px >= Rx && px < PW - Rx && py >= Ry && py < PH - Ry) {
        qi[j] = (px - Rx) + (py - Ry) * QW;
        const V acc = tile_stencil<NT, T>(a, Pt, i, PW);
        const V p = Pt[i];
        rp[j] = vsub(rp[j], vmul(al, vsub(p, vmul(sft, acc))));  // now r_{k+1}
        if (gq[j] >= 0) {
          const int g = gq[j];
          Rout[g] = rp[j];
          Pnew[g] = p;
          X[g] = (k == 0) ? vmul(al, p) : vadd(xq[j], vmul(al, p));
        }
      }
    }
    // one point at a time: keeps the stencil operands of different points
    // from being live together (register pressure -> occupancy)
    __builtin_amdgcn_sched_barrier(0);
  }
  __syncthreads();
  V* Rt = Pt;
#pragma unroll
  for (int j = 0; j < NP; ++j)
    if (qi[j] >= 0) Rt[qi[j]] = rp[j];
  __syncthreads();
  // gamma_{k+1}, delta_{k+1} = r^T A_s r, ||r_{k+1}||^2 at the tile points
  double v[kQ] = {0, 0, 0, 0, 0};
  for (int i = threadIdx.x; i < TX * TY; i += BS) {
    const int iy = fdiv(i, a.m_tx), ix = i - iy * TX;
    if (x0 + ix >= nx || y0 + iy >= ny) continue;
    const int cr = (ix + Rx) + (iy + Ry) * QW;
    const V acc = tile_stencil<NT, T>(a, Rt, cr, QW);
    const V r = Rt[cr];
    const V w = vsub(r, vmul(sft, acc));
    v[0] += (double)r.x * r.x - (double)r.y * r.y;
    v[1] += 2.0 * (double)r.x * r.y;
    v[2] += (double)r.x * w.x - (double)r.y * w.y;
    v[3] += (double)r.x * w.y + (double)r.y * w.x;
    v[4] += (double)r.x * r.x + (double)r.y * r.y;
    __builtin_amdgcn_sched_barrier(0);
  }
  block_sum_w<kQ, BS / 64>(v, sh);
  if (threadIdx.x == 0) {
    double* pb = a.part + (a.fused ? (size_t)(k & 1) * kQ * a.num_sys * a.ntiles : 0);
#pragma unroll
    for (int q = 0; q < kQ; ++q) pb[((size_t)q * a.num_sys + s) * a.ntiles + tile] = v[q];
  }
}

// Row-marching pass (2D, stencil reach RY <= 2 in y): a workgroup owns a strip
// of SX = TX columns and SY = TY rows and walks down it one row per step.
// Step i brings in row y0 - 2RY + i of r_k and p_{k-1} (prefetched two steps
// ahead) and forms p_k there in an LDS ring of 2RY+1 rows; one row behind it
// applies A_s to p_k and forms r_{k+1} in a second ring; another row behind,
// A_s r_{k+1} gives the dot products.  r_k of the last RY+1 rows stays in
// registers.  The y halo is paid only at the strip ends.
template <typename T, int RY, int NT>
__global__ __launch_bounds__(kBlock) void k_cg_march(CgArgs a, int k) {
  using V = typename cvec<T>::type;
  extern __shared__ char smem[];
  __shared__ double sh[4 * kQ];
  __shared__ int act;
  __shared__ double2 sc[2];
  constexpr int NR = 2 * RY + 1;
  const int s = a.sys_list[blockIdx.y];
  int tile = blockIdx.x;
  if (a.xcd_band > 0) tile = (tile & 7) * a.xcd_band + (tile >> 3);
  if (threadIdx.x == 0) act = a.st[s].active;
  __syncthreads();
  if (!act) return;
  if (!cg_prologue<kBlock>(a, k, s, tile, sh, &act, sc)) return;
  const V al = from_d2<V>(sc[0]);
  const V be = from_d2<V>(sc[1]);
  const V sft = from_d2<V>(a.shift[s]);
  const int Rx = a.Rx, SX = a.TX, SY = a.TY;
  const int PWr = SX + 4 * Rx, QWr = SX + 2 * Rx;
  V* Pr = reinterpret_cast<V*>(smem);  // [NR][PWr]: p_k rows
  V* Qr = Pr + NR * PWr;                // [NR][QWr]: r_{k+1} rows
  const int nx = a.g.nx, ny = a.g.ny;
  const int ty = fdiv(tile, a.m_ntx), tx = tile - ty * a.ntx;
  const int x0 = tx * SX, y0 = ty * SY;
  const size_t off = (size_t)s * a.g.N;
  const V* Rin = reinterpret_cast<const V*>(a.R[k & 1]) + off;
  V* Rout = reinterpret_cast<V*>(a.R[(k + 1) & 1]) + off;
  const V* Pold = reinterpret_cast<const V*>(a.P[(k + 1) & 1]) + off;
  V* Pnew = reinterpret_cast<V*>(a.P[k & 1]) + off;
  V* X = reinterpret_cast<V*>(a.X) + off;

  // this thread's positions in a P row: pos = tid and tid + 256
  int pos[2], gx[2];
  bool valid[2], inner[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    pos[j] = threadIdx.x + j * kBlock;
    valid[j] = pos[j] < PWr;
    const int ux = x0 - 2 * Rx + pos[j];
    gx[j] = pmod(ux, nx);
    inner[j] = valid[j] && pos[j] >= 2 * Rx && pos[j] < 2 * Rx + SX && ux < nx;
  }
  const int nsteps = SY + 4 * RY;
  auto load_row = [&](int i, V (&r)[2], V (&p)[2]) {
    const int gy = pmod(y0 - 2 * RY + i, ny) * nx;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (valid[j]) {
        r[j] = Rin[gy + gx[j]];
        if (k > 0) p[j] = Pold[gy + gx[j]];
      }
    }
  };
  V qr0[2], qp0[2], qr1[2], qp1[2];
  load_row(0, qr0, qp0);
  if (nsteps > 1) load_row(1, qr1, qp1);
  V rr[RY + 1][2];
  double v[kQ] = {0, 0, 0, 0, 0};
  for (int i = 0; i < nsteps; ++i) {
    V cr[2], cp[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cr[j] = qr0[j];
      cp[j] = qp0[j];
      qr0[j] = qr1[j];
      qp0[j] = qp1[j];
    }
    if (i + 2 < nsteps) load_row(i + 2, qr1, qp1);
    const int yq = y0 - 3 * RY + i;  // row whose r_{k+1} this step forms
    const bool doq = i >= 2 * RY;
    const bool storeq = doq && yq >= y0 && yq < y0 + SY && yq < ny;
    V xq[2];
    if (storeq && k > 0) {
#pragma unroll
      for (int j = 0; j < 2; ++j)
        if (inner[j]) xq[j] = X[(size_t)yq * nx + gx[j]];
    }
    // (a) p_k on the incoming row
    const int slot_in = i % NR;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (valid[j]) {
        Pr[slot_in * PWr + pos[j]] = (k > 0) ? vadd(cr[j], vmul(be, cp[j])) : cr[j];
      }
      // shift register of r_k: rr[d] holds the row brought in d steps ago
#pragma unroll
      for (int d = RY; d > 0; --d) rr[d][j] = rr[d - 1][j];
      rr[0][j] = cr[j];
    }
    __syncthreads();
    // (b) r_{k+1} = r_k - alpha A_s p_k on row yq (one-hop halo in x)
    if (doq) {
      const int iq = i - RY;
      const int sq = iq % NR;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        if (valid[j] && pos[j] >= Rx && pos[j] < PWr - Rx) {
          V acc = vzero<V>();
          if (NT > 0) {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
              const int sl = (iq + a.taps.dy[t] + NR) % NR;
              acc = vadd(acc, vscale(Pr[sl * PWr + pos[j] + a.taps.dx[t]], (T)a.taps.c[t]));
            }
          } else {
            for (int t = 0; t < a.taps.n; ++t) {
              const int sl = (iq + a.taps.dy[t] + NR) % NR;
              acc = vadd(acc, vscale(Pr[sl * PWr + pos[j] + a.taps.dx[t]], (T)a.taps.c[t]));
            }
          }
          const V p = Pr[sq * PWr + pos[j]];
          const V rn = vsub(rr[RY][j], vmul(al, vsub(p, vmul(sft, acc))));
          Qr[sq * QWr + pos[j] - Rx] = rn;
          if (storeq && inner[j]) {
            const size_t g = (size_t)yq * nx + gx[j];
            Rout[g] = rn;
            Pnew[g] = p;
            X[g] = (k == 0) ? vmul(al, p) : vadd(xq[j], vmul(al, p));
          }
        }
      }
    }
    __syncthreads();
    // (c) gamma, delta = r^T A_s r and ||r||^2 on row yw = yq - RY
    const int yw = yq - RY;
    if (i >= 3 * RY && yw >= y0 && yw < y0 + SY && yw < ny) {
      const int iw = i - 2 * RY;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        if (inner[j]) {
          const int q = pos[j] - Rx;
          V acc = vzero<V>();
          if (NT > 0) {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
              const int sl = (iw + a.taps.dy[t] + NR) % NR;
              acc = vadd(acc, vscale(Qr[sl * QWr + q + a.taps.dx[t]], (T)a.taps.c[t]));
            }
          } else {
            for (int t = 0; t < a.taps.n; ++t) {
              const int sl = (iw + a.taps.dy[t] + NR) % NR;
              acc = vadd(acc, vscale(Qr[sl * QWr + q + a.taps.dx[t]], (T)a.taps.c[t]));
            }
          }
          const V r = Qr[(iw % NR) * QWr + q];
          const V w = vsub(r, vmul(sft, acc));
          v[0] += (double)r.x * r.x - (double)r.y * r.y;
          v[1] += 2.0 * (double)r.x * r.y;
          v[2] += (double)r.x * w.x - (double)r.y * w.y;
          v[3] += (double)r.x * w.y + (double)r.y * w.x;
          v[4] += (double)r.x * r.x + (double)r.y * r.y;
        }
      }
    }
  }
  block_sum<kQ>(v, sh);
  if (threadIdx.x == 0) {
    double* pb = a.part + (a.fused ? (size_t)(k & 1) * kQ * a.num_sys * a.ntiles : 0);
#pragma unroll
    for (int q = 0; q < kQ; ++q) pb[((size_t)q * a.num_sys + s) * a.ntiles + tile] = v[q];
  }
}

// One workgroup per listed system: reduce the tile partials (fixed order) and
// advance the scalars.  k < 0: after k_cg_init; else after pass k.
__global__ __launch_bounds__(kBlock) void k_cg_scalars(CgArgs a, int k) {
  __shared__ double sh[4 * kQ];
  const int s = a.sys_list[blockIdx.x];
  SysState* st = a.st + s;
  if (!st->active) return;
  double v[kQ] = {0, 0, 0, 0, 0};
  for (int c = threadIdx.x; c < a.ntiles; c += kBlock) {
#pragma unroll
    for (int q = 0; q < kQ; ++q) v[q] += cg_part(a, q, s)[c];
  }
  block_sum<kQ>(v, sh);
  if (threadIdx.x != 0) return;
  const double2 gam = mk(v[0], v[1]);
  const double2 del = mk(v[2], v[3]);
  const double rr = v[4];
  if (k < 0) {
    st->bb = rr;
    st->rr = rr;
    st->gamma = gam;
    st->beta = mk(0, 0);
    const double d2 = del.x * del.x + del.y * del.y;
    st->alpha = (rr > 0.0 && d2 > 0.0) ? cdiv(gam, del) : mk(0, 0);  // b = 0: x stays 0
    return;
  }
  st->iters = k + 1;
  st->rr = rr;
  if (rr <= a.tol2 * st->bb) {
    st->active = 0;
    st->flag = 0;
    return;
  }
  if (k + 1 >= a.maxit) {
    st->active = 0;
    st->flag = 1;
    return;
  }
  const double2 g0 = st->gamma, a0 = st->alpha;
  const bool ok0 = (g0.x != 0.0 || g0.y != 0.0) && (a0.x != 0.0 || a0.y != 0.0);
  const double2 be = ok0 ? cdiv(gam, g0) : mk(0, 0);
  const double2 den = ok0 ? csub(del, cdiv(cmul(be, gam), a0)) : mk(0, 0);
  if (!ok0 || (den.x == 0.0 && den.y == 0.0) || !isfinite(den.x) || !isfinite(den.y)) {
    st->active = 0;
    st->flag = 2;
    return;
  }
  st->beta = be;
  st->alpha = cdiv(gam, den);
  st->gamma = gam;
}

}  // namespace

size_t cg_lds_bytes(bool f32, const CgArgs& a) {
  const size_t cs = f32 ? sizeof(float2) : sizeof(double2);
  const size_t pw = a.TX + 4 * a.Rx, ph = a.TY + 4 * a.Ry;
  return pw * ph * cs;  // the one-hop region reuses the same buffer
}

int cg_points_per_thread(const CgArgs& a) {
  const int np = (a.TX + 4 * a.Rx) * (a.TY + 4 * a.Ry);
  return (np + a.block - 1) / a.block;
}

hipError_t launch_cg_init(bool f32, const CgArgs& a, int nact, hipStream_t st) {
  dim3 grid(a.ntiles, nact);
  if (f32) hipLaunchKernelGGL(k_cg_init<float>, grid, dim3(kBlock), 0, st, a);
  else hipLaunchKernelGGL(k_cg_init<double>, grid, dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

size_t cg_march_lds_bytes(bool f32, const CgArgs& a) {
  const size_t cs = f32 ? sizeof(float2) : sizeof(double2);
  const size_t nr = 2 * a.Ry + 1;
  return nr * ((size_t)(a.TX + 4 * a.Rx) + (size_t)(a.TX + 2 * a.Rx)) * cs;
}

hipError_t launch_cg_pass(bool f32, const CgArgs& a, int k, int nact, hipStream_t st) {
  dim3 grid(a.ntiles, nact);
  if (a.march) {
    const size_t lds = cg_march_lds_bytes(f32, a);
    const int nt = (a.taps.n == 5) ? 5 : 0;
#define AAO_CGM(RY, NT)                                                                         \
  do {                                                                                          \
    if (f32) hipLaunchKernelGGL((k_cg_march<float, RY, NT>), grid, dim3(kBlock), lds, st, a, k); \
    else hipLaunchKernelGGL((k_cg_march<double, RY, NT>), grid, dim3(kBlock), lds, st, a, k);   \
  } while (0)
    if (a.Ry == 1) {
      if (nt == 5) AAO_CGM(1, 5);
      else AAO_CGM(1, 0);
    } else if (a.Ry == 2) {
      AAO_CGM(2, 0);
    } else {
      return hipErrorInvalidValue;
    }
#undef AAO_CGM
    return hipGetLastError();
  }
  const size_t lds = cg_lds_bytes(f32, a);
  const int np = cg_points_per_thread(a);
  const int nt = (a.taps.n == 3 || a.taps.n == 5) ? a.taps.n : 0;
  const int bs = a.block;
#define AAO_CGP4(NP, NT, BS)                                                                        \
  do {                                                                                              \
    if (f32) hipLaunchKernelGGL((k_cg_pass<float, NP, NT, BS>), grid, dim3(BS), lds, st, a, k);     \
    else hipLaunchKernelGGL((k_cg_pass<double, NP, NT, BS>), grid, dim3(BS), lds, st, a, k);       \
  } while (0)
#define AAO_CGP3(NP, NT)                     \
  do {                                       \
    if (bs == 512) AAO_CGP4(NP, NT, 512);    \
    else AAO_CGP4(NP, NT, 256);              \
  } while (0)
#define AAO_CGP(NP)                 \
  do {                              \
    if (nt == 3) AAO_CGP3(NP, 3);   \
    else if (nt == 5) AAO_CGP3(NP, 5); \
    else AAO_CGP3(NP, 0);           \
  } while (0)
  if (np <= 2) AAO_CGP(2);
  else if (np <= 3) AAO_CGP(3);
  else if (np <= 4) AAO_CGP(4);
  else if (np <= 6) AAO_CGP(6);
  else if (np <= kMaxPerThread) AAO_CGP(8);
  else return hipErrorInvalidValue;
#undef AAO_CGP4
#undef AAO_CGP3
#undef AAO_CGP
  return hipGetLastError();
}

hipError_t launch_cg_scalars(const CgArgs& a, int k, int nact, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_scalars, dim3(nact), dim3(kBlock), 0, st, a, k);
  return hipGetLastError();
}

}  // namespace aao
