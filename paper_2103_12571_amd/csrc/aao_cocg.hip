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
// Scalars live in SysState.  When a system has at most 256 tiles every pass
// reduces the previous pass's tile sums itself (fused); otherwise a small
// per-system kernel does it between passes.  Passes move x every other pass:
// pass k reads p_{k-1} anyway, so an odd pass applies
//   x_{k+1} = (x_{k-1} + alpha_{k-1} p_{k-1}) + alpha_k p_k
// (the same two roundings in the same order as one update per pass) and an
// even pass neither reads nor writes x.  A fused system that stops in an odd
// pass applies the update still pending from the pass before; with a scalar
// kernel between passes a last kernel does it for systems whose last pass was
// even.  Sums run in a fixed order, so
// results are bitwise reproducible.  A fused solve may change its tiling
// between passes (small tiles once few systems remain): a pass reduces the
// sums of the previous pass's tiling.
#include "aao_device.hpp"
#include "aao_kernels.hpp"

namespace aao {

namespace {

using namespace dev;

constexpr int kQ = 5;       // partial quantities: gamma (re, im), delta (re, im), ||r||^2
constexpr int kInside = 4;  // tile points per thread: TX * TY <= kInside * kBlock

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

// Taps applied to an LDS tile with row pitch W: NT > 0 unrolls a fixed count.
template <int NT, typename T, typename V>
__device__ __forceinline__ V tile_stencil(const CgArgs& a, const LdsCplx<V>& buf, int c, int W) {
  V acc = vzero<V>();
  if (NT > 0) {
#pragma unroll
    for (int t = 0; t < NT; ++t) acc = vadd(acc, vscale(buf.ld(c + a.taps.dx[t] + a.taps.dy[t] * W), (T)a.taps.c[t]));
  } else {
    for (int t = 0; t < a.taps.n; ++t)
      acc = vadd(acc, vscale(buf.ld(c + a.taps.dx[t] + a.taps.dy[t] * W), (T)a.taps.c[t]));
  }
  return acc;
}

// Outcome of advancing the scalars of one system: dec = 0 go on, 1 converged,
// 2 iteration cap, 3 breakdown; al, be = alpha_k, beta_k when dec = 0.
struct CgStep {
  int dec;
  double2 al, be;
};

// Advance from the reduced sums of r_k (gamma_k, delta_k, ||r_k||^2).  k == 0:
// the sums are those of b = r_0.
__device__ __forceinline__ CgStep cg_advance(int k, double2 gam, double2 del, double rr, double bb, double tol2,
                                             int maxit, double2 gam_prev, double2 al_prev) {
  CgStep o{0, mk(0, 0), mk(0, 0)};
  if (k == 0) {
    const double d2 = del.x * del.x + del.y * del.y;
    if (rr > 0.0 && d2 > 0.0) o.al = cdiv(gam, del);  // b = 0: x stays 0
    return o;
  }
  if (rr <= tol2 * bb) {
    o.dec = 1;
    return o;
  }
  if (k >= maxit) {
    o.dec = 2;
    return o;
  }
  if ((gam_prev.x == 0.0 && gam_prev.y == 0.0) || (al_prev.x == 0.0 && al_prev.y == 0.0)) {
    o.dec = 3;
    return o;
  }
  o.be = cdiv(gam, gam_prev);
  const double2 den = csub(del, cdiv(cmul(o.be, gam), al_prev));
  if ((den.x == 0.0 && den.y == 0.0) || !isfinite(den.x) || !isfinite(den.y)) {
    o.dec = 3;
    return o;
  }
  o.al = cdiv(gam, den);
  return o;
}

// A workgroup-uniform double (read from LDS) moved to scalar registers.
__device__ __forceinline__ double2 uniform(double2 v) {
  auto u = [](double x) {
    return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(x)),
                            __builtin_amdgcn_readfirstlane(__double2loint(x)));
  };
  return mk(u(v.x), u(v.y));
}

// Where a workgroup's tile sits: the tile origin, the widths of the two-hop
// (PW x PH) and one-hop (QW wide) regions around it, the slot counts.
struct TileGeo {
  int TX, TY, Rx, Ry, PW, PH, QW, nx, ny, x0, y0, nin, nring;
};

// XCD-aware tile order: workgroups are dealt round-robin to the 8 XCDs (each
// with its own L2), so slot b goes to XCD b % 8; give each XCD a contiguous
// band of tiles so that tile halos are read from its own L2.
__device__ __forceinline__ int tile_of_block(const CgArgs& a) {
  const int b = blockIdx.x;
  return (a.xcd_band > 0) ? (b & 7) * a.xcd_band + (b >> 3) : b;
}

__device__ __forceinline__ TileGeo tile_geo(const CgArgs& a, int tile) {
  TileGeo G;
  G.TX = a.TX;
  G.TY = a.TY;
  G.Rx = a.Rx;
  G.Ry = a.Ry;
  G.PW = G.TX + 4 * G.Rx;
  G.PH = G.TY + 4 * G.Ry;
  G.QW = G.TX + 2 * G.Rx;
  G.nx = a.g.nx;
  G.ny = a.g.ny;
  const int ty = fdiv(tile, a.m_ntx), tx = tile - ty * a.ntx;
  G.x0 = tx * G.TX;
  G.y0 = ty * G.TY;
  G.nin = G.TX * G.TY;
  G.nring = G.PW * G.PH - G.nin;
  return G;
}

// Tile slot j of thread tt: global index g, LDS index l in the two-hop layout
// (-1: no point), index q in the one-hop layout, own: stored by this tile.
// Tile points of a ragged last tile that fall outside the grid hold their
// periodic images (used as neighbours, never stored).
__device__ __forceinline__ void tile_slot(const CgArgs& a, const TileGeo& G, int tt, int j, int& g, int& l, int& q,
                                          bool& own) {
  const int i = tt + j * kBlock;
  const bool valid = i < G.nin;
  const int ii = valid ? i : 0;
  const int iy = fdiv(ii, a.m_tx), ix = ii - iy * G.TX;
  int ux = G.x0 + ix, uy = G.y0 + iy;
  own = valid && ux < G.nx && uy < G.ny;
  ux -= (ux >= G.nx) ? G.nx : 0;  // TX <= nx, TY <= ny
  uy -= (uy >= G.ny) ? G.ny : 0;
  g = uy * G.nx + ux;
  l = valid ? (iy + 2 * G.Ry) * G.PW + ix + 2 * G.Rx : -1;
  q = (iy + G.Ry) * G.QW + ix + G.Rx;
}

// Ring slot j of thread tt: 2Ry full rows above, 2Ry full rows below, then the
// rows of the tile with 2Rx points on each side; q = -1 outside the one-hop
// ring.
__device__ __forceinline__ void ring_slot(const CgArgs& a, const TileGeo& G, int tt, int j, int& g, int& l, int& q) {
  const int h = tt + j * kBlock;
  const bool valid = h < G.nring;
  const int hh = valid ? h : 0;
  const int band = 2 * G.Ry * G.PW;
  int px, py;
  if (hh < band) {
    py = fdiv(hh, a.m_pw);
    px = hh - py * G.PW;
  } else if (hh < 2 * band) {
    const int h2 = hh - band, r2 = fdiv(h2, a.m_pw);
    py = G.PH - 2 * G.Ry + r2;
    px = h2 - r2 * G.PW;
  } else {
    const int h3 = hh - 2 * band, r3 = fdiv(h3, a.m_hw), c3 = h3 - r3 * 4 * G.Rx;
    py = 2 * G.Ry + r3;
    px = (c3 < 2 * G.Rx) ? c3 : G.TX + c3;
  }
  g = pmod(G.y0 - 2 * G.Ry + py, G.ny) * G.nx + pmod(G.x0 - 2 * G.Rx + px, G.nx);
  l = valid ? py * G.PW + px : -1;
  q = (valid && px >= G.Rx && px < G.PW - G.Rx && py >= G.Ry && py < G.PH - G.Ry) ? (py - G.Ry) * G.QW + (px - G.Rx)
                                                                                     : -1;
}

// Snapshot of the systems still iterating after pass snap_k, taken by one
// extra workgroup of the next pass: stop_pass is "never" while a system
// iterates and is set once, to the pass that stops it, so a system counts as
// active iff stop_pass > snap_k, also while this very pass may be stopping it
// (that write only turns "never" into snap_k + 1).  The list is therefore the
// same as reading the active flags after pass snap_k.
__device__ __forceinline__ void cg_snapshot(const CgArgs& a) {
  __shared__ int wcnt[kBlock / 64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int total = 0;
  for (int base = 0; base < a.snap_n; base += kBlock) {
    const int i = base + t;
    const bool act = i < a.snap_n && a.st[i].stop_pass > a.snap_k;
    const unsigned long long bal = __ballot(act);
    if (lane == 0) wcnt[w] = __popcll(bal);
    __syncthreads();
    int o = total;
    for (int j = 0; j < w; ++j) o += wcnt[j];
    if (act) a.snap_list[o + __popcll(bal & ((1ull << lane) - 1))] = i;
    total += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    __syncthreads();
  }
  if (t == 0) {
    a.snap_host[0] = total;
    __threadfence_system();
    a.snap_host[1] = a.snap_tag;
  }
}

// x in a pass: XM_SKIP x untouched (k even), XM_TWO both updates (k odd).
enum : int { XM_SKIP = 1, XM_TWO = 2 };

// gamma_0 = b^T b, delta_0 = b^T A_s b, ||b||^2 over one tile: b on the tile
// and its one-hop ring in LDS (the two-hop layout of the passes), A_s b at
// the tile points.
template <typename T, int NI, int NH, int NT>
__global__ __launch_bounds__(kBlock) void k_cg_init(CgArgs a) {
  using V = typename cvec<T>::type;
  extern __shared__ char smem[];
  __shared__ double sh[4 * kQ];
  const int t = threadIdx.x;
  const int s = a.init_list ? (int)blockIdx.y : a.sys_list[blockIdx.y];
  const int tile = tile_of_block(a);
  if (a.init_list && tile == 0 && t == 0) {  // read by the passes, after this kernel
    a.st[s] = fresh_state();
    a.init_list[s] = s;
  }
  const TileGeo G = tile_geo(a, tile);
  const V* Rb = reinterpret_cast<const V*>(a.R[0]) + (size_t)s * a.g.N;
  const LdsCplx<V> Bt(smem, G.PW * G.PH);
  // every value of the tile and its ring formed before the first LDS store
  // (point by point each point's loads waited for the previous point's
  // store); a ring slot outside the one-hop ring loads the thread's first
  // tile point instead (a cache hit), so no load needs a guard
  V bi[NI], bh[NH > 0 ? NH : 1];
  int bl[NI], hl[NH > 0 ? NH : 1], g0 = 0;
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    int g, q;
    bool own;
    tile_slot(a, G, t, j, g, bl[j], q, own);
    bi[j] = Rb[g];
    if (j == 0) g0 = g;
  }
#pragma unroll
  for (int j = 0; j < NH; ++j) {
    int g, l, q;
    ring_slot(a, G, t, j, g, l, q);
    bh[j] = Rb[q >= 0 ? g : g0];
    hl[j] = (q >= 0) ? l : -1;  // the one-hop ring is enough for one stencil
  }
#pragma unroll
  for (int j = 0; j < NI; ++j)
    if (bl[j] >= 0) Bt.st(bl[j], bi[j]);
#pragma unroll
  for (int j = 0; j < NH; ++j)
    if (hl[j] >= 0) Bt.st(hl[j], bh[j]);
  __syncthreads();
  const V sft = from_d2<V>(a.shift[s]);
  double v[kQ] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    int g, l, q;
    bool own;
    tile_slot(a, G, t, j, g, l, q, own);
    if (own) {
      const V b = bi[j];
      const V w = vsub(b, vmul(sft, tile_stencil<NT, T>(a, Bt, l, G.PW)));
      v[0] += (double)b.x * b.x - (double)b.y * b.y;
      v[1] += 2.0 * (double)b.x * b.y;
      v[2] += (double)b.x * w.x - (double)b.y * w.y;
      v[3] += (double)b.x * w.y + (double)b.y * w.x;
      v[4] += (double)b.x * b.x + (double)b.y * b.y;
    }
  }
  block_sum_wave0<kQ>(v, sh);
  if (t == 0) {
    double* pb = a.part + (a.fused ? a.part_stride : 0);
#pragma unroll
    for (int q = 0; q < kQ; ++q) pb[((size_t)q * a.num_sys + s) * a.ntiles + tile] = v[q];
  }
}

// One COCG iteration for one tile of one system.  Thread t owns tile points
// t + 256 j (j < NI) and points t + 256 j of the two-hop ring around the
// tile (j < NH); it keeps r_k and then r_{k+1} of its points in registers across
// the stages.  NT > 0: the stencil has NT taps (unrolled).  NI = 1 (tiles of
// at most 256 points, used when few systems remain and the pass is bound by
// latency, not bandwidth) also requests x together with r_k and p_{k-1}.
template <typename T, int NI, int NH, int NT, int XM>
__global__ __launch_bounds__(kBlock) void k_cg_pass(CgArgs a, int k) {
  using V = typename cvec<T>::type;
  constexpr bool kEarlyX = NI == 1;
  const bool xread = XM == XM_TWO && k >= 3;  // x read: odd passes after the first
  extern __shared__ char smem[];
  __shared__ double sh[4 * kQ];
  __shared__ int act;
  __shared__ double2 sc[2];
  if ((int)blockIdx.y == a.snap_row) {  // the extra row: one workgroup takes the snapshot
    if (blockIdx.x == 0) cg_snapshot(a);
    return;
  }
  const int t = threadIdx.x;
  const int s = a.sys_list[blockIdx.y];
  const int tile = tile_of_block(a);
  const TileGeo G = tile_geo(a, tile);
  const int PW = G.PW;
  const size_t off = (size_t)s * a.g.N;
  const V* Rin = reinterpret_cast<const V*>(a.R[k & 1]) + off;
  V* Rout = reinterpret_cast<V*>(a.R[(k + 1) & 1]) + off;
  const V* Pold = reinterpret_cast<const V*>(a.P[(k + 1) & 1]) + off;
  V* Pnew = reinterpret_cast<V*>(a.P[k & 1]) + off;
  V* X = reinterpret_cast<V*>(a.X) + off;
  const LdsCplx<V> Pt(smem, G.PW * G.PH);  // p_k on the two-hop region, then r_{k+1} on the one-hop region

  // 1. What decides this pass's scalars is requested first (the previous
  //    pass's tile sums in fused mode, the system state), so that it arrives
  //    ahead of the vectors.
  double pv[kQ] = {0, 0, 0, 0, 0};
  if (a.fused && t < a.ntiles_prev) {
    const double* pp0 = a.part + ((k + 1) & 1) * a.part_stride + (size_t)s * a.ntiles_prev + t;
#pragma unroll
    for (int q = 0; q < kQ; ++q) pv[q] = pp0[(size_t)q * a.num_sys * a.ntiles_prev];
  }
  // the state is read with workgroup-uniform addresses (scalar loads)
  const SysState* st0 = a.st + s;
  // A system that stopped in an earlier pass can still be on the lagged
  // list; its workgroups leave before requesting any vector (nothing below
  // writes for it).  Every wave reads the flag itself, so it must not change
  // during this pass: in fused mode tile 0 of this very pass may stop the
  // system, so the test is on the pass that stopped it (a concurrent write
  // can only turn "never" into k, and neither leaves early); in non-fused
  // mode a separate kernel stops systems between passes.
  if (a.fused ? st0->stop_pass < k : !st0->active) return;
  const double bb0 = a.fused ? st0->bb : 0.0;
  const double2 s0 = a.fused ? st0->gamma2[(k + 1) & 1] : st0->alpha;
  const double2 s1 = a.fused ? st0->alpha2[(k + 1) & 1] : st0->beta;  // fused: alpha_{k-1}
  const double2 sap = a.fused ? s1 : st0->alpha_prev;                 // alpha_{k-1}

  // 2. r_k and p_{k-1} at the tile points and on the two-hop ring.  Tile
  //    points of a ragged last tile that fall outside the grid hold their
  //    periodic images (used as neighbours, never stored).
  V ri[NI], pi[NI], rh[NH], ph[NH], xi[NI];
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    int g, l, q;
    bool own;
    tile_slot(a, G, t, j, g, l, q, own);
    ri[j] = Rin[g];
    pi[j] = (k > 0) ? Pold[g] : vzero<V>();
    if (kEarlyX && XM != XM_SKIP) xi[j] = (xread && own) ? X[g] : vzero<V>();
  }
#pragma unroll
  for (int j = 0; j < NH; ++j) {
    int g, l, q;
    ring_slot(a, G, t, j, g, l, q);
    rh[j] = Rin[g];
    ph[j] = (k > 0) ? Pold[g] : vzero<V>();
  }

  // 3. Scalars of pass k.  Fused: every workgroup of the system reduces the
  //    tile sums of pass k-1 in the same order and takes the same decision;
  //    tile 0 records it.  Converged systems leave here.
  if (a.fused) {
    block_sum_wave0<kQ>(pv, sh);
    if (t == 0) {
      int go = 0;
      CgStep c{0, mk(0, 0), mk(0, 0)};
      {
        const double bb = (k == 0) ? (a.bbfloor ? fmax(pv[4], a.bbfloor[s]) : pv[4]) : bb0;
        c = cg_advance(k, mk(pv[0], pv[1]), mk(pv[2], pv[3]), pv[4], bb, a.tol2, a.maxit, s0, s1);
        go = c.dec == 0;
        if (tile == 0) {
          SysState* st = a.st + s;
          if (k == 0) st->bb = bb;
          st->rr = pv[4];
          if (go) {
            st->gamma2[k & 1] = mk(pv[0], pv[1]);
            st->alpha2[k & 1] = c.al;
          } else {
            st->active = 0;
            st->iters = k;
            st->flag = c.dec - 1;
            st->stop_pass = k;
          }
        }
      }
      act = go;
      sc[0] = c.al;
      sc[1] = c.be;
    }
  } else if (t == 0) {
    act = 1;  // non-fused: an inactive system left above
    sc[0] = s0;
    sc[1] = s1;
  }
  __syncthreads();
  if (!act) {
    if (XM == XM_TWO) {  // stopped: apply the update pending from pass k-1
      const V alp = from_d2<V>(sap);
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        int g, l, q;
        bool own;
        tile_slot(a, G, t, j, g, l, q, own);
        if (own) {
          const V x0 = kEarlyX ? xi[j] : (xread ? X[g] : vzero<V>());
          X[g] = vadd(x0, vmul(alp, pi[j]));
        }
      }
    }
    return;
  }
  const V al = from_d2<V>(uniform(sc[0]));
  const V be = from_d2<V>(uniform(sc[1]));
  const V sft = from_d2<V>(a.shift[s]);
  // Slot indices are recomputed here rather than kept live across the
  // scalar step (register pressure); the empty asm hides that they equal
  // the ones computed for the loads.
  int t2 = t;
  asm volatile("" : "+v"(t2));
  int li[NI], qi[NI], gi[NI], lh[NH], qh[NH];
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    int g;
    bool own;
    tile_slot(a, G, t2, j, g, li[j], qi[j], own);
    gi[j] = own ? g : -1;
  }
#pragma unroll
  for (int j = 0; j < NH; ++j) {
    int g;
    ring_slot(a, G, t2, j, g, lh[j], qh[j]);
  }

  // 4. p_k = r_k + beta_k p_{k-1} on the two-hop region
#pragma unroll
  for (int j = 0; j < NI; ++j)
    if (li[j] >= 0) Pt.st(li[j], (k > 0) ? vadd(ri[j], vmul(be, pi[j])) : ri[j]);
#pragma unroll
  for (int j = 0; j < NH; ++j)
    if (lh[j] >= 0) Pt.st(lh[j], (k > 0) ? vadd(rh[j], vmul(be, ph[j])) : rh[j]);
  if (!kEarlyX && XM != XM_SKIP) {
#pragma unroll
    for (int j = 0; j < NI; ++j) xi[j] = (xread && gi[j] >= 0) ? X[gi[j]] : vzero<V>();
  }
  if (XM == XM_TWO) {  // x_k = x_{k-1} + alpha_{k-1} p_{k-1}
    const V alp = from_d2<V>(sap);
#pragma unroll
    for (int j = 0; j < NI; ++j) xi[j] = vadd(xi[j], vmul(alp, pi[j]));
  }
  __syncthreads();

  // 5. r_{k+1} = r_k - alpha_k (p_k - c A p_k) on the one-hop region; tile
  //    points store r_{k+1}, p_k, x_{k+1}
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    if (li[j] >= 0) {
      const V acc = tile_stencil<NT, T>(a, Pt, li[j], PW);
      const V p = Pt.ld(li[j]);
      ri[j] = vsub(ri[j], vmul(al, vsub(p, vmul(sft, acc))));
      if (gi[j] >= 0) {
        Rout[gi[j]] = ri[j];
        Pnew[gi[j]] = p;
        if (XM != XM_SKIP) X[gi[j]] = vadd(xi[j], vmul(al, p));
      }
    }
    // one point at a time: keeps the stencil operands of different points
    // from being live together (register pressure -> occupancy)
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int j = 0; j < NH; ++j) {
    if (qh[j] >= 0) {
      const V acc = tile_stencil<NT, T>(a, Pt, lh[j], PW);
      rh[j] = vsub(rh[j], vmul(al, vsub(Pt.ld(lh[j]), vmul(sft, acc))));
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  __syncthreads();
  const LdsCplx<V>& Rt = Pt;
#pragma unroll
  for (int j = 0; j < NI; ++j)
    if (li[j] >= 0) Rt.st(qi[j], ri[j]);
#pragma unroll
  for (int j = 0; j < NH; ++j)
    if (qh[j] >= 0) Rt.st(qh[j], rh[j]);
  __syncthreads();

  // 6. gamma_{k+1}, delta_{k+1} = r^T A_s r and ||r_{k+1}||^2 over the tile
  double v[kQ] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    if (gi[j] >= 0) {
      const V acc = tile_stencil<NT, T>(a, Rt, qi[j], G.QW);
      const V r = ri[j];
      const V w = vsub(r, vmul(sft, acc));
      v[0] += (double)r.x * r.x - (double)r.y * r.y;
      v[1] += 2.0 * (double)r.x * r.y;
      v[2] += (double)r.x * w.x - (double)r.y * w.y;
      v[3] += (double)r.x * w.y + (double)r.y * w.x;
      v[4] += (double)r.x * r.x + (double)r.y * r.y;
    }
  }
  block_sum_wave0<kQ>(v, sh);
  if (t == 0) {
    double* pb = a.part + (a.fused ? (k & 1) * a.part_stride : 0);
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
  block_sum_wave0<kQ>(v, sh);
  if (threadIdx.x != 0) return;
  const double2 gam = mk(v[0], v[1]);
  const double2 del = mk(v[2], v[3]);
  const double rr = v[4];
  if (k < 0) {
    st->bb = a.bbfloor ? fmax(rr, a.bbfloor[s]) : rr;
    st->rr = rr;
    st->gamma = gam;
    st->beta = mk(0, 0);
    const double d2 = del.x * del.x + del.y * del.y;
    st->alpha = (rr > 0.0 && d2 > 0.0) ? cdiv(gam, del) : mk(0, 0);  // b = 0: x stays 0
    st->alpha_prev = mk(0, 0);
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
  st->alpha_prev = a0;
  st->alpha = cdiv(gam, den);
  st->gamma = gam;
}

// The update a system's last pass k = iters - 1 left pending when k is even:
// x_{k+1} = x_k + alpha_k p_k (x_k = 0 when k = 0); alpha_k is still in the
// state (a stopping scalar step leaves it), p_k in P[k & 1].
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_xfix(CgArgs a) {
  using V = typename cvec<T>::type;
  const int s = blockIdx.y;
  const SysState* st = a.st + s;
  const int k = st->iters - 1;
  if (k < 0 || (k & 1)) return;
  const size_t off = (size_t)s * a.g.N;
  const V* Pk = reinterpret_cast<const V*>(a.P[k & 1]) + off;
  V* X = reinterpret_cast<V*>(a.X) + off;
  const V al = from_d2<V>(st->alpha);
  for (int n = blockIdx.x * kBlock + threadIdx.x; n < a.g.N; n += gridDim.x * kBlock)
    X[n] = vadd(k > 0 ? X[n] : vzero<V>(), vmul(al, Pk[n]));
}


// ----------------------------------------------------------------------------
// Batched BiCGStab on the COCG tiles (2D grids, at most 256 tiles per
// system): the two phases with a matrix-vector product form their vector on
// the tile and its one-hop ring in LDS (read once per point, the ring's
// points recomputed from their own inputs) and apply the stencil from there,
// instead of rebuilding the vector at every neighbour from global memory.
// Grid (tiles, active systems); tile t writes chunk t of the partial sums.
// Scalars, stopping test and breakdown flags are those of the chunked
// kernels (aao_kernels.hip, k_bicg1 and k_bicg2); the update phase (k_bicg3)
// is shared, with as many chunks as there are tiles.

// Phase 1: convergence test, beta, p = r + beta (p_old - omega v_old),
// v = (I - cA) p, partial <r_hat, v> (k = 0: p = r_hat = r, <r, r>).
template <typename T, int NI, int NH, int NT>
__global__ __launch_bounds__(kBlock) void k_bicg_t1(CgArgs g, KrylovArgs a, int k) {
  using V = typename cvec<T>::type;
  extern __shared__ char smem[];
  __shared__ double sh[4 * 8];
  __shared__ int act;
  const int t = threadIdx.x;
  const int s = a.sys_list[blockIdx.y];
  SysState* st = a.st + s;
  const int tile = tile_of_block(g);
  // one read of the flag per workgroup (tile 0 may clear it concurrently)
  if (t == 0) act = st->active;
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
  V bt = vzero<V>(), om = vzero<V>();
  if (k > 0) {
    const int qs[4] = {QP_RHO0_RE + 2 * cur, QP_RHO0_IM + 2 * cur, QP_RR0 + cur, QP_BB};
    const int nw[4] = {a.wps_rho, a.wps_rho, a.wps_rho, a.wps_bb};
    double v[4];
    reduce_parts<4>(a, qs, nw, s, v, sh);
    const bool conv = v[2] <= a.tol2 * (a.bbfloor ? fmax(v[3], a.bbfloor[s]) : v[3]);
    if (conv || k >= a.maxit || st->breakdown) {
      if (tile == 0 && t == 0) {
        st->active = 0;
        st->iters = k;
        st->flag = conv ? 0 : (st->breakdown ? 2 : 1);
      }
      return;
    }
    const double2 rho = mk(v[0], v[1]);
    bt = from_d2<V>(cmul(cdiv(rho, st->rho), cdiv(st->alpha, st->omega)));
    om = from_d2<V>(st->omega);
  }
  // p at a point (k = 0: r) from its r, p_{k-1}, v_{k-1}; the three loads are
  // made whatever k is (the buffers always exist), so that every point's
  // loads can be in flight together
  struct Prv { V r, po, vo; };
  auto pload = [&](int i) { return Prv{R[i], Po[i], Vo[i]}; };
  auto pform = [&](const Prv& x) { return k == 0 ? x.r : vadd(x.r, vmul(bt, vsub(x.po, vmul(om, x.vo)))); };
  const TileGeo G = tile_geo(g, tile);
  const LdsCplx<V> Pt(smem, G.PW * G.PH);
  // every value of the tile and its ring formed before the first LDS store
  // (point by point each point's loads waited for the previous point's
  // store); a ring slot outside the one-hop ring loads the thread's first
  // tile point instead (a cache hit), so no load needs a guard
  Prv xi[NI], xh[NH > 0 ? NH : 1];
  int pl[NI], hl[NH > 0 ? NH : 1], g0 = 0;
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    int gi, q;
    bool own;
    tile_slot(g, G, t, j, gi, pl[j], q, own);
    xi[j] = pload(gi);
    if (j == 0) g0 = gi;
  }
#pragma unroll
  for (int j = 0; j < NH; ++j) {
    int gi, l, q;
    ring_slot(g, G, t, j, gi, l, q);
    xh[j] = pload(q >= 0 ? gi : g0);
    hl[j] = (q >= 0) ? l : -1;  // one stencil: the one-hop ring is enough
  }
  V pv[NI], ph[NH > 0 ? NH : 1];
#pragma unroll
  for (int j = 0; j < NI; ++j) pv[j] = pform(xi[j]);
#pragma unroll
  for (int j = 0; j < NH; ++j) ph[j] = pform(xh[j]);
#pragma unroll
  for (int j = 0; j < NI; ++j)
    if (pl[j] >= 0) Pt.st(pl[j], pv[j]);
#pragma unroll
  for (int j = 0; j < NH; ++j)
    if (hl[j] >= 0) Pt.st(hl[j], ph[j]);
  __syncthreads();
  double hv_re = 0, hv_im = 0, bb = 0;
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    int gi, l, q;
    bool own;
    tile_slot(g, G, t, j, gi, l, q, own);
    if (own) {
      const V p = pv[j];
      const V v = vsub(p, vmul(sft, tile_stencil<NT, T>(g, Pt, l, G.PW)));
      Pn[gi] = p;
      Vn[gi] = v;
      if (k == 0) {
        Rh[gi] = p;
        hv_re += (double)p.x * v.x + (double)p.y * v.y;
        hv_im += (double)p.x * v.y - (double)p.y * v.x;
        bb += (double)p.x * p.x + (double)p.y * p.y;
      } else {
        const V rh = Rh[gi];
        hv_re += (double)rh.x * v.x + (double)rh.y * v.y;
        hv_im += (double)rh.x * v.y - (double)rh.y * v.x;
      }
    }
  }
  if (k == 0) {
    // rho_0 = <r_hat, r> = ||b||^2 (real)
    double w[4] = {hv_re, hv_im, bb, bb};
    const int qs[4] = {QP_A_RE, QP_A_IM, QP_BB, QP_RHO0_RE};
    write_parts<4>(a, qs, s, tile, w, sh);
    if (t == 0) qpart(a, QP_RHO0_IM, s)[tile] = 0.0;
  } else {
    double w[2] = {hv_re, hv_im};
    const int qw[2] = {QP_A_RE, QP_A_IM};
    write_parts<2>(a, qw, s, tile, w, sh);
  }
}

// Phase 2: alpha = rho_k / <r_hat, v>; s = r - alpha v; t = (I - cA) s;
// partials <t, s>, <t, t>.  Tile 0 records rho_k and alpha_k.
template <typename T, int NI, int NH, int NT>
__global__ __launch_bounds__(kBlock) void k_bicg_t2(CgArgs g, KrylovArgs a, int k) {
  using V = typename cvec<T>::type;
  extern __shared__ char smem[];
  __shared__ double sh[4 * 8];
  __shared__ int act;
  const int t = threadIdx.x;
  const int s = a.sys_list[blockIdx.y];
  SysState* st = a.st + s;
  const int tile = tile_of_block(g);
  if (t == 0) act = st->active;
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
  else if (tile == 0 && t == 0 && (rho.x != 0.0 || rho.y != 0.0)) st->breakdown = 1;
  if (tile == 0 && t == 0) {
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
  auto sval = [&](int i) { return vsub(R[i], vmul(av, Vc[i])); };
  const TileGeo G = tile_geo(g, tile);
  const LdsCplx<V> St(smem, G.PW * G.PH);
  // every value of the tile and its ring formed before the first LDS store
  // (point by point each point's loads waited for the previous point's
  // store); a ring slot outside the one-hop ring loads the thread's first
  // tile point instead (a cache hit), so no load needs a guard
  V sv[NI], sh2[NH > 0 ? NH : 1];
  int sl[NI], hl[NH > 0 ? NH : 1], g0 = 0;
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    int gi, q;
    bool own;
    tile_slot(g, G, t, j, gi, sl[j], q, own);
    sv[j] = sval(gi);
    if (j == 0) g0 = gi;
  }
#pragma unroll
  for (int j = 0; j < NH; ++j) {
    int gi, l, q;
    ring_slot(g, G, t, j, gi, l, q);
    sh2[j] = sval(q >= 0 ? gi : g0);
    hl[j] = (q >= 0) ? l : -1;
  }
#pragma unroll
  for (int j = 0; j < NI; ++j)
    if (sl[j] >= 0) St.st(sl[j], sv[j]);
#pragma unroll
  for (int j = 0; j < NH; ++j)
    if (hl[j] >= 0) St.st(hl[j], sh2[j]);
  __syncthreads();
  double ts_re = 0, ts_im = 0, tt = 0;
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    int gi, l, q;
    bool own;
    tile_slot(g, G, t, j, gi, l, q, own);
    if (own) {
      const V x = sv[j];
      const V tv = vsub(x, vmul(sft, tile_stencil<NT, T>(g, St, l, G.PW)));
      Sv[gi] = x;
      Tv[gi] = tv;
      ts_re += (double)tv.x * x.x + (double)tv.y * x.y;
      ts_im += (double)tv.x * x.y - (double)tv.y * x.x;
      tt += (double)tv.x * tv.x + (double)tv.y * tv.y;
    }
  }
  double w[3] = {ts_re, ts_im, tt};
  const int qs[3] = {QP_B_RE, QP_B_IM, QP_TT};
  write_parts<3>(a, qs, s, tile, w, sh);
}
}  // namespace

size_t cg_lds_bytes(bool f32, const CgArgs& a) {
  const int n = (a.TX + 4 * a.Rx) * (a.TY + 4 * a.Ry);  // the one-hop region reuses the same buffer
  return f32 ? LdsCplx<float2>::bytes(n) : LdsCplx<double2>::bytes(n);
}

int cg_ring_slots(const CgArgs& a) {
  const int nring = (a.TX + 4 * a.Rx) * (a.TY + 4 * a.Ry) - a.TX * a.TY;
  return (nring + kBlock - 1) / kBlock;
}

hipError_t launch_cg_init(bool f32, const CgArgs& a, int nact, hipStream_t st) {
  if (a.TX * a.TY > kInside * kBlock) return hipErrorInvalidValue;
  dim3 grid(a.ntiles, nact);
  const size_t lds = cg_lds_bytes(f32, a);
  const int nh = cg_ring_slots(a);
  const int nt = (a.taps.n == 3 || a.taps.n == 5) ? a.taps.n : 0;
  const bool one = a.TX * a.TY <= kBlock;
#define AAO_CGI3(NI, NH, NT)                                                                        \
  do {                                                                                              \
    if (f32) hipLaunchKernelGGL((k_cg_init<float, NI, NH, NT>), grid, dim3(kBlock), lds, st, a);    \
    else hipLaunchKernelGGL((k_cg_init<double, NI, NH, NT>), grid, dim3(kBlock), lds, st, a);       \
  } while (0)
#define AAO_CGI2(NH, NT)             \
  do {                               \
    if (one) AAO_CGI3(1, NH, NT);    \
    else AAO_CGI3(kInside, NH, NT);  \
  } while (0)
#define AAO_CGI(NH)                      \
  do {                                   \
    if (nt == 3) AAO_CGI2(NH, 3);        \
    else if (nt == 5) AAO_CGI2(NH, 5);   \
    else AAO_CGI2(NH, 0);                \
  } while (0)
  if (nh <= 1) AAO_CGI(1);
  else if (nh <= 2) AAO_CGI(2);
  else if (nh <= 4) AAO_CGI(4);
  else if (nh <= 8) AAO_CGI(8);
  else return hipErrorInvalidValue;
#undef AAO_CGI3
#undef AAO_CGI2
#undef AAO_CGI
  return hipGetLastError();
}

hipError_t launch_cg_pass(bool f32, const CgArgs& a, int k, int nact, hipStream_t st) {
  if (a.TX * a.TY > kInside * kBlock) return hipErrorInvalidValue;
  if (a.fused && (a.ntiles > kBlock || a.ntiles_prev < 1 || a.ntiles_prev > kBlock)) return hipErrorInvalidValue;
  if (a.snap_row >= 0 && (!a.fused || a.snap_row != nact || !a.snap_list || !a.snap_host || a.snap_n < 1 ||
                          a.snap_n > a.num_sys))
    return hipErrorInvalidValue;
  dim3 grid(a.ntiles, nact + (a.snap_row >= 0 ? 1 : 0));
  const size_t lds = cg_lds_bytes(f32, a);
  const int nh = cg_ring_slots(a);
  const int nt = (a.taps.n == 3 || a.taps.n == 5) ? a.taps.n : 0;
  const bool one = a.TX * a.TY <= kBlock;
#define AAO_CGP4(NI, NH, NT, XM)                                                                        \
  do {                                                                                                  \
    if (f32) hipLaunchKernelGGL((k_cg_pass<float, NI, NH, NT, XM>), grid, dim3(kBlock), lds, st, a, k); \
    else hipLaunchKernelGGL((k_cg_pass<double, NI, NH, NT, XM>), grid, dim3(kBlock), lds, st, a, k);    \
  } while (0)
#define AAO_CGP3(NI, NH, NT)                 \
  do {                                       \
    if (k & 1) AAO_CGP4(NI, NH, NT, XM_TWO); \
    else AAO_CGP4(NI, NH, NT, XM_SKIP);      \
  } while (0)
#define AAO_CGP2(NH, NT)         \
  do {                           \
    if (one) AAO_CGP3(1, NH, NT); \
    else AAO_CGP3(kInside, NH, NT); \
  } while (0)
#define AAO_CGP(NH)                  \
  do {                               \
    if (nt == 3) AAO_CGP2(NH, 3);    \
    else if (nt == 5) AAO_CGP2(NH, 5); \
    else AAO_CGP2(NH, 0);            \
  } while (0)
  if (nh <= 1) AAO_CGP(1);
  else if (nh <= 2) AAO_CGP(2);
  else if (nh <= 4) AAO_CGP(4);
  else if (nh <= 8) AAO_CGP(8);
  else return hipErrorInvalidValue;
#undef AAO_CGP4
#undef AAO_CGP3
#undef AAO_CGP2
#undef AAO_CGP
  return hipGetLastError();
}

hipError_t launch_cg_scalars(const CgArgs& a, int k, int nact, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_scalars, dim3(nact), dim3(kBlock), 0, st, a, k);
  return hipGetLastError();
}

hipError_t launch_cg_xfix(bool f32, const CgArgs& a, int nsys, hipStream_t st) {
  if (nsys < 1 || nsys > 65535) return hipErrorInvalidValue;
  const int blocks = std::max(1, std::min((a.g.N + kBlock - 1) / kBlock, 1024));
  dim3 grid(blocks, nsys);
  if (f32) hipLaunchKernelGGL(k_cg_xfix<float>, grid, dim3(kBlock), 0, st, a);
  else hipLaunchKernelGGL(k_cg_xfix<double>, grid, dim3(kBlock), 0, st, a);
  return hipGetLastError();
}


bool bicg_tiled_fits(const CgArgs& g) {
  return g.TX * g.TY <= kInside * kBlock && g.ntiles <= kBlock && cg_ring_slots(g) <= 8;
}

hipError_t launch_bicg_tiled(int phase, bool f32, const CgArgs& g, const KrylovArgs& a, int k, int nact,
                             hipStream_t st) {
  if (!bicg_tiled_fits(g) || a.wps != g.ntiles || a.wps > a.wps_stride || a.wps_rho < 1 ||
      a.wps_rho > a.wps_stride || a.wps_bb < 1 || a.wps_bb > a.wps_stride || (phase != 1 && phase != 2))
    return hipErrorInvalidValue;
  dim3 grid(g.ntiles, nact);
  const size_t lds = cg_lds_bytes(f32, g);
  const int nh = cg_ring_slots(g);
  const int nt = (g.taps.n == 3 || g.taps.n == 5) ? g.taps.n : 0;
  const bool one = g.TX * g.TY <= kBlock;
#define AAO_BT4(T, NI, NH, NT)                                                                          \
  do {                                                                                                  \
    if (phase == 1) hipLaunchKernelGGL((k_bicg_t1<T, NI, NH, NT>), grid, dim3(kBlock), lds, st, g, a, k); \
    else hipLaunchKernelGGL((k_bicg_t2<T, NI, NH, NT>), grid, dim3(kBlock), lds, st, g, a, k);           \
  } while (0)
#define AAO_BT3(NI, NH, NT)                 \
  do {                                      \
    if (f32) AAO_BT4(float, NI, NH, NT);    \
    else AAO_BT4(double, NI, NH, NT);       \
  } while (0)
#define AAO_BT2(NH, NT)                 \
  do {                                  \
    if (one) AAO_BT3(1, NH, NT);        \
    else AAO_BT3(kInside, NH, NT);      \
  } while (0)
#define AAO_BT(NH)                      \
  do {                                  \
    if (nt == 3) AAO_BT2(NH, 3);        \
    else if (nt == 5) AAO_BT2(NH, 5);   \
    else AAO_BT2(NH, 0);                \
  } while (0)
  if (nh <= 1) AAO_BT(1);
  else if (nh <= 2) AAO_BT(2);
  else if (nh <= 4) AAO_BT(4);
  else AAO_BT(8);
#undef AAO_BT4
#undef AAO_BT3
#undef AAO_BT2
#undef AAO_BT
  return hipGetLastError();
}

}  // namespace aao
