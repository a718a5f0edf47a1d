// Spatial-FFT direct solve of the shifted systems (I - c_s A) x_s = b_s (row
// a3, variant for periodic constant-coefficient A).
//
// A periodic stencil is diagonalised by the DFT: for the mode e^{2 pi i k.n/N}
// it acts as lambda(k) = sum_t c_t e^{2 pi i (kx dx_t / nx + ky dy_t / ny)}, so
// x = F^{-1}[ F b / (1 - c_s lambda(k)) ] exactly.  Transforms run in LDS with
// radix-2 butterflies: decimation in frequency (natural input, bit-reversed
// output) forward, decimation in time (bit-reversed input, natural output) for
// the inverse, so spectra stay in bit-reversed order between the two and no
// reordering pass is needed; the divide takes the frequency of a position as
// its bit reversal.  1D: one workgroup per system does forward, divide and
// inverse.  2D: rows forward (in place; a row's spectrum is left in
// bit-reversed kx order), then columns forward + divide + inverse (in place),
// then rows inverse into x.
//
// A length n that is not a power of two goes through Bluestein's chirp-z form
// of the DFT: with jk = (j^2 + k^2 - (k - j)^2) / 2, X_k = ch_k (a * b)_k for
// a_j = ch_j x_j and b_m = conj(ch_m), ch_j = e^{-i pi j^2 / n}, where * is a
// cyclic convolution of length P >= 2n - 1 done by radix-2 transforms (the
// inverse DFT uses the conjugate chirps).  Between a forward and an inverse
// transform of the same data the outgoing and incoming chirps cancel, so the
// divide step only scales the convolution by 1 / (P (1 - c lambda)).
#include "aao_device.hpp"
#include "aao_kernels.hpp"

namespace aao {

namespace {

using namespace dev;

template <typename V> struct scal;
template <> struct scal<double2> { using type = double; };
template <> struct scal<float2> { using type = float; };

// LDS index of transform element i: one pad slot after every eight elements,
// so that the eight-element groups of the first and last FFT passes (and
// lines that sit a power of two apart) fall into different banks.
__device__ __forceinline__ int padi(int i) { return i + (i >> 3); }

// a / b for a >= 0, b > 0 (unsigned: a power-of-two constant b is a shift)
__device__ __forceinline__ int udiv(int a, int b) { return (int)((unsigned)a / (unsigned)b); }

// Copy elements i = threadIdx.x + nth j (i < tot) of global memory into LDS,
// kLdBatch per thread at a time: every load of a batch is issued before the
// first LDS store (a loop of load-then-store waits out one memory round trip
// per element).  get(i) loads element i, put(i, v) stores it.
constexpr int kLdBatch = 8;
template <typename V, typename Get, typename Put>
__device__ __forceinline__ void load_to_lds(int tot, int nth, const Get& get, const Put& put) {
  for (int i0 = threadIdx.x; i0 < tot; i0 += kLdBatch * nth) {
    V v[kLdBatch];
#pragma unroll
    for (int j = 0; j < kLdBatch; ++j) {
      const int i = i0 + j * nth;
      v[j] = (i < tot) ? get(i) : vzero<V>();
    }
#pragma unroll
    for (int j = 0; j < kLdBatch; ++j) {
      const int i = i0 + j * nth;
      if (i < tot) put(i, v[j]);
    }
  }
}

// v e^{2 pi i e / 8} for e in 0 .. 3 (the roots of unity that separate the
// twiddles of one group).
__device__ __forceinline__ double2 root8_mul(double2 v, int e) {
  constexpr double h = 0.70710678118654752440;  // cos(pi / 4)
  if (e == 0) return v;
  if (e == 1) return mk((v.x - v.y) * h, (v.x + v.y) * h);
  if (e == 2) return mk(-v.y, v.x);
  return mk(-(v.x + v.y) * h, (v.x - v.y) * h);
}

// Radix-2 stages on a group of 2^K elements held in registers: element t is
// transform element i0 + t 2^slo (bits slo .. slo+K-1 of i0 clear, pos0 =
// i0 mod 2^slo).  DIT: stages slo .. slo+K-1 with butterflies (a, b) -> (a +
// w b, a - w b); DIF: stages slo+K-1 down to slo with (a, d) -> (a + d,
// (a - d) w).  Stage slo+q pairs t and t + 2^q (bit q of t clear) with the
// twiddle e^{2 pi i (pos0 + j 2^slo) / 2^(slo+q+1)}, j = t mod 2^q, which is
// w^(2^(K-1-q)) e^{2 pi i j / 2^(q+1)} for the group's base twiddle w =
// e^{2 pi i pos0 / 2^(slo+K)}: one table read per group, the rest by complex
// squaring and eighth roots of unity.  The forward transform takes the
// conjugates.
template <typename V, bool DIT, bool INV, int K>
__device__ __forceinline__ void group_stages(V (&v)[1 << K], double2 w) {
  using T = typename scal<V>::type;
  constexpr int R = 1 << K;
  double2 wq[K];
  wq[K - 1] = w;
#pragma unroll
  for (int q = K - 2; q >= 0; --q) wq[q] = cmul(wq[q + 1], wq[q + 1]);
#pragma unroll
  for (int qq = 0; qq < K; ++qq) {
    const int q = DIT ? qq : K - 1 - qq;
    const int half = 1 << q;
    V tw[R / 2];
#pragma unroll
    for (int j = 0; j < half; ++j) {
      const double2 wd = root8_mul(wq[q], j << (2 - q));
      tw[j].x = (T)wd.x;
      tw[j].y = INV ? (T)wd.y : (T)-wd.y;
    }
#pragma unroll
    for (int t = 0; t < R; ++t) {
      if (t & half) continue;
      const V wt = tw[t & (half - 1)];
      const V a = v[t];
      if (DIT) {
        const V b = vmul(wt, v[t + half]);
        v[t] = vadd(a, b);
        v[t + half] = vsub(a, b);
      } else {
        const V d = v[t + half];
        v[t] = vadd(a, d);
        v[t + half] = vmul(vsub(a, d), wt);
      }
    }
  }
}

// One pass of K stages over nb transforms of length n in LDS (element (b, i)
// at b sb + padi(i) se), one group of 2^K elements per thread and trip.  W:
// e^{+2 pi i k / n} (k < n / 2 is read), in global memory.
// MID (the lowest stages, slo = 0): DIF forward stages, the element-wise
// multiply by mul(b, k) at frequency k (element i holds frequency bitrev(i)),
// then the same stages as DIT inverse (the last forward pass, the divide and
// the first inverse pass of a forward-divide-inverse solve in one trip).
// FASTB: consecutive threads take consecutive transforms (b).
template <typename V, bool DIT, bool INV, bool FASTB, int K, bool MID = false, typename Mul = int>
__device__ __forceinline__ void fft_pass(const LdsCplx<V>& c, const double2* W, int n, int logn, int slo, int nb,
                                         int sb, int se, int nth, const Mul& mul = 0) {
  constexpr int R = 1 << K;
  const int lng = logn - K;  // 2^lng groups per transform
  const int span = 1 << slo;
  const int wstride = n >> (slo + K);
  __syncthreads();
  for (int idx = threadIdx.x; idx < (nb << lng); idx += nth) {
    const int g = FASTB ? udiv(idx, nb) : idx & ((1 << lng) - 1);
    const int b = FASTB ? idx - g * nb : idx >> lng;
    const int pos0 = g & (span - 1);
    const int i0 = ((g >> slo) << (slo + K)) + pos0;
    const int base = b * sb;
    const double2 w = W[pos0 * wstride];
    V v[R];
#pragma unroll
    for (int t = 0; t < R; ++t) v[t] = c.ld(base + padi(i0 + t * span) * se);
    if constexpr (MID) {
      group_stages<V, false, false, K>(v, w);
#pragma unroll
      for (int t = 0; t < R; ++t) v[t] = vmul(v[t], mul(b, bitrev(i0 + t * span, logn)));
      group_stages<V, true, true, K>(v, w);
    } else {
      group_stages<V, DIT, INV, K>(v, w);
    }
#pragma unroll
    for (int t = 0; t < R; ++t) c.st(base + padi(i0 + t * span) * se, v[t]);
  }
}

template <typename V, bool DIT, bool INV, bool FASTB>
__device__ __forceinline__ void fft_pass_k(const LdsCplx<V>& c, const double2* W, int n, int logn, int slo, int k,
                                           int nb, int sb, int se, int nth) {
  if (k == 3) fft_pass<V, DIT, INV, FASTB, 3>(c, W, n, logn, slo, nb, sb, se, nth);
  else if (k == 2) fft_pass<V, DIT, INV, FASTB, 2>(c, W, n, logn, slo, nb, sb, se, nth);
  else fft_pass<V, DIT, INV, FASTB, 1>(c, W, n, logn, slo, nb, sb, se, nth);
}

// DIT passes over stages lo .. logn-1 (upwards, three at a time, the last
// pass partial) and DIF passes over stages logn-1 down to lo.
template <typename V, bool INV, bool FASTB>
__device__ __forceinline__ void dit_passes(const LdsCplx<V>& c, const double2* W, int n, int logn, int lo, int nb,
                                           int sb, int se, int nth) {
  for (int slo = lo; slo < logn; slo += 3)
    fft_pass_k<V, true, INV, FASTB>(c, W, n, logn, slo, min(3, logn - slo), nb, sb, se, nth);
}
template <typename V, bool INV, bool FASTB>
__device__ __forceinline__ void dif_passes(const LdsCplx<V>& c, const double2* W, int n, int logn, int lo, int nb,
                                           int sb, int se, int nth) {
  for (int hi = logn; hi > lo; hi -= 3) {
    const int k = min(3, hi - lo);
    fft_pass_k<V, false, INV, FASTB>(c, W, n, logn, hi - k, k, nb, sb, se, nth);
  }
}

// Forward transform (DIF: natural input, bit-reversed output), element-wise
// multiply by mul(b, k) at frequency k, inverse transform (DIT: bit-reversed
// input, natural output), with the last forward pass, the multiply and the
// first inverse pass (stages 0 .. 2) in one trip.
template <typename V, bool FASTB, typename Mul>
__device__ __forceinline__ void fft_mul_ifft(const LdsCplx<V>& c, const double2* W, int n, int logn, int nb, int sb,
                                             int se, int nth, const Mul& mul) {
  const int km = min(3, logn);
  dif_passes<V, false, FASTB>(c, W, n, logn, km, nb, sb, se, nth);
  if (km == 3) fft_pass<V, true, false, FASTB, 3, true>(c, W, n, logn, 0, nb, sb, se, nth, mul);
  else if (km == 2) fft_pass<V, true, false, FASTB, 2, true>(c, W, n, logn, 0, nb, sb, se, nth, mul);
  else if (km == 1) fft_pass<V, true, false, FASTB, 1, true>(c, W, n, logn, 0, nb, sb, se, nth, mul);
  else {  // n = 1: the transforms are the identity
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += nth) c.st(b * sb, vmul(c.ld(b * sb), mul(b, 0)));
  }
  dit_passes<V, true, FASTB>(c, W, n, logn, km, nb, sb, se, nth);
  __syncthreads();
}

// (k d) mod n for a tap offset d in [-4, 4]
__device__ __forceinline__ int tap_mod(int v, int n, int pow2) { return pow2 ? (v & (n - 1)) : ((v % n) + n) % n; }

// The symbol lambda(kx, ky) = sum_t c_t e^{2 pi i (kx dx_t / nx + ky dy_t / ny)}
// in three parts: taps along x (dy = 0), taps along y (dx = 0, dy != 0) and
// the rest (both offsets nonzero; a.diag says whether there are any), so that
// a column's x part is summed once.
__device__ __forceinline__ double2 sym_x(const FftArgs& a, int kx) {
  double2 lam = mk(0, 0);
  for (int t = 0; t < a.taps.n; ++t) {
    if (a.taps.dy[t] != 0) continue;
    const double2 e = a.Wx[tap_mod(kx * a.taps.dx[t], a.nx, a.px2)];
    lam.x += a.taps.c[t] * e.x;
    lam.y += a.taps.c[t] * e.y;
  }
  return lam;
}
__device__ __forceinline__ double2 sym_rest(const FftArgs& a, int kx, int ky) {
  double2 lam = mk(0, 0);
  for (int t = 0; t < a.taps.n; ++t) {
    const int dx = a.taps.dx[t], dy = a.taps.dy[t];
    if (dy == 0 || (dx != 0 && !a.diag)) continue;
    double2 e = a.Wy[tap_mod(ky * dy, a.ny, a.py2)];
    if (dx != 0) e = cmul(a.Wx[tap_mod(kx * dx, a.nx, a.px2)], e);
    lam.x += a.taps.c[t] * e.x;
    lam.y += a.taps.c[t] * e.y;
  }
  return lam;
}
// 1 / ((1 - c lambda) * nx * ny): the inverse transforms are unnormalised.
__device__ __forceinline__ double2 inv_den(const FftArgs& a, double2 c, double2 lam) {
  const double2 den = mk((1.0 - (c.x * lam.x - c.y * lam.y)) * a.norm, (-(c.x * lam.y + c.y * lam.x)) * a.norm);
  return cdiv(mk(1, 0), den);
}
__device__ __forceinline__ double2 inv_symbol(const FftArgs& a, double2 c, int kx, int ky) {
  return inv_den(a, c, cadd(sym_x(a, kx), sym_rest(a, kx, ky)));
}

// Bluestein convolution of nb sequences of length P held in c (element (b, i)
// at b * sb + padi(i) * se) in natural order: forward radix-2 transform,
// multiply by the filter's transform F, inverse radix-2 transform.  Leaves P
// times the cyclic convolution, again in natural order.
template <typename V, bool FASTB>
__device__ __forceinline__ void blue_conv(const LdsCplx<V>& c, const BlueDim& d, const double2* F, int nb, int sb,
                                          int se, int nth) {
  fft_mul_ifft<V, FASTB>(c, d.W, d.P, d.logP, nb, sb, se, nth, [&](int, int k) { return from_d2<V>(F[k]); });
}

__device__ __forceinline__ double2 cscale(double2 v, double s) { return mk(v.x * s, v.y * s); }

// Frequency kx of column x of a row spectrum: radix-2 rows leave their
// spectra in bit-reversed order, Bluestein rows in natural order.
__device__ __forceinline__ int kx_of(const FftArgs& a, int x) { return a.bx.P > 0 ? x : bitrev(x, a.lognx); }

// Threads of the column kernel: one per group of eight elements of the
// tile (cols x line), at least 64 and at most 1024 (launch_fft_solve).

// Rows: MODE 0 forward (in place), MODE 1 inverse (R -> X), MODE 2 forward,
// divide and inverse (1D, R -> X).  grid (ny / rows, nsys).  Row r of the
// tile starts at r * padi(line) in LDS.  BLUE: nx is transformed through
// length-P convolutions.
template <typename V, int MODE, bool BLUE>
__global__ __launch_bounds__(kBlock) void k_fft_rows(FftArgs a) {
  extern __shared__ char smem[];
  const int s = blockIdx.y;
  const int nx = a.nx, rows = a.rows;
  const int ls = padi(BLUE ? a.bx.P : nx);
  const LdsCplx<V> c(smem, rows * ls);
  int grp = blockIdx.x;
  if ((gridDim.x & 7) == 0) grp = (grp & 7) * (gridDim.x >> 3) + (grp >> 3);
  const int y0 = grp * rows;
  const V* in = reinterpret_cast<const V*>(a.R) + (size_t)s * a.N + (size_t)y0 * nx;
  V* out = reinterpret_cast<V*>(MODE == 0 ? a.R : a.X) + (size_t)s * a.N + (size_t)y0 * nx;
  const int tot = rows * nx;
  if (BLUE) {
    const BlueDim& d = a.bx;
    const int P = d.P, logP = d.logP;
    const double invP = 1.0 / P;
    for (int i = threadIdx.x; i < rows * P; i += kBlock) {
      const int r = i >> logP, j = i & (P - 1);
      V v = vzero<V>();
      if (j < nx) v = vmul(in[r * nx + j], from_d2<V>(MODE == 1 ? cconj(d.ch[j]) : d.ch[j]));
      c.st(r * ls + padi(j), v);
    }
    blue_conv<V, false>(c, d, MODE == 1 ? d.Bi : d.Bf, rows, ls, 1, kBlock);
    if (MODE == 2) {
      const double2 sh = a.shift[s];
      for (int k = threadIdx.x; k < P; k += kBlock) {
        const int o = padi(k);
        c.st(o, k < nx ? vmul(c.ld(o), from_d2<V>(cscale(inv_symbol(a, sh, k, 0), invP))) : vzero<V>());
      }
      blue_conv<V, false>(c, d, d.Bi, 1, ls, 1, kBlock);
    }
    for (int i = threadIdx.x; i < tot; i += kBlock) {
      const int r = i / nx, k = i - r * nx;
      const double2 chk = cscale(MODE == 0 ? d.ch[k] : cconj(d.ch[k]), invP);
      out[i] = vmul(c.ld(r * ls + padi(k)), from_d2<V>(chk));
    }
    return;
  }
  // natural order in and out: the forward rows (DIF) leave the spectrum in
  // bit-reversed order, which the inverse rows (DIT) take
  load_to_lds<V>(tot, kBlock, [&](int i) { return in[i]; }, [&](int i, V v) {
    const int r = i / nx, x = i - r * nx;
    c.st(r * ls + padi(x), v);
  });
  if (MODE == 1) {
    dit_passes<V, true, false>(c, a.Wx, nx, a.lognx, 0, rows, ls, 1, kBlock);
    __syncthreads();
  } else if (MODE == 0) {
    dif_passes<V, false, false>(c, a.Wx, nx, a.lognx, 0, rows, ls, 1, kBlock);
    __syncthreads();
  } else {
    const double2 sh = a.shift[s];
    fft_mul_ifft<V, false>(c, a.Wx, nx, a.lognx, rows, ls, 1, kBlock,
                           [&](int, int k) { return from_d2<V>(inv_symbol(a, sh, k, 0)); });
  }
  for (int i = threadIdx.x; i < tot; i += kBlock) {
    const int r = i / nx, x = i - r * nx;
    out[i] = c.ld(r * ls + padi(x));
  }
}

// Columns: forward along y, divide, inverse along y, in place on R.
// grid (nx / cols, nsys); column col, row y at col + padi(y) cols in LDS (a
// cache line of cols consecutive elements per row).  BLUE: ny through
// length-P convolutions.  CL > 0: cols = CL at compile time (the index
// splits i / cols, i % cols and the LDS strides are shifts), else a.cols.
template <typename V, bool BLUE, int CL>
__global__ __launch_bounds__(1024) void k_fft_cols(FftArgs a) {
  const int CB = blockDim.x;
  extern __shared__ char smem[];
  const int s = blockIdx.y;
  const int nx = a.nx, ny = a.ny, cols = CL > 0 ? CL : a.cols;
  const LdsCplx<V> c(smem, padi(BLUE ? a.by.P : ny) * cols);
  int grp = blockIdx.x;  // XCD-banded: neighbouring column groups share cache lines
  if ((gridDim.x & 7) == 0) grp = (grp & 7) * (gridDim.x >> 3) + (grp >> 3);
  const int x0 = grp * cols;
  V* base = reinterpret_cast<V*>(a.R) + (size_t)s * a.N + x0;
  const int tot = ny * cols;
  if (BLUE) {
    const BlueDim& d = a.by;
    const int P = d.P;
    const double invP = 1.0 / P;
    for (int i = threadIdx.x; i < P * cols; i += CB) {
      const int j = udiv(i, cols), col = i - j * cols;
      c.st(padi(j) * cols + col,
           j < ny ? vmul(base[(size_t)j * nx + col], from_d2<V>(d.ch[j])) : vzero<V>());
    }
    blue_conv<V, true>(c, d, d.Bf, cols, 1, cols, CB);
    const double2 sh = a.shift[s];
    for (int i = threadIdx.x; i < P * cols; i += CB) {
      const int k = udiv(i, cols), col = i - k * cols;
      const int o = padi(k) * cols + col;
      c.st(o, k < ny ? vmul(c.ld(o), from_d2<V>(cscale(inv_symbol(a, sh, kx_of(a, x0 + col), k), invP)))
                     : vzero<V>());
    }
    blue_conv<V, true>(c, d, d.Bi, cols, 1, cols, CB);
    for (int i = threadIdx.x; i < tot; i += CB) {
      const int k = udiv(i, cols), col = i - k * cols;
      base[(size_t)k * nx + col] =
          vmul(c.ld(padi(k) * cols + col), from_d2<V>(cscale(cconj(d.ch[k]), invP)));
    }
    return;
  }
  // forward (DIF) leaves row y of the tile at frequency ky = bitrev(y); the
  // inverse (DIT) takes that order back to natural
  load_to_lds<V>(tot, CB, [&](int i) {
    const int y = udiv(i, cols), col = i - y * cols;
    return base[(size_t)y * nx + col];
  }, [&](int i, V v) {
    const int y = udiv(i, cols), col = i - y * cols;
    c.st(padi(y) * cols + col, v);
  });
  const double2 sh = a.shift[s];
  dif_passes<V, false, true>(c, a.Wy, ny, a.logny, 0, cols, 1, cols, CB);
  __syncthreads();
  // the divide in a pass of its own (in the last forward pass it would hold
  // the group's registers through the symbol evaluation).  When the block
  // size is a multiple of cols every trip of a thread is on the same column:
  // its x part is summed once.
  const bool same_col = (CB % cols) == 0;
  const double2 lx = sym_x(a, kx_of(a, x0 + threadIdx.x % cols));
  for (int i = threadIdx.x; i < tot; i += CB) {
    const int y = udiv(i, cols), col = i - y * cols;
    const int o = padi(y) * cols + col;
    const int kx = kx_of(a, x0 + col);
    const double2 f = inv_den(a, sh, cadd(same_col ? lx : sym_x(a, kx), sym_rest(a, kx, bitrev(y, a.logny))));
    c.st(o, vmul(c.ld(o), from_d2<V>(f)));
  }
  dit_passes<V, true, true>(c, a.Wy, ny, a.logny, 0, cols, 1, cols, CB);
  __syncthreads();
  for (int i = threadIdx.x; i < tot; i += CB) {
    const int y = udiv(i, cols), col = i - y * cols;
    base[(size_t)y * nx + col] = c.ld(padi(y) * cols + col);
  }
}

}  // namespace

hipError_t launch_fft_solve(bool f32, const FftArgs& a, int nsys, hipStream_t st) {
  auto lbytes = [&](int n) { return f32 ? LdsCplx<float2>::bytes(n) : LdsCplx<double2>::bytes(n); };
  const bool bx = a.bx.P > 0, by = a.by.P > 0;
  // padded line lengths (padi of the line)
  const int lx = fft_pad_line(bx ? a.bx.P : a.nx), ly = fft_pad_line(by ? a.by.P : a.ny);
#define AAO_ROWS(V, MODE, grid, lds)                                                          \
  do {                                                                                         \
    if (bx) hipLaunchKernelGGL((k_fft_rows<V, MODE, true>), grid, dim3(kBlock), lds, st, a);   \
    else hipLaunchKernelGGL((k_fft_rows<V, MODE, false>), grid, dim3(kBlock), lds, st, a);     \
  } while (0)
#define AAO_COLS1(V, BL, grid, lds)                                                                  \
  do {                                                                                               \
    switch (a.cols) {                                                                                \
      case 2: hipLaunchKernelGGL((k_fft_cols<V, BL, 2>), grid, dim3(cthreads), lds, st, a); break;   \
      case 4: hipLaunchKernelGGL((k_fft_cols<V, BL, 4>), grid, dim3(cthreads), lds, st, a); break;   \
      case 8: hipLaunchKernelGGL((k_fft_cols<V, BL, 8>), grid, dim3(cthreads), lds, st, a); break;   \
      case 16: hipLaunchKernelGGL((k_fft_cols<V, BL, 16>), grid, dim3(cthreads), lds, st, a); break; \
      default: hipLaunchKernelGGL((k_fft_cols<V, BL, 0>), grid, dim3(cthreads), lds, st, a);         \
    }                                                                                                \
  } while (0)
#define AAO_COLS(V, grid, lds)                 \
  do {                                         \
    if (by) AAO_COLS1(V, true, grid, lds);     \
    else AAO_COLS1(V, false, grid, lds);       \
  } while (0)
  if (a.ny == 1) {
    dim3 grid(1, nsys);
    const size_t lds = lbytes(lx);
    if (f32) AAO_ROWS(float2, 2, grid, lds);
    else AAO_ROWS(double2, 2, grid, lds);
    return hipGetLastError();
  }
  if (a.rows < 1 || a.cols < 1 || a.ny % a.rows != 0 || a.nx % a.cols != 0) return hipErrorInvalidValue;
  dim3 grow(a.ny / a.rows, nsys), gcol(a.nx / a.cols, nsys);
  const size_t lrow = lbytes(a.rows * lx), lcol = lbytes(a.cols * ly);
  int cthreads = 64;  // one thread per group of eight tile elements, a multiple of 64
  while (cthreads < 1024 && cthreads * 8 < a.cols * (by ? a.by.P : a.ny)) cthreads *= 2;
  if (f32) {
    AAO_ROWS(float2, 0, grow, lrow);
    AAO_COLS(float2, gcol, lcol);
    AAO_ROWS(float2, 1, grow, lrow);
  } else {
    AAO_ROWS(double2, 0, grow, lrow);
    AAO_COLS(double2, gcol, lcol);
    AAO_ROWS(double2, 1, grow, lrow);
  }
#undef AAO_ROWS
#undef AAO_COLS
#undef AAO_COLS1
  return hipGetLastError();
}

}  // namespace aao
