// Spatial-FFT direct solve of the shifted systems (I - c_s A) x_s = b_s (row
// a3, variant for periodic constant-coefficient A).
//
// A periodic stencil is diagonalised by the DFT: for the mode e^{2 pi i k.n/N}
// it acts as lambda(k) = sum_t c_t e^{2 pi i (kx dx_t / nx + ky dy_t / ny)}, so
// x = F^{-1}[ F b / (1 - c_s lambda(k)) ] exactly.  Transforms run in LDS with
// radix-2 butterflies: decimation in time (bit-reversed input, natural output)
// forward, decimation in frequency (natural input, bit-reversed output) for the
// inverse, so no reordering pass is needed.  1D: one workgroup per system does
// forward, divide and inverse.  2D: rows forward (in place), then columns
// forward + divide + inverse (in place), then rows inverse into x.
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

// Element (b, i) of a batch of transforms lives at c[b * sb + i * se] (an LDS
// complex array).  The table W holds e^{+2 pi i k / n}, k < n.
template <typename V, bool INV, bool FASTB>
__device__ __forceinline__ void fft_dit(const LdsCplx<V>& c, const double2* W, int n, int logn, int nb, int sb,
                                        int se) {
  using T = typename scal<V>::type;
  const int half_n = n >> 1;
  for (int s = 0; s < logn; ++s) {
    const int half = 1 << s;
    const int tstride = n >> (s + 1);
    __syncthreads();
    for (int idx = threadIdx.x; idx < nb * half_n; idx += kBlock) {
      const int b = FASTB ? idx % nb : idx / half_n;
      const int k = FASTB ? idx / nb : idx % half_n;
      const int pos = k & (half - 1);
      const int i0 = ((k >> s) << (s + 1)) + pos;
      const double2 wd = W[pos * tstride];
      V w;
      w.x = (T)wd.x;
      w.y = INV ? (T)wd.y : (T)-wd.y;
      const int o0 = b * sb + i0 * se, o1 = o0 + half * se;
      const V a = c.ld(o0);
      const V t = vmul(w, c.ld(o1));
      c.st(o0, vadd(a, t));
      c.st(o1, vsub(a, t));
    }
  }
  __syncthreads();
}

template <typename V, bool INV, bool FASTB>
__device__ __forceinline__ void fft_dif(const LdsCplx<V>& c, const double2* W, int n, int logn, int nb, int sb,
                                        int se) {
  using T = typename scal<V>::type;
  const int half_n = n >> 1;
  for (int s = logn - 1; s >= 0; --s) {
    const int half = 1 << s;
    const int tstride = n >> (s + 1);
    __syncthreads();
    for (int idx = threadIdx.x; idx < nb * half_n; idx += kBlock) {
      const int b = FASTB ? idx % nb : idx / half_n;
      const int k = FASTB ? idx / nb : idx % half_n;
      const int pos = k & (half - 1);
      const int i0 = ((k >> s) << (s + 1)) + pos;
      const double2 wd = W[pos * tstride];
      V w;
      w.x = (T)wd.x;
      w.y = INV ? (T)wd.y : (T)-wd.y;
      const int o0 = b * sb + i0 * se, o1 = o0 + half * se;
      const V a = c.ld(o0);
      const V d = c.ld(o1);
      c.st(o0, vadd(a, d));
      c.st(o1, vmul(vsub(a, d), w));
    }
  }
  __syncthreads();
}

// 1 / ((1 - c lambda(kx, ky)) * nx * ny): the inverse transforms are unnormalised
__device__ __forceinline__ double2 inv_symbol(const FftArgs& a, double2 c, int kx, int ky) {
  double2 lam = mk(0, 0);
  for (int t = 0; t < a.taps.n; ++t) {
    const int ix = ((kx * a.taps.dx[t]) % a.nx + a.nx) % a.nx;
    const int iy = ((ky * a.taps.dy[t]) % a.ny + a.ny) % a.ny;
    const double2 e = cmul(a.Wx[ix], a.Wy[iy]);
    lam.x += a.taps.c[t] * e.x;
    lam.y += a.taps.c[t] * e.y;
  }
  const double2 den = mk((1.0 - (c.x * lam.x - c.y * lam.y)) * a.norm, (-(c.x * lam.y + c.y * lam.x)) * a.norm);
  return cdiv(mk(1, 0), den);
}

// Bluestein convolution of nb sequences of length P held in c (element (b, i)
// at b * sb + i * se) at bit-reversed positions: forward radix-2 transform,
// multiply by the filter's transform F, inverse radix-2 transform.  Leaves P
// times the cyclic convolution, again at bit-reversed positions.
template <typename V, bool FASTB>
__device__ __forceinline__ void blue_conv(const LdsCplx<V>& c, const BlueDim& d, const double2* F, int nb, int sb,
                                          int se) {
  fft_dit<V, false, FASTB>(c, d.W, d.P, d.logP, nb, sb, se);
  for (int idx = threadIdx.x; idx < nb * d.P; idx += kBlock) {
    const int b = FASTB ? idx % nb : idx >> d.logP;
    const int k = FASTB ? idx / nb : idx & (d.P - 1);
    const int o = b * sb + k * se;
    c.st(o, vmul(c.ld(o), from_d2<V>(F[k])));
  }
  fft_dif<V, true, FASTB>(c, d.W, d.P, d.logP, nb, sb, se);
}

__device__ __forceinline__ double2 cscale(double2 v, double s) { return mk(v.x * s, v.y * s); }
__device__ __forceinline__ double2 cconj(double2 v) { return mk(v.x, -v.y); }

// Rows: MODE 0 forward (in place), MODE 1 inverse (R -> X), MODE 2 forward,
// divide and inverse (1D, R -> X).  grid (ny / rows, nsys).  BLUE: nx is
// transformed through length-P convolutions (LDS rows of P).
template <typename V, int MODE, bool BLUE>
__global__ __launch_bounds__(kBlock) void k_fft_rows(FftArgs a) {
  extern __shared__ char smem[];
  const int s = blockIdx.y;
  const int nx = a.nx, rows = a.rows;
  const LdsCplx<V> c(smem, rows * (BLUE ? a.bx.P : nx));
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
      c.st(r * P + dev::bitrev(j, logP), v);
    }
    blue_conv<V, false>(c, d, MODE == 1 ? d.Bi : d.Bf, rows, P, 1);
    if (MODE == 2) {
      const double2 sh = a.shift[s];
      for (int k = threadIdx.x; k < P; k += kBlock) {
        const int o = dev::bitrev(k, logP);
        c.st(o, k < nx ? vmul(c.ld(o), from_d2<V>(cscale(inv_symbol(a, sh, k, 0), invP))) : vzero<V>());
      }
      blue_conv<V, false>(c, d, d.Bi, 1, P, 1);
    }
    for (int i = threadIdx.x; i < tot; i += kBlock) {
      const int r = i / nx, k = i - r * nx;
      const double2 chk = cscale(MODE == 0 ? d.ch[k] : cconj(d.ch[k]), invP);
      out[i] = vmul(c.ld(r * P + dev::bitrev(k, logP)), from_d2<V>(chk));
    }
    return;
  }
  for (int i = threadIdx.x; i < tot; i += kBlock) {
    const int r = i / nx, x = i - r * nx;
    const int dst = (MODE == 1) ? i : r * nx + dev::bitrev(x, a.lognx);
    c.st(dst, in[i]);
  }
  if (MODE == 1) {
    fft_dif<V, true, false>(c, a.Wx, nx, a.lognx, rows, nx, 1);
  } else {
    fft_dit<V, false, false>(c, a.Wx, nx, a.lognx, rows, nx, 1);
  }
  if (MODE == 2) {
    const double2 sh = a.shift[s];
    for (int i = threadIdx.x; i < nx; i += kBlock) {
      const double2 f = inv_symbol(a, sh, i, 0);
      const V fv = from_d2<V>(f);
      c.st(i, vmul(c.ld(i), fv));
    }
    fft_dif<V, true, false>(c, a.Wx, nx, a.lognx, 1, nx, 1);
  }
  for (int i = threadIdx.x; i < tot; i += kBlock) {
    const int r = i / nx, x = i - r * nx;
    const int src = (MODE == 0) ? i : r * nx + dev::bitrev(x, a.lognx);
    out[i] = c.ld(src);
  }
}

// Columns: forward along y, divide, inverse along y, in place on R.
// grid (nx / cols, nsys); LDS c[y][col].  BLUE: ny through length-P
// convolutions (LDS c[P][col]).
template <typename V, bool BLUE>
__global__ __launch_bounds__(kBlock) void k_fft_cols(FftArgs a) {
  extern __shared__ char smem[];
  const int s = blockIdx.y;
  const int nx = a.nx, ny = a.ny, cols = a.cols;
  const LdsCplx<V> c(smem, (BLUE ? a.by.P : ny) * cols);
  int grp = blockIdx.x;  // XCD-banded: neighbouring column groups share cache lines
  if ((gridDim.x & 7) == 0) grp = (grp & 7) * (gridDim.x >> 3) + (grp >> 3);
  const int x0 = grp * cols;
  V* base = reinterpret_cast<V*>(a.R) + (size_t)s * a.N + x0;
  const int tot = ny * cols;
  if (BLUE) {
    const BlueDim& d = a.by;
    const int P = d.P, logP = d.logP;
    const double invP = 1.0 / P;
    for (int i = threadIdx.x; i < P * cols; i += kBlock) {
      const int j = i / cols, col = i - j * cols;
      c.st(dev::bitrev(j, logP) * cols + col,
           j < ny ? vmul(base[(size_t)j * nx + col], from_d2<V>(d.ch[j])) : vzero<V>());
    }
    blue_conv<V, true>(c, d, d.Bf, cols, 1, cols);
    const double2 sh = a.shift[s];
    for (int i = threadIdx.x; i < P * cols; i += kBlock) {
      const int k = i / cols, col = i - k * cols;
      const int o = dev::bitrev(k, logP) * cols + col;
      c.st(o, k < ny ? vmul(c.ld(o), from_d2<V>(cscale(inv_symbol(a, sh, x0 + col, k), invP))) : vzero<V>());
    }
    blue_conv<V, true>(c, d, d.Bi, cols, 1, cols);
    for (int i = threadIdx.x; i < tot; i += kBlock) {
      const int k = i / cols, col = i - k * cols;
      base[(size_t)k * nx + col] =
          vmul(c.ld(dev::bitrev(k, logP) * cols + col), from_d2<V>(cscale(cconj(d.ch[k]), invP)));
    }
    return;
  }
  for (int i = threadIdx.x; i < tot; i += kBlock) {
    const int y = i / cols, col = i - y * cols;
    c.st(dev::bitrev(y, a.logny) * cols + col, base[(size_t)y * nx + col]);
  }
  fft_dit<V, false, true>(c, a.Wy, ny, a.logny, cols, 1, cols);
  const double2 sh = a.shift[s];
  for (int i = threadIdx.x; i < tot; i += kBlock) {
    const int y = i / cols, col = i - y * cols;
    const V fv = from_d2<V>(inv_symbol(a, sh, x0 + col, y));
    c.st(i, vmul(c.ld(i), fv));
  }
  fft_dif<V, true, true>(c, a.Wy, ny, a.logny, cols, 1, cols);
  for (int i = threadIdx.x; i < tot; i += kBlock) {
    const int y = i / cols, col = i - y * cols;
    base[(size_t)y * nx + col] = c.ld(dev::bitrev(y, a.logny) * cols + col);
  }
}

}  // namespace

hipError_t launch_fft_solve(bool f32, const FftArgs& a, int nsys, hipStream_t st) {
  auto lbytes = [&](int n) { return f32 ? LdsCplx<float2>::bytes(n) : LdsCplx<double2>::bytes(n); };
  const bool bx = a.bx.P > 0, by = a.by.P > 0;
  const int lx = bx ? a.bx.P : a.nx, ly = by ? a.by.P : a.ny;
#define AAO_ROWS(V, MODE, grid, lds)                                                          \
  do {                                                                                         \
    if (bx) hipLaunchKernelGGL((k_fft_rows<V, MODE, true>), grid, dim3(kBlock), lds, st, a);   \
    else hipLaunchKernelGGL((k_fft_rows<V, MODE, false>), grid, dim3(kBlock), lds, st, a);     \
  } while (0)
#define AAO_COLS(V, grid, lds)                                                           \
  do {                                                                                    \
    if (by) hipLaunchKernelGGL((k_fft_cols<V, true>), grid, dim3(kBlock), lds, st, a);    \
    else hipLaunchKernelGGL((k_fft_cols<V, false>), grid, dim3(kBlock), lds, st, a);      \
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
  return hipGetLastError();
}

}  // namespace aao
