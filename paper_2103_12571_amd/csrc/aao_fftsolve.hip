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

// Rows: MODE 0 forward (in place), MODE 1 inverse (R -> X), MODE 2 forward,
// divide and inverse (1D, R -> X).  grid (ny / rows, nsys).
template <typename V, int MODE>
__global__ __launch_bounds__(kBlock) void k_fft_rows(FftArgs a) {
  extern __shared__ char smem[];
  const int s = blockIdx.y;
  const int nx = a.nx, rows = a.rows;
  const LdsCplx<V> c(smem, rows * nx);
  int grp = blockIdx.x;
  if ((gridDim.x & 7) == 0) grp = (grp & 7) * (gridDim.x >> 3) + (grp >> 3);
  const int y0 = grp * rows;
  const V* in = reinterpret_cast<const V*>(a.R) + (size_t)s * a.N + (size_t)y0 * nx;
  V* out = reinterpret_cast<V*>(MODE == 0 ? a.R : a.X) + (size_t)s * a.N + (size_t)y0 * nx;
  const int tot = rows * nx;
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
// grid (nx / cols, nsys); LDS c[y][col].
template <typename V>
__global__ __launch_bounds__(kBlock) void k_fft_cols(FftArgs a) {
  extern __shared__ char smem[];
  const int s = blockIdx.y;
  const int nx = a.nx, ny = a.ny, cols = a.cols;
  const LdsCplx<V> c(smem, ny * cols);
  int grp = blockIdx.x;  // XCD-banded: neighbouring column groups share cache lines
  if ((gridDim.x & 7) == 0) grp = (grp & 7) * (gridDim.x >> 3) + (grp >> 3);
  const int x0 = grp * cols;
  V* base = reinterpret_cast<V*>(a.R) + (size_t)s * a.N + x0;
  const int tot = ny * cols;
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
  if (a.ny == 1) {
    dim3 grid(1, nsys);
    const size_t lds = lbytes(a.nx);
    if (f32) hipLaunchKernelGGL((k_fft_rows<float2, 2>), grid, dim3(kBlock), lds, st, a);
    else hipLaunchKernelGGL((k_fft_rows<double2, 2>), grid, dim3(kBlock), lds, st, a);
    return hipGetLastError();
  }
  dim3 grow(a.ny / a.rows, nsys), gcol(a.nx / a.cols, nsys);
  const size_t lrow = lbytes(a.rows * a.nx), lcol = lbytes(a.cols * a.ny);
  if (f32) {
    hipLaunchKernelGGL((k_fft_rows<float2, 0>), grow, dim3(kBlock), lrow, st, a);
    hipLaunchKernelGGL((k_fft_cols<float2>), gcol, dim3(kBlock), lcol, st, a);
    hipLaunchKernelGGL((k_fft_rows<float2, 1>), grow, dim3(kBlock), lrow, st, a);
  } else {
    hipLaunchKernelGGL((k_fft_rows<double2, 0>), grow, dim3(kBlock), lrow, st, a);
    hipLaunchKernelGGL((k_fft_cols<double2>), gcol, dim3(kBlock), lcol, st, a);
    hipLaunchKernelGGL((k_fft_rows<double2, 1>), grow, dim3(kBlock), lrow, st, a);
  }
  return hipGetLastError();
}

}  // namespace aao
