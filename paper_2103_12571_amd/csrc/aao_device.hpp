// Device helpers shared by the HIP sources of libaao.so (internal).
#pragma once
#include <hip/hip_runtime.h>

#include "aao_kernels.hpp"

namespace aao {
namespace dev {

template <typename T> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float> { using type = float2; };

__device__ __forceinline__ double2 mk(double x, double y) { double2 r; r.x = x; r.y = y; return r; }
__device__ __forceinline__ float2 mkf(float x, float y) { float2 r; r.x = x; r.y = y; return r; }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return mk(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return mk(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // a * conj(b)
  return mk(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ double2 cconj(double2 a) { return mk(a.x, -a.y); }
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  double d = b.x * b.x + b.y * b.y;
  return mk((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ double2 to_d2(double2 a) { return a; }
__device__ __forceinline__ double2 to_d2(float2 a) { return mk(a.x, a.y); }
template <typename V> __device__ __forceinline__ V from_d2(double2 a);
template <> __device__ __forceinline__ double2 from_d2<double2>(double2 a) { return a; }
template <> __device__ __forceinline__ float2 from_d2<float2>(double2 a) {
  return mkf((float)a.x, (float)a.y);
}

// generic complex arithmetic for T2 in {double2, float2}
template <typename V> __device__ __forceinline__ V vadd(V a, V b) { V r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename V> __device__ __forceinline__ V vsub(V a, V b) { V r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename V> __device__ __forceinline__ V vmul(V a, V b) {
  V r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
template <typename V, typename S> __device__ __forceinline__ V vscale(V a, S s) { V r; r.x = a.x * s; r.y = a.y * s; return r; }
template <typename V> __device__ __forceinline__ V vzero() { V r; r.x = 0; r.y = 0; return r; }

__device__ __forceinline__ int wrap_index(int x, int y, int dx, int dy, const Geo& g) {
  int xx = x + dx;
  xx += (xx < 0) ? g.nx : 0;
  xx -= (xx >= g.nx) ? g.nx : 0;
  int yy = y + dy;
  yy += (yy < 0) ? g.ny : 0;
  yy -= (yy >= g.ny) ? g.ny : 0;
  return yy * g.nx + xx;
}

__device__ __forceinline__ int bitrev(int v, int logL) {
  return logL == 0 ? 0 : (int)(__brev((unsigned)v) >> (32 - logL));
}

// Sum of K values over the 256-thread block; every thread receives the result.
// The butterfly over lanes adds each pair in both orders, which is exact-equal,
// so all lanes (and every workgroup doing the same reduction) agree bitwise.
// Same for a block of NW wavefronts (sh holds NW * K doubles).
template <int K, int NW>
__device__ __forceinline__ void block_sum_w(double (&v)[K], double* sh) {
#pragma unroll
  for (int i = 0; i < K; ++i) {
    double x = v[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    v[i] = x;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < K; ++i) sh[wid * K + i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < K; ++i) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) t += sh[w * K + i];
    v[i] = t;
  }
}

template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* sh) {
#pragma unroll
  for (int i = 0; i < K; ++i) {
    double x = v[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    v[i] = x;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < K; ++i) sh[wid * K + i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < K; ++i) v[i] = (sh[i] + sh[K + i]) + (sh[2 * K + i] + sh[3 * K + i]);
}

__device__ __forceinline__ double block_max(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  return fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

// In-place radix-2 DIT FFT over the row index of c[L][ncol] (bit-reversed
// input order, natural output order).  INV selects e^{+2 pi i ...}.
template <bool INV>
__device__ __forceinline__ void lds_fft(double2* c, const double2* tw, int L, int logL, int ncol) {
  for (int s = 0; s < logL; ++s) {
    const int half = 1 << s;
    const int tstride = L >> (s + 1);
    __syncthreads();
    const int total = (L >> 1) * ncol;
    for (int idx = threadIdx.x; idx < total; idx += kBlock) {
      const int col = idx % ncol;
      const int k = idx / ncol;
      const int pos = k & (half - 1);
      const int i0 = ((k >> s) << (s + 1)) + pos;
      const int i1 = i0 + half;
      double2 w = tw[pos * tstride];
      if (INV) w.y = -w.y;
      const double2 a = c[i0 * ncol + col];
      const double2 b = cmul(w, c[i1 * ncol + col]);
      c[i0 * ncol + col] = cadd(a, b);
      c[i1 * ncol + col] = csub(a, b);
    }
  }
  __syncthreads();
}

}  // namespace dev
}  // namespace aao
