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
  const double inv = 1.0 / (b.x * b.x + b.y * b.y);  // one division per quotient
  return mk((a.x * b.x + a.y * b.y) * inv, (a.y * b.x - a.x * b.y) * inv);
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

// Lane permutations inside each row of 16 lanes (DPP), on a double split into
// its two 32-bit halves.  CTRL: 0xB1 swaps neighbours, 0x4E swaps pairs,
// 0x141 mirrors each half-row, 0x140 mirrors the row.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_f64(double x, int lane) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), lane),
                          __builtin_amdgcn_readlane(__double2loint(x), lane));
}

// Sum over the 64 lanes of a wavefront (all lanes active).  The four in-row
// steps add each pair in both orders, so all 16 lanes of a row hold the same
// bits; the four row sums are then added in a fixed order.  Wave-uniform.
__device__ __forceinline__ double wave_sum(double x) {
  x += dpp_f64<0xB1>(x);
  x += dpp_f64<0x4E>(x);
  x += dpp_f64<0x141>(x);
  x += dpp_f64<0x140>(x);
  return (lane_f64(x, 0) + lane_f64(x, 16)) + (lane_f64(x, 32) + lane_f64(x, 48));
}

__device__ __forceinline__ double wave_max(double x) {
  x = fmax(x, dpp_f64<0xB1>(x));
  x = fmax(x, dpp_f64<0x4E>(x));
  x = fmax(x, dpp_f64<0x141>(x));
  x = fmax(x, dpp_f64<0x140>(x));
  return fmax(fmax(lane_f64(x, 0), lane_f64(x, 16)), fmax(lane_f64(x, 32), lane_f64(x, 48)));
}

// Sum of K values over the 256-thread block (4 wavefronts); every thread
// receives the result, and every workgroup doing the same reduction gets the
// same bits.  sh holds 4 * K doubles; called by all threads.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* sh) {
#pragma unroll
  for (int i = 0; i < K; ++i) v[i] = wave_sum(v[i]);
  const int wid = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int i = 0; i < K; ++i) sh[wid * K + i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < K; ++i) v[i] = (sh[i] + sh[K + i]) + (sh[2 * K + i] + sh[3 * K + i]);
}

// Same sums, delivered to wavefront 0 only (lane q of wavefront 0 adds the
// four wavefront sums of quantity q, then every lane of wavefront 0 reads all
// K totals): fewer registers than every thread reading every partial.
template <int K>
__device__ __forceinline__ void block_sum_wave0(double (&v)[K], double* sh) {
  static_assert(K <= 64, "one lane per quantity");
#pragma unroll
  for (int i = 0; i < K; ++i) v[i] = wave_sum(v[i]);
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < K; ++i) sh[wid * K + i] = v[i];
  }
  __syncthreads();
  if (wid == 0) {
    const int q = lane < K ? lane : 0;
    const double tq = (sh[q] + sh[K + q]) + (sh[2 * K + q] + sh[3 * K + q]);
#pragma unroll
    for (int i = 0; i < K; ++i) v[i] = lane_f64(tq, i);
  }
}

__device__ __forceinline__ double block_max(double v, double* sh) {
  v = wave_max(v);
  const int wid = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[wid] = v;
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
