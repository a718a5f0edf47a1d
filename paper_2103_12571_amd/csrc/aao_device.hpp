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

// LDS arrays of complex128 are kept as two planes of doubles (real parts,
// then imaginary parts): 8-byte LDS accesses avoid the stalls that 16-byte
// accesses at arbitrary element offsets incur.  The imaginary plane starts
// kPlanePad doubles after the real one ends, which puts the two halves of a
// wavefront's access on different banks.
constexpr int kPlanePad = 8;

// A complex array of n elements in LDS: complex128 as planes (re, im, padded
// as above), complex64 interleaved (8-byte elements already).
template <typename V> struct LdsCplx;
template <> struct LdsCplx<double2> {
  double* re;
  double* im;
  // the pad is dropped where it would push the array past 64 KiB
  static constexpr int stride(int n) { return 2 * (n + kPlanePad) * 8 <= 65536 ? n + kPlanePad : n; }
  static constexpr size_t bytes(int n) { return 2 * (size_t)stride(n) * sizeof(double); }
  __device__ LdsCplx(void* base, int n) : re(static_cast<double*>(base)), im(static_cast<double*>(base) + stride(n)) {}
  __device__ double2 ld(int i) const { return mk(re[i], im[i]); }
  __device__ void st(int i, double2 v) const {
    re[i] = v.x;
    im[i] = v.y;
  }
};
template <> struct LdsCplx<float2> {
  float2* p;
  __device__ LdsCplx(void* base, int) : p(static_cast<float2*>(base)) {}
  static constexpr size_t bytes(int n) { return (size_t)n * sizeof(float2); }
  __device__ float2 ld(int i) const { return p[i]; }
  __device__ void st(int i, float2 v) const { p[i] = v; }
};

// K consecutive radix-2 DIT stages s .. s+K-1 on the group of 2^K rows
// i0 + t 2^s (t < 2^K; bits s .. s+K-1 of i0 clear, pos = i0 mod 2^s) of one
// column, in registers.  Stage s+q pairs rows t and t + 2^q (bit q of t
// clear) with twiddle index (pos + (t mod 2^q) 2^s) L / 2^(s+q+1).
template <int K, bool INV>
__device__ __forceinline__ void fft_group(double* re, double* im, const double* twr, const double* twi, int L,
                                          int s, int i0, int pos, int ncol, int col) {
  constexpr int R = 1 << K;
  const int span = 1 << s;
  double2 v[R];
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int o = (i0 + t * span) * ncol + col;
    v[t] = mk(re[o], im[o]);
  }
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const int half = 1 << q;
    const int tstride = L >> (s + q + 1);
#pragma unroll
    for (int t = 0; t < R; ++t) {
      if (t & half) continue;
      const int ti = (pos + (t & (half - 1)) * span) * tstride;
      const double2 w = mk(twr[ti], INV ? -twi[ti] : twi[ti]);
      const double2 x0 = v[t];
      const double2 x1 = cmul(w, v[t + half]);
      v[t] = mk(x0.x + x1.x, x0.y + x1.y);
      v[t + half] = mk(x0.x - x1.x, x0.y - x1.y);
    }
  }
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int o = (i0 + t * span) * ncol + col;
    re[o] = v[t].x;
    im[o] = v[t].y;
  }
}

// In-place radix-2 DIT FFT over the row index of the complex array c[L][ncol]
// held as planes (re, im): bit-reversed input order, natural output order.
// (twr, twi) = e^{-2 pi i k / L}, k < L/2; INV uses the conjugates.  The
// stages are taken three at a time in registers (groups of eight rows, one
// barrier per three stages); every element sees the butterflies of the
// stage-by-stage form in the same order, so the result is the same bit for bit.
template <bool INV>
__device__ __forceinline__ void lds_fft(double* re, double* im, const double* twr, const double* twi, int L,
                                        int logL, int ncol) {
  for (int s = 0; s < logL; s += 3) {
    const int k = min(3, logL - s);
    const int span = 1 << s;
    const int ngroups = (L >> k) * ncol;
    __syncthreads();
    for (int idx = threadIdx.x; idx < ngroups; idx += kBlock) {
      const int col = idx % ncol;
      const int g = idx / ncol;
      const int pos = g & (span - 1);
      const int i0 = ((g >> s) << (s + k)) + pos;
      if (k == 3) fft_group<3, INV>(re, im, twr, twi, L, s, i0, pos, ncol, col);
      else if (k == 2) fft_group<2, INV>(re, im, twr, twi, L, s, i0, pos, ncol, col);
      else fft_group<1, INV>(re, im, twr, twi, L, s, i0, pos, ncol, col);
    }
  }
  __syncthreads();
}

// Per-chunk partial sums of the batched BiCGStab ([quantity][system][chunk],
// chunk < wps_stride).  Every workgroup reduces them in the same fixed order,
// so the scalars are bitwise identical across workgroups and no grid-wide
// synchronisation is needed.
__device__ __forceinline__ double* qpart(const KrylovArgs& a, int q, int s) {
  return a.part + ((size_t)q * a.num_sys + s) * a.wps_stride;
}

// Sum quantity qs[i] over the nw[i] chunks that wrote it (fixed order).
template <int K>
__device__ __forceinline__ void reduce_parts(const KrylovArgs& a, const int (&qs)[K], const int (&nw)[K], int s,
                                             double (&v)[K], double* sh) {
#pragma unroll
  for (int i = 0; i < K; ++i) v[i] = 0.0;
  for (int c = threadIdx.x; c < a.wps_stride; c += kBlock) {
#pragma unroll
    for (int i = 0; i < K; ++i)
      if (c < nw[i]) v[i] += qpart(a, qs[i], s)[c];
  }
  block_sum<K>(v, sh);
}

// This workgroup's sums of quantities qs, as chunk `chunk` of system s.
template <int K>
__device__ __forceinline__ void write_parts(const KrylovArgs& a, const int (&qs)[K], int s, int chunk,
                                            double (&v)[K], double* sh) {
  block_sum<K>(v, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < K; ++i) qpart(a, qs[i], s)[chunk] = v[i];
  }
}

}  // namespace dev
}  // namespace aao
