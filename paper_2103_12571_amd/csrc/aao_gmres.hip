// Gram-Schmidt kernels of the outer flexible GMRES on C u = w (right
// preconditioner C_alpha): several dot products against one vector in one
// pass, and a combination of several vectors in one pass.  Vectors are
// [B][D] FP64 with D = L M N; basis vector i starts at i * stride.  Both
// kernels stream their operands once from HBM.
#include "aao_device.hpp"
#include "aao_kernels.hpp"

namespace aao {

namespace {

using namespace dev;

// part[(b nblk + blk) K + i] = the block's share of <V_i[b], t[b]>, i < nvec
// (zero for nvec <= i < K).  Grid (nblk, B).
template <int K>
__global__ __launch_bounds__(kBlock) void k_mdot(const double* __restrict__ V, size_t stride, int nvec,
                                                const double* __restrict__ t, int64_t D,
                                                double* __restrict__ part) {
  __shared__ double sh[4 * K];
  const size_t off = (size_t)blockIdx.y * D;
  double acc[K];
#pragma unroll
  for (int i = 0; i < K; ++i) acc[i] = 0.0;
  for (int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x; x < D; x += (int64_t)gridDim.x * kBlock) {
    const double tv = t[off + x];
#pragma unroll
    for (int i = 0; i < K; ++i)
      if (i < nvec) acc[i] = fma(V[i * stride + off + x], tv, acc[i]);
  }
  block_sum_wave0<K>(acc, sh);
  if (threadIdx.x == 0) {
    double* p = part + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * K;
#pragma unroll
    for (int i = 0; i < K; ++i) p[i] = acc[i];
  }
}

// out[b] = s[b] in[b] + sum_{i < nvec} c[b][i] V_i[b] (in may be out);
// part[b nblk + blk] = the block's share of ||out[b]||^2 (if part).
// c is [B][kGmresMax].  Grid (nblk, B).
template <int K>
__global__ __launch_bounds__(kBlock) void k_maxpy(double* out, const double* in, const double* __restrict__ s,
                                                 const double* __restrict__ V, size_t stride, int nvec,
                                                 const double* __restrict__ c, int64_t D, double* part) {
  __shared__ double sh[4];
  const int b = blockIdx.y;
  const size_t off = (size_t)b * D;
  double cf[K];
#pragma unroll
  for (int i = 0; i < K; ++i) cf[i] = (i < nvec) ? c[b * kGmresMax + i] : 0.0;
  const double sb = s[b];
  double n2 = 0.0;
  for (int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x; x < D; x += (int64_t)gridDim.x * kBlock) {
    double v = sb * in[off + x];
#pragma unroll
    for (int i = 0; i < K; ++i)
      if (i < nvec) v = fma(cf[i], V[i * stride + off + x], v);
    out[off + x] = v;
    n2 = fma(v, v, n2);
  }
  if (part) {
    double r[1] = {n2};
    block_sum<1>(r, sh);
    if (threadIdx.x == 0) part[(size_t)b * gridDim.x + blockIdx.x] = r[0];
  }
}

}  // namespace

int gmres_bucket(int nvec) { return nvec <= 4 ? 4 : nvec <= 8 ? 8 : nvec <= 16 ? 16 : 32; }

hipError_t launch_mdot(const double* V, size_t stride, int nvec, const double* t, int64_t D, int B, double* part,
                       int nblk, hipStream_t st) {
  if (nvec < 1 || nvec > kGmresMax || B < 1 || nblk < 1) return hipErrorInvalidValue;
  const dim3 grid(nblk, B);
  switch (gmres_bucket(nvec)) {
    case 4: hipLaunchKernelGGL(k_mdot<4>, grid, dim3(kBlock), 0, st, V, stride, nvec, t, D, part); break;
    case 8: hipLaunchKernelGGL(k_mdot<8>, grid, dim3(kBlock), 0, st, V, stride, nvec, t, D, part); break;
    case 16: hipLaunchKernelGGL(k_mdot<16>, grid, dim3(kBlock), 0, st, V, stride, nvec, t, D, part); break;
    default: hipLaunchKernelGGL(k_mdot<32>, grid, dim3(kBlock), 0, st, V, stride, nvec, t, D, part); break;
  }
  return hipGetLastError();
}

hipError_t launch_maxpy(double* out, const double* in, const double* s, const double* V, size_t stride, int nvec,
                        const double* c, int64_t D, int B, double* part, int nblk, hipStream_t st) {
  if (nvec < 0 || nvec > kGmresMax || B < 1 || nblk < 1) return hipErrorInvalidValue;
  const dim3 grid(nblk, B);
  switch (gmres_bucket(nvec)) {
    case 4: hipLaunchKernelGGL(k_maxpy<4>, grid, dim3(kBlock), 0, st, out, in, s, V, stride, nvec, c, D, part); break;
    case 8: hipLaunchKernelGGL(k_maxpy<8>, grid, dim3(kBlock), 0, st, out, in, s, V, stride, nvec, c, D, part); break;
    case 16:
      hipLaunchKernelGGL(k_maxpy<16>, grid, dim3(kBlock), 0, st, out, in, s, V, stride, nvec, c, D, part);
      break;
    default:
      hipLaunchKernelGGL(k_maxpy<32>, grid, dim3(kBlock), 0, st, out, in, s, V, stride, nvec, c, D, part);
      break;
  }
  return hipGetLastError();
}

}  // namespace aao
