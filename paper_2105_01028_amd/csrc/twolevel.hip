// Two-level angular grid (Sec. 2.1: the source function is computed on a
// coarser set of directions, from the mean intensity over the fine bins of
// each coarse bin).  In photon numbers, with r^2 fine children per coarse bin:
//   M[J][v] = sum over children i of J of X[i][v]         (coarse_sum_kernel)
//   T = b (P_c M)            (the resident collide kernel on the coarse field)
//   Y[i][v] = a_v X[i][v] + T[parent(i)][v] / r^2          (apply_kernel)
// Both kernels are bound by HBM: each reads the fine field once, with lanes
// running along the voxels of one direction.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace trinity {

namespace {

constexpr int kTwoThreads = 256;

// Sum of a double over the workgroup, written by thread 0 to *out.
__device__ double tl_block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kTwoThreads / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

// Workgroup (voxel block bx, coarse group by): coarse bins J = by, by + gy, ...
// of the block's voxels; the budget partials cover the fine rows of those bins.
__global__ __launch_bounds__(kTwoThreads) void coarse_sum_kernel(TwoLevelArgs A) {
  __shared__ double red[kTwoThreads / 64];
  const long long v = (long long)blockIdx.x * kTwoThreads + threadIdx.x;
  double colsum = 0.0;
  float av = 0.f, bv = 0.f;
  if (v < A.V) {
    av = A.a[v];
    bv = A.b[v];
    for (int J = blockIdx.y; J < A.nc; J += gridDim.y) {
      const int* kids = A.children + size_t(J) * A.nkids;
      float s = 0.0f;
      for (int k = 0; k < A.nkids; ++k) s += A.X[size_t(kids[k]) * A.Vp + v];
      A.M[size_t(J) * A.Vp + v] = s;
      colsum += double(s);
    }
  }
  const double ab = tl_block_sum((1.0 - double(av) - double(bv)) * colsum, red);
  const double tt = tl_block_sum(colsum, red);
  const long long nwg = (long long)gridDim.x * gridDim.y;
  const long long wg = (long long)blockIdx.y * gridDim.x + blockIdx.x;
  if (threadIdx.x == 0) {
    A.part[wg] = ab;
    A.part[nwg + wg] = tt;
  }
}

__global__ __launch_bounds__(kTwoThreads) void apply_kernel(TwoLevelArgs A) {
  const long long v = (long long)blockIdx.x * kTwoThreads + threadIdx.x;
  if (v >= A.V) return;
  const float av = A.a[v];
  for (int i = blockIdx.y; i < A.ndir; i += gridDim.y) {
    const size_t k = size_t(i) * A.Vp + v;
    A.Y[k] = fmaf(av, A.X[k], A.T[size_t(A.parent[i]) * A.Vp + v] * A.share);
  }
}

}  // namespace

int coarse_sum_groups(const TwoLevelArgs& a) {
  return a.nc < 16 ? a.nc : 16;
}

hipError_t launch_coarse_sum(const TwoLevelArgs& a, hipStream_t s) {
  dim3 grid(unsigned((a.V + kTwoThreads - 1) / kTwoThreads), unsigned(coarse_sum_groups(a)));
  hipLaunchKernelGGL(coarse_sum_kernel, grid, dim3(kTwoThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_apply(const TwoLevelArgs& a, hipStream_t s) {
  const int gy = a.ndir < 64 ? a.ndir : 64;
  dim3 grid(unsigned((a.V + kTwoThreads - 1) / kTwoThreads), unsigned(gy));
  hipLaunchKernelGGL(apply_kernel, grid, dim3(kTwoThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace trinity
