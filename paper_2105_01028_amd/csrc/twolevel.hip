// Two-level angular grid (Sec. 2.1: the source function is computed on a
// coarser set of directions, from the mean intensity over the fine bins of
// each coarse bin).  In photon numbers, with r^2 fine children per coarse bin:
//   M[J][v] = sum over children i of J of X[i][v]         (coarse_sum_kernel)
//   T = b (P_c M)            (the resident collide kernel on the coarse field)
//   Y[i][v] = a_v X[i][v] + T[parent(i)][v] / r^2          (apply_kernel)
// With the phase advance the sweep forms Y as it reads (kernels.hip) and
// apply_kernel is not used; with the retarded history apply_hop_kernel writes
// the hop collision of every fine direction into the history instead.  The
// kernels here are bound by HBM: each reads the fine field once, with lanes
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

// Lanes hold four consecutive voxels (16-byte loads; rows start on 1 KiB
// boundaries because Vp is a multiple of 256).  The one quad that straddles V
// takes the scalar path.
__device__ __forceinline__ float4 ld4(const float* p) {
  return *reinterpret_cast<const float4*>(p);
}
__device__ __forceinline__ void st4(float* p, float4 v) {
  *reinterpret_cast<float4*>(p) = v;
}

// The children table is never written on the device: reading it through the
// constant address space lets the uniform index loads go to scalar registers
// instead of a vector load and a wait in front of every batch.
typedef const __attribute__((address_space(4))) int* const_ints;
__device__ __forceinline__ const_ints kids_of(const TwoLevelArgs& A, int J) {
  return (const_ints)(A.children + size_t(J) * A.nkids);
}

typedef const __attribute__((address_space(4))) float* const_floats;
constexpr float kLog2e = 1.44269504088896341f;

// The flux-weighted coarse sums of the retarded advance:
//   M[J][v] = sum over children i of J of (1 - a_i(v)) X[i][v] / D_i,
// a_i(v) = exp(-mu_t(v) dx / |Omega_a|_i), computed as apply_hop_kernel does.
__device__ void coarse_sum_flux(const TwoLevelArgs& A, long long v0) {
  const const_floats ic = (const_floats)A.hinvc;
  const const_floats iD = (const_floats)A.hinvD;
  const int ne = v0 + 4 <= A.V ? 4 : int(A.V - v0);
  float ml2[4] = {0.f, 0.f, 0.f, 0.f};
  for (int e = 0; e < ne; ++e) ml2[e] = A.mutdx[v0 + e] * kLog2e;
  for (int J = blockIdx.y; J < A.nc; J += gridDim.y) {
    const const_ints kids = kids_of(A, J);
    float s[4] = {0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < A.nkids; ++k) {
      const int i = kids[k];
      const size_t o = size_t(i) * A.Vp + v0;
      const float c = ic[i], w = iD[i];
      float x[4] = {0.f, 0.f, 0.f, 0.f};
      if (ne == 4) {
        const float4 x4 = ld4(A.X + o);
        x[0] = x4.x;
        x[1] = x4.y;
        x[2] = x4.z;
        x[3] = x4.w;
      } else {
        for (int e = 0; e < ne; ++e) x[e] = A.X[o + e];
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float a = __builtin_amdgcn_exp2f(-ml2[e] * c);
        s[e] = fmaf((1.0f - a) * x[e], w, s[e]);
      }
    }
    if (ne == 4)
      st4(A.M + size_t(J) * A.Vp + v0, make_float4(s[0], s[1], s[2], s[3]));
    else
      for (int e = 0; e < ne; ++e) A.M[size_t(J) * A.Vp + v0 + e] = s[e];
  }
}

// Workgroup (quad block bx, coarse group by): coarse bins J = by, by + gy, ...
// of the block's voxels; the budget partials cover the fine rows of those bins
// (the retarded advance replaces them in apply_hop_kernel).
__global__ __launch_bounds__(kTwoThreads) void coarse_sum_kernel(TwoLevelArgs A) {
  __shared__ double red[kTwoThreads / 64];
  // the field of this step's parity when it alternates between two buffers
  if (A.X2 && (*A.step_ctr & 1)) A.X = A.X2;
  const long long v0 = 4 * ((long long)blockIdx.x * kTwoThreads + threadIdx.x);
  if (A.flux) {
    if (v0 < A.V) coarse_sum_flux(A, v0);
    return;
  }
  double col[4] = {0.0, 0.0, 0.0, 0.0};
  double ab = 0.0;
  if (v0 + 4 <= A.V) {
    for (int J = blockIdx.y; J < A.nc; J += gridDim.y) {
      const const_ints kids = kids_of(A, J);
      float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll 16
      for (int k = 0; k < A.nkids; ++k) {
        const float4 x = ld4(A.X + size_t(kids[k]) * A.Vp + v0);
        s.x += x.x;
        s.y += x.y;
        s.z += x.z;
        s.w += x.w;
      }
      st4(A.M + size_t(J) * A.Vp + v0, s);
      col[0] += double(s.x);
      col[1] += double(s.y);
      col[2] += double(s.z);
      col[3] += double(s.w);
    }
  } else if (v0 < A.V) {
    for (int J = blockIdx.y; J < A.nc; J += gridDim.y) {
      const const_ints kids = kids_of(A, J);
      for (long long v = v0; v < A.V; ++v) {
        float s = 0.0f;
        for (int k = 0; k < A.nkids; ++k) s += A.X[size_t(kids[k]) * A.Vp + v];
        A.M[size_t(J) * A.Vp + v] = s;
        col[v - v0] += double(s);
      }
    }
  }
  for (int e = 0; e < 4; ++e)
    if (v0 + e < A.V) ab += (1.0 - double(A.a[v0 + e]) - double(A.b[v0 + e])) * col[e];
  ab = tl_block_sum(ab, red);
  const double tt = tl_block_sum(col[0] + col[1] + col[2] + col[3], red);
  const long long nwg = (long long)gridDim.x * gridDim.y;
  const long long wg = (long long)blockIdx.y * gridDim.x + blockIdx.x;
  if (threadIdx.x == 0) {
    A.part[wg] = ab;
    A.part[nwg + wg] = tt;
  }
}

// Workgroup (quad block bx, coarse group by): the fine rows of coarse bins
// J = by, by + gy, ...; T[J] is read once for all of J's children.
__global__ __launch_bounds__(kTwoThreads) void apply_kernel(TwoLevelArgs A) {
  const long long v0 = 4 * ((long long)blockIdx.x * kTwoThreads + threadIdx.x);
  if (v0 >= A.V) return;
  if (v0 + 4 <= A.V) {
    const float4 av = ld4(A.a + v0);
    for (int J = blockIdx.y; J < A.nc; J += gridDim.y) {
      const const_ints kids = kids_of(A, J);
      float4 t = ld4(A.T + size_t(J) * A.Vp + v0);
      t.x *= A.share;
      t.y *= A.share;
      t.z *= A.share;
      t.w *= A.share;
      // four children per batch: all loads are issued before the first store
      // (X and Y may alias as far as the compiler knows)
      int k = 0;
      for (; k + 4 <= A.nkids; k += 4) {
        size_t o[4];
        float4 x[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          o[j] = size_t(kids[k + j]) * A.Vp + v0;
          x[j] = ld4(A.X + o[j]);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
          st4(A.Y + o[j], make_float4(fmaf(av.x, x[j].x, t.x), fmaf(av.y, x[j].y, t.y),
                                      fmaf(av.z, x[j].z, t.z), fmaf(av.w, x[j].w, t.w)));
      }
      for (; k < A.nkids; ++k) {
        const size_t o = size_t(kids[k]) * A.Vp + v0;
        const float4 x = ld4(A.X + o);
        st4(A.Y + o, make_float4(fmaf(av.x, x.x, t.x), fmaf(av.y, x.y, t.y),
                                 fmaf(av.z, x.z, t.z), fmaf(av.w, x.w, t.w)));
      }
    }
  } else {
    for (int J = blockIdx.y; J < A.nc; J += gridDim.y) {
      const const_ints kids = kids_of(A, J);
      for (long long v = v0; v < A.V; ++v) {
        const float t = A.T[size_t(J) * A.Vp + v] * A.share;
        for (int k = 0; k < A.nkids; ++k) {
          const size_t o = size_t(kids[k]) * A.Vp + v;
          A.Y[o] = fmaf(A.a[v], A.X[o], t);
        }
      }
    }
  }
}

// Retarded stepping on the two-level grid (the hop collision of the retarded
// form of Eq. 10 with the source from the coarse bins): fine direction i hops
// dx/|Omega_a|_i, so
//   C[i][v] = a X[i][v] + (1 - a) T[J(i)][v] / r^2,  a = exp(-mu_t(v) dx / |Omega_a|_i),
// with T = omega (P_c M) from the coarse collide; with the flux-weighted
// source D_i T[J(i)][v] / r^2 in place of the second term (M then holds the
// weighted sums of coarse_sum_flux).  C goes to the history slot of the step.  The budget partials (absorbed (1 - a)(1 - omega) X / D_i per
// element, total X) replace those coarse_sum wrote, in the same layout.
__global__ __launch_bounds__(kTwoThreads) void apply_hop_kernel(TwoLevelArgs A) {
  __shared__ double red[kTwoThreads / 64];
  const long long v0 = 4 * ((long long)blockIdx.x * kTwoThreads + threadIdx.x);
  const int m = *A.step_ctr;
  float* __restrict__ C = A.ring + size_t(m % A.H) * size_t(A.slot);
  const const_floats ic = (const_floats)A.hinvc;
  const const_floats iD = (const_floats)A.hinvD;
  const const_floats hD = (const_floats)A.hD;
  const bool flux = A.flux != 0;
  double lost[4] = {0.0, 0.0, 0.0, 0.0}, tot[4] = {0.0, 0.0, 0.0, 0.0};
  float om[4] = {0.f, 0.f, 0.f, 0.f};
  if (v0 < A.V) {
    const int ne = v0 + 4 <= A.V ? 4 : int(A.V - v0);
    float ml2[4] = {0.f, 0.f, 0.f, 0.f};
    for (int e = 0; e < ne; ++e) {
      ml2[e] = A.mutdx[v0 + e] * kLog2e;
      om[e] = A.omega[v0 + e];
    }
    for (int J = blockIdx.y; J < A.nc; J += gridDim.y) {
      const const_ints kids = kids_of(A, J);
      float t[4] = {0.f, 0.f, 0.f, 0.f};
      for (int e = 0; e < ne; ++e) t[e] = A.T[size_t(J) * A.Vp + v0 + e] * A.share;
      float lf[4] = {0.f, 0.f, 0.f, 0.f}, tf[4] = {0.f, 0.f, 0.f, 0.f};
      for (int k = 0; k < A.nkids; ++k) {
        const int i = kids[k];
        const size_t o = size_t(i) * A.Vp + v0;
        const float c = ic[i], w = iD[i], Di = flux ? hD[i] : 0.0f;
        float x[4] = {0.f, 0.f, 0.f, 0.f};
        if (ne == 4) {
          const float4 x4 = ld4(A.X + o);
          x[0] = x4.x;
          x[1] = x4.y;
          x[2] = x4.z;
          x[3] = x4.w;
        } else {
          for (int e = 0; e < ne; ++e) x[e] = A.X[o + e];
        }
        float y[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float a = __builtin_amdgcn_exp2f(-ml2[e] * c);
          const float oma = 1.0f - a;
          y[e] = fmaf(a, x[e], (flux ? Di : oma) * t[e]);
          lf[e] = fmaf(oma * x[e], w, lf[e]);
          tf[e] += x[e];
        }
        if (ne == 4)
          st4(C + o, make_float4(y[0], y[1], y[2], y[3]));
        else
          for (int e = 0; e < ne; ++e) C[o + e] = y[e];
      }
      for (int e = 0; e < 4; ++e) {
        lost[e] += double(lf[e]);
        tot[e] += double(tf[e]);
      }
    }
  }
  double ab = 0.0, tt = 0.0;
  for (int e = 0; e < 4; ++e) {
    ab += (1.0 - double(om[e])) * lost[e];
    tt += tot[e];
  }
  ab = tl_block_sum(ab, red);
  tt = tl_block_sum(tt, red);
  const long long nwg = (long long)gridDim.x * gridDim.y;
  const long long wg = (long long)blockIdx.y * gridDim.x + blockIdx.x;
  if (threadIdx.x == 0) {
    A.part[wg] = ab;
    A.part[nwg + wg] = tt;
  }
}

}  // namespace

namespace {

unsigned quad_blocks(const TwoLevelArgs& a) {
  return unsigned((a.V + 4 * kTwoThreads - 1) / (4 * kTwoThreads));
}

unsigned coarse_sum_groups(const TwoLevelArgs& a) {
  return unsigned(a.nc < 16 ? a.nc : 16);
}

}  // namespace

long long coarse_sum_workgroups(const TwoLevelArgs& a) {
  return (long long)quad_blocks(a) * coarse_sum_groups(a);
}

hipError_t launch_coarse_sum(const TwoLevelArgs& a, hipStream_t s) {
  dim3 grid(quad_blocks(a), coarse_sum_groups(a));
  hipLaunchKernelGGL(coarse_sum_kernel, grid, dim3(kTwoThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_apply_hop(const TwoLevelArgs& a, hipStream_t s) {
  dim3 grid(quad_blocks(a), coarse_sum_groups(a));
  hipLaunchKernelGGL(apply_hop_kernel, grid, dim3(kTwoThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_apply(const TwoLevelArgs& a, hipStream_t s) {
  dim3 grid(quad_blocks(a), coarse_sum_groups(a));
  hipLaunchKernelGGL(apply_kernel, grid, dim3(kTwoThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace trinity
