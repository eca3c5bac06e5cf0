// HIP kernels (gfx950) of the TRINITY time step: injection, the scattering
// contraction on MFMA, the long-characteristic transport sweep, Fresnel
// redistribution and the per-step tallies.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace trinity {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int kThreads = 256;

// Sum of a double over the 64 lanes of a wavefront (all lanes get the total).
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the workgroup of `count` doubles per thread, written by thread 0 to
// out[q * stride] (q = 0..count-1).  Fixed order: deterministic.
template <int COUNT>
__device__ inline void block_sums(const double (&vals)[COUNT], double* out, long long stride) {
  __shared__ double red[COUNT][kThreads / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < COUNT; ++q) {
    double s = wave_sum(vals[q]);
    if (lane == 0) red[q][wave] = s;
  }
  __syncthreads();
  if (threadIdx.x < COUNT) {
    double s = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) s += red[threadIdx.x][w];
    out[threadIdx.x * stride] = s;
  }
}

// Move rule of phase mode: after m steps direction d has advanced
// floor(nu m + 1/2) planes; it moves at step m iff that count goes up.
// Products and sums are rounded separately (no fused multiply-add) so that
// every caller takes the same decision.
__device__ inline float phase_move(double nu, int m) {
  double lo = floor(__dadd_rn(__dmul_rn(nu, double(m)), 0.5));
  double hi = floor(__dadd_rn(__dmul_rn(nu, double(m + 1)), 0.5));
  return float(hi - lo);
}

__device__ inline int pick(int axis, int x, int y, int z) {
  return axis == 0 ? x : (axis == 1 ? y : z);
}

// bf16 round-to-nearest-even of a finite float, as raw bits.
__device__ inline unsigned short bf16_bits(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline float bf16_to_float(unsigned short h) { return __uint_as_float(unsigned(h) << 16); }

}  // namespace

// ---------------------------------------------------------------------------
// Injection: the pulse's photons of step m spread over (source direction,
// source voxel) pairs (Sec. 3.1).  One wavefront.
__global__ void inject_kernel(InjectArgs A) {
  const int m = *A.step_ctr;
  const double q = m < A.cap ? A.q[m] : 0.0;
  const float share = float(q / double(A.npairs));
  for (int i = threadIdx.x; i < A.npairs; i += blockDim.x) {
    const int d = A.pairs[2 * i], v = A.pairs[2 * i + 1];
    A.X[size_t(d) * A.Vp + v] += share;
  }
  if (threadIdx.x == 0 && m < A.cap) A.budget[size_t(m) * 9 + 0] = double(share) * A.npairs;
}

// ---------------------------------------------------------------------------
// Collision (Eq. 10 with the explicit source of Eq. 2/12):
//   Y[:, v] = a_v X[:, v] + b_v (P X)[:, v]
// A GEMM with M = K = NP (directions) and N = voxels, on v_mfma_f32_32x32x2f32.
// Workgroup tile: MT rows (directions) x 128 columns (voxels), four wavefronts
// of 32 columns each, every wavefront holding all MT rows in accumulators.
// P is staged through LDS in chunks of KC directions as [k][row], read from
// its transpose PT (A.P holds P^T, row k = column k of P, contiguous in row);
// X goes straight from HBM into the B operand.
// The epilogue applies a, b per voxel and sums the FP64 budget partials:
// absorbed = sum_v (1 - a_v - b_v) sum_d X[d][v], total = sum X.
template <int MT>
__global__ __launch_bounds__(kThreads, 2) void collide_f32_kernel(CollideArgs A) {
  constexpr int KC = 32;
  constexpr int NQ = MT / 32;
  __shared__ float Ps[KC * MT];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int hl = lane >> 5, cl = lane & 31;
  const long long col = (long long)blockIdx.x * 128 + wave * 32 + cl;
  const int row0 = blockIdx.y * MT;
  floatx16 acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[q][r] = 0.0f;

  const float* xcol = A.X + col;
  for (int k0 = 0; k0 < A.NP; k0 += KC) {
    __syncthreads();
    for (int e = tid * 4; e < KC * MT; e += kThreads * 4) {
      const int k = e / MT, rr = e - k * MT;
      const float4 v = *reinterpret_cast<const float4*>(A.P + size_t(k0 + k) * A.NP + row0 + rr);
      *reinterpret_cast<float4*>(Ps + k * MT + rr) = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int s = 0; s < KC / 2; ++s) {
      const float bv = xcol[size_t(k0 + 2 * s + hl) * A.Vp];
      const float* prow = Ps + (2 * s + hl) * MT + cl;
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(prow[q * 32], bv, acc[q], 0, 0, 0);
    }
  }

  const float av = A.a[col], bv = A.b[col];
  double colsum = 0.0;
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = row0 + q * 32 + 8 * (r >> 2) + 4 * hl + (r & 3);
      const size_t idx = size_t(row) * A.Vp + col;
      const float x = A.X[idx];
      A.Y[idx] = av * x + bv * acc[q][r];
      colsum += double(x);
    }
  const double vals[2] = {(1.0 - double(av) - double(bv)) * colsum, colsum};
  const long long nwg = (long long)gridDim.x * gridDim.y;
  block_sums<2>(vals, A.part + (long long)blockIdx.y * gridDim.x + blockIdx.x, nwg);
}

// Same contraction with P and X each split into bf16 high and low parts,
// X = X_hi + X_lo, P = P_hi + P_lo, and (P X) ~ P_hi X_hi + P_hi X_lo + P_lo X_hi
// on v_mfma_f32_32x32x16_bf16 with fp32 accumulation (the dropped P_lo X_lo term
// is below 2^-16 of the product).  P_hi / P_lo are staged through LDS as
// [row][k] so each lane reads its 8 consecutive k in one 16-byte load.
template <int MT>
__global__ __launch_bounds__(kThreads, 2) void collide_bf16split_kernel(CollideArgs A) {
  constexpr int KC = 32;
  constexpr int NQ = MT / 32;
  constexpr int LDK = KC + 8;   // row pitch in bf16, padded against bank conflicts
  __shared__ unsigned short Sh[MT * LDK];
  __shared__ unsigned short Sl[MT * LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int hl = lane >> 5, cl = lane & 31;
  const long long col = (long long)blockIdx.x * 128 + wave * 32 + cl;
  const int row0 = blockIdx.y * MT;
  floatx16 acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[q][r] = 0.0f;

  const float* xcol = A.X + col;
  for (int k0 = 0; k0 < A.NP; k0 += KC) {
    __syncthreads();
    // stage rows row0..row0+MT-1, columns k0..k0+KC-1 of P_hi and P_lo (8 bf16 per load)
    for (int e = tid; e < MT * (KC / 8); e += kThreads) {
      const int rr = e / (KC / 8), kk = (e - rr * (KC / 8)) * 8;
      const size_t g = size_t(row0 + rr) * A.NP + k0 + kk;
      *reinterpret_cast<uint4*>(Sh + rr * LDK + kk) = *reinterpret_cast<const uint4*>(A.Phi + g);
      *reinterpret_cast<uint4*>(Sl + rr * LDK + kk) = *reinterpret_cast<const uint4*>(A.Plo + g);
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < KC / 16; ++s) {
      bf16x8 xh, xl;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float x = xcol[size_t(k0 + 16 * s + 8 * hl + j) * A.Vp];
        const unsigned short h = bf16_bits(x);
        const unsigned short l = bf16_bits(x - bf16_to_float(h));
        xh[j] = __builtin_bit_cast(__bf16, h);
        xl[j] = __builtin_bit_cast(__bf16, l);
      }
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int off = (q * 32 + cl) * LDK + 16 * s + 8 * hl;
        const bf16x8 ph = *reinterpret_cast<const bf16x8*>(Sh + off);
        const bf16x8 pl = *reinterpret_cast<const bf16x8*>(Sl + off);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ph, xh, acc[q], 0, 0, 0);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ph, xl, acc[q], 0, 0, 0);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pl, xh, acc[q], 0, 0, 0);
      }
    }
  }

  const float av = A.a[col], bv = A.b[col];
  double colsum = 0.0;
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = row0 + q * 32 + 8 * (r >> 2) + 4 * hl + (r & 3);
      const size_t idx = size_t(row) * A.Vp + col;
      const float x = A.X[idx];
      A.Y[idx] = av * x + bv * acc[q][r];
      colsum += double(x);
    }
  const double vals[2] = {(1.0 - double(av) - double(bv)) * colsum, colsum};
  const long long nwg = (long long)gridDim.x * gridDim.y;
  block_sums<2>(vals, A.part + (long long)blockIdx.y * gridDim.x + blockIdx.x, nwg);
}

// ---------------------------------------------------------------------------
// Transport sweep (Eq. 10 along long characteristics, Fig. 1).  For direction d
// the voxel at plane k (counted from d's entry face) takes the moving part of
// its upwind voxel in plane k-1, shifted by the ray's transverse step at plane k;
// upwind voxels outside the box contribute nothing (vacuum inflow) and moving
// light whose downwind voxel is outside the box leaves through the face it
// crosses (dominant axis first, then b, then c).
//   X[d][v] = (1 - f_v) Y[d][v] + f_u Y[d][u]
// Phase mode: f is 0 or 1 for the whole direction at step m.  Split mode:
// f_v = nu_d r_v.  Grid: (blocks per direction, directions); x runs along lanes
// so each wavefront reads and writes contiguous voxels.
template <bool SPLIT, bool FRESNEL>
__global__ __launch_bounds__(kThreads) void sweep_kernel(SweepArgs A) {
  const int d = blockIdx.y;
  const DevDir D = A.dirs[d];
  const int m = *A.step_ctr;
  const float fph = SPLIT ? 0.0f : phase_move(D.nu64, m);
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const int ea = pick(D.axis, nx, ny, nz), eb = pick(D.bax, nx, ny, nz),
            ec = pick(D.cax, nx, ny, nz);
  const long long sxy = (long long)nx * ny;
  const long long sa = D.axis == 0 ? 1 : (D.axis == 1 ? nx : sxy);
  const long long sb = D.bax == 0 ? 1 : (D.bax == 1 ? nx : sxy);
  const long long sc = D.cax == 0 ? 1 : (D.cax == 1 ? nx : sxy);
  const int8_t* db = A.delta + (size_t(d) * 2 + 0) * A.dstride;
  const int8_t* dc = A.delta + (size_t(d) * 2 + 1) * A.dstride;
  const float* Yd = A.Y + size_t(d) * A.Vp;
  float* Xd = A.X + size_t(d) * A.Vp;
  double esc_a = 0, esc_b0 = 0, esc_b1 = 0, esc_c0 = 0, esc_c1 = 0, dom = 0;
  const bool moving = SPLIT || fph != 0.0f;

  for (int v = blockIdx.x * kThreads + threadIdx.x; v < A.V; v += gridDim.x * kThreads) {
    const int x = v % nx, t = v / nx, y = t % ny, z = t / ny;
    const int pa = pick(D.axis, x, y, z), pb = pick(D.bax, x, y, z), pc = pick(D.cax, x, y, z);
    const int k = D.sign > 0 ? pa : ea - 1 - pa;
    const float yv = Yd[v];
    const float fv = SPLIT ? D.nu * A.r[v] : fph;
    float out = (1.0f - fv) * yv;
    if (moving && k > 0) {
      const int dbk = db[k], dck = dc[k];
      const int ub = pb - dbk, uc = pc - dck;
      if ((unsigned)ub < (unsigned)eb && (unsigned)uc < (unsigned)ec) {
        const long long u = v - D.sign * sa - dbk * sb - dck * sc;
        bool blocked = false;
        if (FRESNEL) blocked = A.iface[u] && A.nvox[u] != A.nvox[v];
        if (!blocked) {
          const float fu = SPLIT ? D.nu * A.r[u] : fph;
          out = fmaf(fu, Yd[u], out);
        }
      }
    }
    Xd[v] = out;
    dom += double(out);
    if (moving) {
      const float mv = fv * yv;
      if (k + 1 >= ea) {
        esc_a += double(mv);
      } else {
        const int dbn = db[k + 1], dcn = dc[k + 1];
        const int wb = pb + dbn, wc = pc + dcn;
        if ((unsigned)wb >= (unsigned)eb) {
          if (dbn > 0) esc_b1 += double(mv); else esc_b0 += double(mv);
        } else if ((unsigned)wc >= (unsigned)ec) {
          if (dcn > 0) esc_c1 += double(mv); else esc_c0 += double(mv);
        } else if (FRESNEL && A.iface[v]) {
          const long long w = v + D.sign * sa + dbn * sb + dcn * sc;
          if (A.nvox[w] != A.nvox[v]) {
            A.icptF[size_t(A.islot[v]) * A.ndir + d] = mv;
            dom += double(mv);
          }
        }
      }
    }
  }
  double face[6] = {0, 0, 0, 0, 0, 0};
  // map the five per-direction accumulators onto faces (uniform per block)
  const int fa = 2 * D.axis + (D.sign > 0 ? 1 : 0);
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    double s = 0;
    if (f == fa) s += esc_a;
    if (f == 2 * D.bax) s += esc_b0;
    if (f == 2 * D.bax + 1) s += esc_b1;
    if (f == 2 * D.cax) s += esc_c0;
    if (f == 2 * D.cax + 1) s += esc_c1;
    face[f] = s;
  }
  const double vals[7] = {face[0], face[1], face[2], face[3], face[4], face[5], dom};
  const long long nwg = (long long)gridDim.x * gridDim.y;
  block_sums<7>(vals, A.part + (long long)blockIdx.y * gridDim.x + blockIdx.x, nwg);
}

// Fresnel redistribution (Eq. 13-14): every target (direction, voxel) adds the
// reflected or refracted share of the light intercepted at an index jump.
__global__ void gather_kernel(GatherArgs A) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= A.ntgt) return;
  float s = 0.0f;
  for (int j = A.ptr[t]; j < A.ptr[t + 1]; ++j) {
    const float F = A.icptF[A.src[j]], w = A.w[j];
    // w >= 0: reflected share w F; w < 0: refracted share F - |w| F (one rounding)
    s += w >= 0.0f ? w * F : fmaf(w, F, F);
  }
  A.X[size_t(A.tgt_d[t]) * A.Vp + A.tgt_v[t]] += s;
}

// Per-step tallies (one workgroup, fixed summation order): budget of step m and
// the light leaving through each detector patch, then advance the step counter.
__global__ __launch_bounds__(kThreads) void reduce_kernel(ReduceArgs A) {
  __shared__ double red[kThreads];
  __shared__ double res[8];
  const int tid = threadIdx.x;
  const int m = *A.step_ctr;
  for (int q = 0; q < 8; ++q) {
    const double* src;
    long long n;
    if (q == 0) {
      src = A.cpart;               // absorbed
      n = A.cnwg;
    } else {
      src = A.spart + (long long)(q == 1 ? 6 : q - 2) * A.snwg;   // in the box, faces 0..5
      n = A.snwg;
    }
    double s = 0;
    for (long long i = tid; i < n; i += kThreads) s += src[i];
    red[tid] = s;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) res[q] = red[0];
    __syncthreads();
  }
  const bool ok = m < A.cap;
  for (int k = tid; k < A.ndet; k += kThreads) {
    double s = 0;
    const int v = A.det_vox[k];
    for (int p = A.det_first[k]; p < A.det_first[k + 1]; ++p) {
      const int d = A.det_pairs[2 * p + 1];
      const DevDir D = A.dirs[d];
      const float f = A.split ? D.nu * A.r[v] : phase_move(D.nu64, m);
      s += double(f * A.Y[size_t(d) * A.Vp + v]);
    }
    if (ok) A.det_steps[size_t(k) * A.cap + m] = s;
  }
  if (tid == 0) {
    if (ok) {
      double* b = A.budget + size_t(m) * 9;
      b[1] = res[0];
      b[2] = res[1];
      for (int f = 0; f < 6; ++f) b[3 + f] = res[2 + f];
      bool finite = true;
      for (int q = 0; q < 9; ++q) finite = finite && isfinite(b[q]);
      if (!finite) atomicOr(A.flag, 1);
    } else {
      atomicOr(A.flag, 2);
    }
    __threadfence();
    *A.step_ctr = m + 1;
  }
}

__global__ void energy_kernel(const float* X, long long Vp, int ndir, int V, float* E) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  float s = 0.0f;
  for (int d = 0; d < ndir; ++d) s += X[size_t(d) * Vp + v];
  E[v] = s;
}

// ---------------------------------------------------------------------------
// Launchers

hipError_t launch_inject(const InjectArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(inject_kernel, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}

namespace {
int collide_mt(int NP) {
  for (int mt = 256; mt >= 32; mt -= 32)
    if (NP % mt == 0) return mt;
  return 32;
}

template <template <int> class K>
struct Dummy;

template <int MT>
hipError_t launch_collide_mt(const CollideArgs& a, const Field& f, int bf16split, hipStream_t s) {
  dim3 grid(unsigned(f.Vp / 128), unsigned(f.NP / MT));
  if (bf16split)
    hipLaunchKernelGGL(collide_bf16split_kernel<MT>, grid, dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL(collide_f32_kernel<MT>, grid, dim3(kThreads), 0, s, a);
  return hipGetLastError();
}
}  // namespace

int collide_nwg(const Field& f) { return int(f.Vp / 128) * (f.NP / collide_mt(f.NP)); }

hipError_t launch_collide(const CollideArgs& a, const Field& f, int bf16split, int, hipStream_t s) {
  switch (collide_mt(f.NP)) {
    case 256: return launch_collide_mt<256>(a, f, bf16split, s);
    case 224: return launch_collide_mt<224>(a, f, bf16split, s);
    case 192: return launch_collide_mt<192>(a, f, bf16split, s);
    case 160: return launch_collide_mt<160>(a, f, bf16split, s);
    case 128: return launch_collide_mt<128>(a, f, bf16split, s);
    case 96: return launch_collide_mt<96>(a, f, bf16split, s);
    case 64: return launch_collide_mt<64>(a, f, bf16split, s);
    default: return launch_collide_mt<32>(a, f, bf16split, s);
  }
}

int sweep_blocks_per_dir(const Field& f) {
  int b = (f.V + kThreads * 16 - 1) / (kThreads * 16);
  return b < 1 ? 1 : (b > 64 ? 64 : b);
}

hipError_t launch_sweep(const SweepArgs& a, const Field& f, int split, int fresnel, int bpd,
                        hipStream_t s) {
  dim3 grid(unsigned(bpd), unsigned(f.ndir));
  if (split && fresnel)
    hipLaunchKernelGGL((sweep_kernel<true, true>), grid, dim3(kThreads), 0, s, a);
  else if (split)
    hipLaunchKernelGGL((sweep_kernel<true, false>), grid, dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL((sweep_kernel<false, false>), grid, dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gather(const GatherArgs& a, hipStream_t s) {
  if (a.ntgt == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_kernel, dim3(unsigned((a.ntgt + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_energy(const float* X, long long Vp, int ndir, int V, float* E, hipStream_t s) {
  hipLaunchKernelGGL(energy_kernel, dim3(unsigned((V + 255) / 256)), dim3(256), 0, s, X, Vp, ndir,
                     V, E);
  return hipGetLastError();
}

}  // namespace trinity
