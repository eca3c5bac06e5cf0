// HIP kernels (gfx950) of the TRINITY time step: injection, the scattering
// contraction on MFMA, the long-characteristic transport sweep, Fresnel
// redistribution and the per-step tallies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "device.hpp"

namespace trinity {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int kThreads = 256;
using f32x4 = float __attribute__((ext_vector_type(4)));

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

// x as hi + lo, hi = bf16(x) and lo = bf16(x - hi), each rounded to nearest
// even (the conversion is one gfx950 instruction); hi + lo holds 16 of x's 24
// significand bits.
__device__ inline __bf16 bf16_rest(float x, __bf16 hi) {
  return static_cast<__bf16>(x - static_cast<float>(hi));
}

}  // namespace

// ---------------------------------------------------------------------------
// Injection: the pulse's photons of step m spread over (source direction,
// source voxel) pairs (Sec. 3.1).  One wavefront.
__device__ __forceinline__ void inject_body(const InjectArgs& A) {
  const int m = *A.step_ctr;
  const double q = m < A.cap ? A.q[m] : 0.0;
  const float share = float(q / double(A.npairs));
  float* X = A.X2 && (m & 1) ? A.X2 : A.X;
  for (int i = threadIdx.x; i < A.npairs; i += blockDim.x) {
    const int d = A.pairs[2 * i], v = A.pairs[2 * i + 1];
    float content = share;
    if (A.retarded)
      content = share * (A.rDc ? A.rDc[d * 128 + (A.mat[v] & 0x7f)] : A.dirs[d].rD);
    X[size_t(d) * A.Vp + v] += content;
  }
  if (threadIdx.x == 0 && m < A.cap) A.budget[size_t(m) * 9 + 0] = double(share) * A.npairs;
}

__global__ void inject_kernel(InjectArgs A) { inject_body(A); }

// ---------------------------------------------------------------------------
// Collision (Eq. 10 with the explicit source of Eq. 2/12):
//   Y[:, v] = a_v X[:, v] + b_v (P X)[:, v]
// a GEMM with M = K = NP (directions) and N = voxels on MFMA; the epilogue's
// FP64 budget partials are absorbed = sum_v (1 - a_v - b_v) sum_d X[d][v] and
// total = sum X.  Lanes address X and Y with 32-bit byte offsets spanning up to
// five rows, so a medium holds fewer than 2^31 / 20 padded voxels (checked at
// creation).

// Collision with P resident in LDS (NP <= 192, 147 KB): a persistent kernel,
// one 512-thread workgroup per CU, each wavefront owning 32 voxel columns of a
// 256-column tile and all NP direction rows.  In chunk c of the K loop (rows
// 32c .. 32c+31) lane half h loads the X rows 32c + 8(s/4) + 4h + s%4,
// s = 0..15, which are exactly the rows of accumulator block c that the lane
// holds, so the a_v X term is added to the accumulator as those rows arrive:
//   acc = sum_k P[i][k] (b_v X[k][v]) + a_v X[i][v] = Y[i][v]
// and the epilogue only stores.  The next chunk's X is loaded into registers
// while the current one feeds the MFMAs; P comes from LDS as [row][k] with a
// padded pitch, four k per 16-byte read.
template <int NP>
__device__ __forceinline__ void load_p_lds(const float* __restrict__ Prow, float* Ps) {
  constexpr int LDK = NP + 4;
  for (int e = threadIdx.x * 4; e < NP * NP; e += 512 * 4) {
    const int r = e / NP, k = e - r * NP;
    *reinterpret_cast<float4*>(Ps + r * LDK + k) =
        *reinterpret_cast<const float4*>(Prow + size_t(r) * NP + k);
  }
}

// One 256-column tile (eight wavefronts of 32 columns) into the accumulators:
// lane (h, c) of wavefront w holds column 256 tile + 32 w + c and, in acc[q][s],
// row 32q + 8(s/4) + 4h + s%4.  Adds this thread's share of the tile's budget
// sums to absorbed and total.
// The lane's X rows of a chunk: row block c, step s, lane half h holds row
// 32c + 8(s/4) + 4h + s%4 (the 4h part in the lane's offset).
struct TileHead {
  float x[16];   // chunk 0 of the lane's column
  float av, bv;  // the column's collision coefficients
};

__device__ __forceinline__ unsigned tile_lane_offset(const CollideArgs& A, int tile) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long col = (long long)tile * 256 + wave * 32 + (lane & 31);
  return unsigned(size_t(col) * sizeof(float) + size_t(4 * (lane >> 5)) * size_t(A.Vp) * sizeof(float));
}

__device__ __forceinline__ float tile_x(const CollideArgs& A, unsigned voff, int c, int s) {
  const char* rb = reinterpret_cast<const char*>(A.X) +
                   size_t(32 * c + 8 * (s >> 2) + (s & 3)) * size_t(A.Vp) * sizeof(float);
  return *reinterpret_cast<const float*>(rb + voff);
}

__device__ __forceinline__ void load_tile_head(const CollideArgs& A, int tile, TileHead& H) {
  const unsigned voff = tile_lane_offset(A, tile);
  const long long col = (long long)tile * 256 + (threadIdx.x >> 6) * 32 + (threadIdx.x & 31);
#pragma unroll
  for (int s = 0; s < 16; ++s) H.x[s] = tile_x(A, voff, 0, s);
  H.av = A.a[col];
  H.bv = A.b[col];
}

// H holds the tile's head on entry; with next >= 0 it holds tile next's head
// on return, loaded during the last chunk's MFMAs (else it is spent).
template <int NP>
__device__ __forceinline__ void collide_res_acc(const CollideArgs& A, const float* Ps, int tile,
                                                floatx16 (&acc)[NP / 32], double& absorbed,
                                                double& total, TileHead& H, int next) {
  constexpr int NQ = NP / 32;
  constexpr int LDK = NP + 4;
  const int lane = threadIdx.x & 63;
  const int hl = lane >> 5, cl = lane & 31;
  const float* __restrict__ Pl = Ps + cl * LDK + 4 * hl;
  const unsigned voff = tile_lane_offset(A, tile);
  const unsigned voffn = tile_lane_offset(A, next >= 0 ? next : tile);
  const float av = H.av, bv = H.bv;
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[q][r] = 0.0f;
  float bcur[16], bnext[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) bcur[s] = H.x[s];
  double colsum64 = 0.0;
#pragma unroll 1
  for (int c = 0; c < NQ; ++c) {
    // the last chunk loads the next tile's head (or its own first chunk again)
    const bool last = c + 1 == NQ;
    const unsigned vo = last ? voffn : voff;
    const int cn = last ? 0 : c + 1;
#pragma unroll
    for (int s = 0; s < 16; ++s) bnext[s] = tile_x(A, vo, cn, s);
    float colsum = 0.0f;
#pragma unroll
    for (int s = 0; s < 16; ++s) colsum += bcur[s];
    colsum64 += double(colsum);
    // a_v X for the rows of accumulator block c (uniform branch)
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      if (q == c) {
#pragma unroll
        for (int s = 0; s < 16; ++s) acc[q][s] = fmaf(av, bcur[s], acc[q][s]);
      }
#pragma unroll
    for (int s = 0; s < 16; ++s) bcur[s] *= bv;
#pragma unroll
    for (int s4 = 0; s4 < 16; s4 += 4) {
      // k of step s (s = s4..s4+3): 32c + 8(s/4) + 4h + s%4 -> four consecutive k per half
      const int kk = 32 * c + 8 * (s4 >> 2);
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const float4 a4 = *reinterpret_cast<const float4*>(Pl + q * 32 * LDK + kk);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.x, bcur[s4 + 0], acc[q], 0, 0, 0);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.y, bcur[s4 + 1], acc[q], 0, 0, 0);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.z, bcur[s4 + 2], acc[q], 0, 0, 0);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.w, bcur[s4 + 3], acc[q], 0, 0, 0);
      }
    }
#pragma unroll
    for (int s = 0; s < 16; ++s) bcur[s] = bnext[s];
  }
  absorbed += (1.0 - double(av) - double(bv)) * colsum64;
  total += colsum64;
  if (next >= 0) {
    const long long coln = (long long)next * 256 + (threadIdx.x >> 6) * 32 + cl;
#pragma unroll
    for (int s = 0; s < 16; ++s) H.x[s] = bcur[s];
    H.av = A.a[coln];
    H.bv = A.b[coln];
  }
}

template <int NP>
__device__ __forceinline__ void collide_res_acc(const CollideArgs& A, const float* Ps, int tile,
                                                floatx16 (&acc)[NP / 32], double& absorbed,
                                                double& total) {
  TileHead H;
  load_tile_head(A, tile, H);
  collide_res_acc<NP>(A, Ps, tile, acc, absorbed, total, H, -1);
}

// Stores a tile's accumulators (the layout of collide_res_acc) to Y.
template <int NQ>
__device__ __forceinline__ void store_res_tile(const CollideArgs& A, const floatx16 (&acc)[NQ],
                                               int tile) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int hl = lane >> 5, cl = lane & 31;
  const size_t rowbytes = size_t(A.Vp) * sizeof(float);
  const long long col = (long long)tile * 256 + wave * 32 + cl;
  const unsigned voff = unsigned(size_t(col) * sizeof(float) + size_t(4 * hl) * rowbytes);
  char* __restrict__ yb0 = reinterpret_cast<char*>(A.Y);
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r)
      *reinterpret_cast<float*>(yb0 + size_t(q * 32 + 8 * (r >> 2) + (r & 3)) * rowbytes + voff) =
          acc[q][r];
}

template <int NP>
__device__ __forceinline__ void collide_res_tile(const CollideArgs& A, const float* Ps, int tile,
                                                 double& absorbed, double& total) {
  floatx16 acc[NP / 32];
  collide_res_acc<NP>(A, Ps, tile, acc, absorbed, total);
  store_res_tile<NP / 32>(A, acc, tile);
}

// Sums of two doubles over a 512-thread workgroup, written by thread 0 and 1.
__device__ __forceinline__ void block_sums512(double a, double t, double* out_a, double* out_t) {
  __shared__ double red2[2][8];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double sa = wave_sum(a), st = wave_sum(t);
  __syncthreads();
  if (lane == 0) {
    red2[0][wave] = sa;
    red2[1][wave] = st;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double s = 0;
    for (int w = 0; w < 8; ++w) s += red2[threadIdx.x][w];
    *(threadIdx.x == 0 ? out_a : out_t) = s;
  }
}

template <int NP>
__global__ __launch_bounds__(512, 1) void collide_f32_res_kernel(CollideArgs A, int ntiles) {
  extern __shared__ float Ps[];
  load_p_lds<NP>(A.Prow, Ps);
  __syncthreads();
  double absorbed = 0.0, total = 0.0;
#pragma unroll 1
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
    collide_res_tile<NP>(A, Ps, tile, absorbed, total);
  block_sums512(absorbed, total, A.part + blockIdx.x, A.part + gridDim.x + blockIdx.x);
}

// Collision over one hop, for stepping below Courant one (Sec. 2.1, the
// retarded form of Eq. 10 with S1 := S0).  Direction i hops dr_i = dx/|Omega_a|
// between planes, so its coefficients depend on the row as well as the voxel:
//   a[i][v] = exp(-mu_t(v) dr_i),  b[i][v] = omega_v (1 - a[i][v]).
// With e = 1 - a the result is C = e (w X + omega P X), w = a / e: the B
// operand is omega_v X, and w X is added to the accumulator as the lane's own
// rows of X arrive (the row order of collide_res_tile), so X is read once.
// The factor e cancels on the X term (e * (a/e) = a up to rounding), and the
// P X term carries the absolute error of e, 2^-25.  Voxels with
// mu_t dx < 2^-20 come with omega = 0 from the host and take C = X (a = 1).
// C goes to the history slot of the current step.  Absorbed per step, with the
// light of a hop spread over its D_i steps: e (1 - omega) X[i][v] / D_i.
// With a varying index the hop from v lasts D_i / rvox[v] steps (the absorbed
// tally takes the factor rvox[v]).
// FLUX: the source weighted by the light each direction scatters per step,
//   C_i = a_i X_i + D_i omega sum_j P_ij e_j X_j / D_j,
// so scattering conserves photons; the B operand is omega e_j X_j / D_j, the
// lane's own rows add a_i X_i / D_i, and the epilogue multiplies by D_i (the
// voxel factor rvox cancels in D_i / D_j).  A voxel that does not scatter
// keeps C = a X.
template <int NP, bool FLUX>
__device__ __forceinline__ void collide_hop_tile(const CollideArgs& A, const float* Ps,
                                                 const float* sinvc, const float* sinvD,
                                                 const float* sD, float* __restrict__ Cout,
                                                 int tile, double& absorbed, double& total) {
  constexpr int NQ = NP / 32;
  constexpr int LDK = NP + 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int hl = lane >> 5, cl = lane & 31;
  const size_t rowbytes = size_t(A.Vp) * sizeof(float);
  const float* __restrict__ Pl = Ps + cl * LDK + 4 * hl;
  const long long col = (long long)tile * 256 + wave * 32 + cl;
  const unsigned voff = unsigned(size_t(col) * sizeof(float) + size_t(4 * hl) * rowbytes);
  const char* __restrict__ xb0 = reinterpret_cast<const char*>(A.X);
  const float mx = A.mutdx[col], om = A.omega[col];
  // exp(-mu_t dx / |Omega_a|) = exp2(-(mu_t dx log2 e) / |Omega_a|) on the hardware exp2
  const float ml2 = mx * 1.44269504088896341f;
  // the lane half's rows of the hop tables: one base, constant offsets
  const float* __restrict__ ic = sinvc + 4 * hl;
  const float* __restrict__ iD = sinvD + 4 * hl;
  floatx16 acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[q][r] = 0.0f;
  auto ld = [&](int c, int s) {
    const char* rb = xb0 + size_t(32 * c + 8 * (s >> 2) + (s & 3)) * rowbytes;
    return *reinterpret_cast<const float*>(rb + voff);
  };
  float bcur[16], bnext[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) bcur[s] = ld(0, s);
  double colsum = 0.0, lost = 0.0;
#pragma unroll 1
  for (int c = 0; c < NQ; ++c) {
    const int cn = c + 1 < NQ ? c + 1 : c;
#pragma unroll
    for (int s = 0; s < 16; ++s) bnext[s] = ld(cn, s);
    // w X for the rows of accumulator block c (uniform branch); the chunk's
    // tallies in FP32, then into the FP64 sums
    float csum = 0.0f, clost = 0.0f;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int ro = 32 * c + 8 * (s >> 2) + (s & 3);   // row minus 4h
      const float a = __builtin_amdgcn_exp2f(-ml2 * ic[ro]);
      const float e = 1.0f - a;
      // FLUX without scattering (air, pure absorbers): C = a X exactly
      const float w = FLUX ? (om > 0.0f ? a * iD[ro] : a)
                           : (e > 0.0f ? a * __builtin_amdgcn_rcpf(e) : 1.0f);
      csum += bcur[s];
      clost = fmaf(e * bcur[s], iD[ro], clost);
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        if (q == c) acc[q][s] = fmaf(w, bcur[s], acc[q][s]);
      if (FLUX) bcur[s] *= om * (e * iD[ro]);
    }
    colsum += double(csum);
    lost += double(clost);
    if (!FLUX) {
#pragma unroll
      for (int s = 0; s < 16; ++s) bcur[s] *= om;
    }
#pragma unroll
    for (int s4 = 0; s4 < 16; s4 += 4) {
      const int kk = 32 * c + 8 * (s4 >> 2);
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const float4 a4 = *reinterpret_cast<const float4*>(Pl + q * 32 * LDK + kk);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.x, bcur[s4 + 0], acc[q], 0, 0, 0);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.y, bcur[s4 + 1], acc[q], 0, 0, 0);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.z, bcur[s4 + 2], acc[q], 0, 0, 0);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.w, bcur[s4 + 3], acc[q], 0, 0, 0);
      }
    }
#pragma unroll
    for (int s = 0; s < 16; ++s) bcur[s] = bnext[s];
  }
  char* __restrict__ cb0 = reinterpret_cast<char*>(Cout);
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    char* cq = cb0 + size_t(32 * q) * rowbytes + voff;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int ro = q * 32 + 8 * (r >> 2) + (r & 3);
      float f;
      if (FLUX) {
        f = om > 0.0f ? sD[ro + 4 * hl] : 1.0f;
      } else {
        const float e = 1.0f - __builtin_amdgcn_exp2f(-ml2 * ic[ro]);
        f = e > 0.0f ? e : 1.0f;
      }
      *reinterpret_cast<float*>(cq + size_t(8 * (r >> 2) + (r & 3)) * rowbytes) = f * acc[q][r];
    }
  }
  const double rv = A.rvox ? double(A.rvox[col]) : 1.0;
  absorbed += (1.0 - double(om)) * lost * rv;
  total += colsum;
}

template <int NP, bool FLUX>
__global__ __launch_bounds__(512, 1) void collide_hop_kernel(CollideArgs A, int ntiles) {
  extern __shared__ float Ps[];
  float* sinvc = Ps + NP * (NP + 4);
  float* sinvD = sinvc + NP;
  float* sD = sinvD + NP;
  load_p_lds<NP>(A.Prow, Ps);
  for (int i = threadIdx.x; i < NP; i += 512) {
    sinvc[i] = A.hinvc[i];
    sinvD[i] = A.hinvD[i];
    if (FLUX) sD[i] = A.hD[i];
  }
  __syncthreads();
  const int m = *A.step_ctr;
  float* Cout = A.ring + size_t(m % A.H) * size_t(NP) * size_t(A.Vp);
  double absorbed = 0.0, total = 0.0;
#pragma unroll 1
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
    collide_hop_tile<NP, FLUX>(A, Ps, sinvc, sinvD, sD, Cout, tile, absorbed, total);
  block_sums512(absorbed, total, A.part + blockIdx.x, A.part + gridDim.x + blockIdx.x);
}

// BF16-split collision with P_hi and P_lo resident in LDS (NP <= 192, 154 KB):
// the persistent layout of collide_f32_res_kernel on v_mfma_f32_32x32x16_bf16.
// A 16-deep K step takes 8 k per lane half; the k slots are mapped to physical
// rows so that, over the two K steps of row block c, lane half h loads exactly
// the 16 rows 32c + 8(s/4) + 4h + s%4 (s = 0..15) its accumulator holds, and
// a_v X is again added as the rows arrive: slot j of K step t is row
// 32c + 4h + 8(2t + j/4) + j%4, s = 8t + j.  P's columns are stored in LDS in
// that slot order, so each lane's 8 k of a K step are one 16-byte read.
template <int NP>
__device__ __forceinline__ void load_p_bf16_lds(const uint16_t* __restrict__ Phi,
                                                const uint16_t* __restrict__ Plo, uint16_t* Sh,
                                                uint16_t* Sl) {
  constexpr int LDK = NP + 8;
  // groups of 4 slots: kappa = 32c + 16t + 8h + 4g2 holds physical columns
  // 32c + 4h + 8(2t + g2) .. +3
  for (int e = threadIdx.x; e < NP * (NP / 4); e += 512) {
    const int r = e / (NP / 4), kap = (e - r * (NP / 4)) * 4;
    const int c = kap >> 5, t = (kap >> 4) & 1, h = (kap >> 3) & 1, g2 = (kap >> 2) & 1;
    const int ph = 32 * c + 4 * h + 8 * (2 * t + g2);
    *reinterpret_cast<uint2*>(Sh + r * LDK + kap) =
        *reinterpret_cast<const uint2*>(Phi + size_t(r) * NP + ph);
    *reinterpret_cast<uint2*>(Sl + r * LDK + kap) =
        *reinterpret_cast<const uint2*>(Plo + size_t(r) * NP + ph);
  }
}

// The bf16-split form of collide_res_acc (same layouts; H as there).
template <int NP>
__device__ __forceinline__ void collide_bf16_res_acc(const CollideArgs& A, const uint16_t* Sh,
                                                     const uint16_t* Sl, int tile,
                                                     floatx16 (&acc)[NP / 32], double& absorbed,
                                                     double& total, TileHead& H, int next) {
  constexpr int NQ = NP / 32;
  constexpr int LDK = NP + 8;
  const int lane = threadIdx.x & 63;
  const int hl = lane >> 5, cl = lane & 31;
  const unsigned voff = tile_lane_offset(A, tile);
  const unsigned voffn = tile_lane_offset(A, next >= 0 ? next : tile);
  const uint16_t* __restrict__ Ph = Sh + cl * LDK + 8 * hl;
  const uint16_t* __restrict__ Pl = Sl + cl * LDK + 8 * hl;
  const float av = H.av, bv = H.bv;
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[q][r] = 0.0f;
  float bcur[16], bnext[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) bcur[s] = H.x[s];
  double colsum64 = 0.0;
#pragma unroll 1
  for (int c = 0; c < NQ; ++c) {
    const bool last = c + 1 == NQ;
    const unsigned vo = last ? voffn : voff;
    const int cn = last ? 0 : c + 1;
#pragma unroll
    for (int s = 0; s < 16; ++s) bnext[s] = tile_x(A, vo, cn, s);
    float colsum = 0.0f;
#pragma unroll
    for (int s = 0; s < 16; ++s) colsum += bcur[s];
    colsum64 += double(colsum);
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      if (q == c) {
#pragma unroll
        for (int s = 0; s < 16; ++s) acc[q][s] = fmaf(av, bcur[s], acc[q][s]);
      }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      bf16x8 xh, xl;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float x = bcur[8 * t + j] * bv;
        xh[j] = static_cast<__bf16>(x);
        xl[j] = bf16_rest(x, xh[j]);
      }
      const int kk = 32 * c + 16 * t;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const bf16x8 ph = *reinterpret_cast<const bf16x8*>(Ph + q * 32 * LDK + kk);
        const bf16x8 pl = *reinterpret_cast<const bf16x8*>(Pl + q * 32 * LDK + kk);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ph, xh, acc[q], 0, 0, 0);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ph, xl, acc[q], 0, 0, 0);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pl, xh, acc[q], 0, 0, 0);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pl, xl, acc[q], 0, 0, 0);
      }
    }
#pragma unroll
    for (int s = 0; s < 16; ++s) bcur[s] = bnext[s];
  }
  absorbed += (1.0 - double(av) - double(bv)) * colsum64;
  total += colsum64;
  if (next >= 0) {
    const long long coln = (long long)next * 256 + (threadIdx.x >> 6) * 32 + cl;
#pragma unroll
    for (int s = 0; s < 16; ++s) H.x[s] = bcur[s];
    H.av = A.a[coln];
    H.bv = A.b[coln];
  }
}

template <int NP>
__device__ __forceinline__ void collide_bf16_res_acc(const CollideArgs& A, const uint16_t* Sh,
                                                     const uint16_t* Sl, int tile,
                                                     floatx16 (&acc)[NP / 32], double& absorbed,
                                                     double& total) {
  TileHead H;
  load_tile_head(A, tile, H);
  collide_bf16_res_acc<NP>(A, Sh, Sl, tile, acc, absorbed, total, H, -1);
}

template <int NP>
__device__ __forceinline__ void collide_bf16_res_tile(const CollideArgs& A, const uint16_t* Sh,
                                                      const uint16_t* Sl, int tile,
                                                      double& absorbed, double& total) {
  floatx16 acc[NP / 32];
  collide_bf16_res_acc<NP>(A, Sh, Sl, tile, acc, absorbed, total);
  store_res_tile<NP / 32>(A, acc, tile);
}

template <int NP>
__global__ __launch_bounds__(512, 1) void collide_bf16_res_kernel(CollideArgs A, int ntiles) {
  extern __shared__ uint16_t Sm[];
  uint16_t* Sh = Sm;
  uint16_t* Sl = Sm + NP * (NP + 8);
  load_p_bf16_lds<NP>(A.Phi, A.Plo, Sh, Sl);
  __syncthreads();
  double absorbed = 0.0, total = 0.0;
#pragma unroll 1
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
    collide_bf16_res_tile<NP>(A, Sh, Sl, tile, absorbed, total);
  block_sums512(absorbed, total, A.part + blockIdx.x, A.part + gridDim.x + blockIdx.x);
}

// ---------------------------------------------------------------------------
// Phase stepping with the moves in the collision's epilogue.  In phase mode a
// direction either stays this step (the collided value is the new value) or
// moves all its photons one plane along its characteristic (Sec. 2.1, the ray
// lattice), so the transport is a permutation of the collided field plus the
// light that leaves the box.  After the MFMA main loop a lane holds the
// collided values of its voxel for 16 rows per row block; it writes each one
// straight to the downwind voxel in the other field, and the collided field is
// never stored and read back.
//   * The moves of a direction are one-to-one (the transverse shift at a plane
//     is the same for the whole plane): a destination gets one value or none.
//     Wrapped around the box they map it onto itself, so a value that leaves
//     sends a zero to its wrapped destination, a voxel that nothing flows into.
//   * Light leaves and inflow is missing only at voxels on the box surface.  A
//     voxel on one face sends all its leaving light through that face, so one
//     FP32 sum per lane suffices; a wavefront holding an edge voxel (two or
//     more faces) applies the sweep's precedence (dominant axis, then b, then c)
//     value by value.
//   * A value that leaves a detector's voxel is written over the lane's own
//     column of the input field, which no other workgroup reads; the
//     detectors read it there.  Elsewhere leaving light is only tallied.

struct MoveLane {
  unsigned P;    // x | y << 10 | z << 20
  unsigned LF;   // faces the voxel lies on (bit 2 axis + side); all six on padding columns
};

__device__ __forceinline__ MoveLane move_lane(const CollideArgs& A, long long col) {
  MoveLane L{0u, 0x3Fu};
  if (col < A.nvox) {
    const int nxy = A.nx * A.ny;
    const int v = int(col);
    const int z = v / nxy, rem = v - z * nxy;
    const int y = rem / A.nx, x = rem - y * A.nx;
    L.P = unsigned(x) | unsigned(y) << 10 | unsigned(z) << 20;
    L.LF = unsigned(x == 0) | unsigned(x == A.nx - 1) << 1 | unsigned(y == 0) << 2 |
           unsigned(y == A.ny - 1) << 3 | unsigned(z == 0) << 4 | unsigned(z == A.nz - 1) << 5;
  }
  return L;
}

// Buffer resource over `bytes` bytes at p (gfx9 layout: raw, no stride).  A
// buffer store whose offset is at or beyond `bytes` is dropped by the hardware.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, int(bytes), 0x00020000);
}
constexpr unsigned kDropOffset = 0x80000000u;   // above every resource made here

// The scatter of one tile's accumulators (the layout of collide_res_acc).
// fld: both fields; dsv: byte offset of the lane's column in this step's
// output half (with the lane half's 4-row shift); wrap4[f]: the byte offset
// that takes a move out through face f back around the box.  A value that
// stays in the box goes to its downwind voxel.  A value that leaves sends a
// zero to its downwind voxel wrapped around the box: with unit shifts the
// wrapped moves map the box one-to-one onto itself, so the wrapped
// destinations of the values that leave are exactly the voxels that nothing
// flows into, and every voxel of the new field is written once.
// SLOW, for wavefronts holding a voxel on two or more faces, a detector's
// voxel or a padding column: face precedence and wrap per value, the light
// leaving a detector's voxel kept at ssv (the drop offset elsewhere), nothing
// stored for padding columns.  Adds this lane's escape per face and light in
// the box.
template <int NQ, bool SLOW>
__device__ __forceinline__ void move_tile(const int2* sdesc, __amdgpu_buffer_rsrc_t tab,
                                          __amdgpu_buffer_rsrc_t fld, const floatx16 (&acc)[NQ],
                                          const MoveLane& L, const int (&wrap4)[6], unsigned ssv,
                                          unsigned dsv, bool live, unsigned rowbytes, int hl,
                                          double (&esc)[6], double& dom) {
  // a lane on one face leaves through it only
  const int face = L.LF ? __builtin_ctz(L.LF) : 6;
  int wo4 = 0;
#pragma unroll
  for (int i = 0; i < 6; ++i) wo4 = face == i ? wrap4[i] : wo4;
  double lesc = 0.0;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    float fdom = 0.0f, fesc = 0.0f;
    float fe6[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    {
      // the block's 16 table entries (64 offset + face mask) in flight at once
      int w[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int2 dsc = sdesc[q * 32 + 8 * (r >> 2) + (r & 3) + 4 * hl];
        const unsigned p = __builtin_amdgcn_ubfe(L.P, unsigned(dsc.y) & 31u, 10u);
        w[r] = __builtin_amdgcn_raw_buffer_load_b32(tab, int(unsigned(dsc.x) + (p << 2)), 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float val = acc[q][r];
        const unsigned hits = unsigned(w[r]) & L.LF;
        const bool ex = hits != 0u;
        const unsigned ro = unsigned(32 * q + 8 * (r >> 2) + (r & 3)) * rowbytes;
        const unsigned dst = ro + dsv + 4u * unsigned(w[r] >> 6);
        unsigned off;
        if (SLOW) {
          int wr = 0;
#pragma unroll
          for (int i = 0; i < 6; ++i) wr += ((hits >> i) & 1u) ? wrap4[i] : 0;
          off = live ? dst - unsigned(wr) : kDropOffset;
        } else {
          off = ex ? dst - unsigned(wo4) : dst;
        }
        __builtin_amdgcn_raw_buffer_store_b32(ex ? 0u : __float_as_uint(val), fld, int(off), 0, 0);
        if (SLOW)
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(val), fld,
                                                int(ex ? ro + ssv : kDropOffset), 0, 0);
        const float e = ex ? val : 0.0f;
        fdom += val - e;
        if (SLOW) {
          // the sweep's precedence: the dominant-axis face, else the face on the
          // lowest axis hit (b < c); hits holds one face per axis at most
          const unsigned dy = unsigned(sdesc[q * 32 + 8 * (r >> 2) + (r & 3) + 4 * hl].y);
          const unsigned ha = hits & (dy >> 8);
          const unsigned f = unsigned(__builtin_ctz((ha ? ha : hits) | 64u));
#pragma unroll
          for (int i = 0; i < 6; ++i) fe6[i] += f == unsigned(i) ? e : 0.0f;
        } else {
          fesc += e;
        }
      }
    }
    dom += double(fdom);
    if (SLOW) {
#pragma unroll
      for (int i = 0; i < 6; ++i) esc[i] += double(fe6[i]);
    } else {
      lesc += double(fesc);
    }
  }
  if (!SLOW) {
#pragma unroll
    for (int i = 0; i < 6; ++i) esc[i] += face == i ? lesc : 0.0;
  }
}

// This step's direction descriptors (table row, coordinate shift,
// dominant-axis faces), for the whole workgroup; directions that stay point
// at the table's zero row.
template <int NP>
__device__ __forceinline__ void move_descriptors(const CollideArgs& A, int2* sdesc, int m) {
  for (int d = threadIdx.x; d < NP; d += blockDim.x) {
    const bool mv = d < A.ndir && phase_move(A.dirs[d].nu64, m) != 0.0f;
    sdesc[d] = make_int2((mv ? d : NP) * A.mvext * 4, A.mvdir[d]);
  }
}

// What the scatter of step m needs, the same for the whole workgroup: the
// field halves (input so, output dso) behind one buffer resource, the table,
// and the byte offset of a move out through face f (2 axis + side) back
// around the box.
struct MoveStep {
  __amdgpu_buffer_rsrc_t fld, tab;
  unsigned so, dso;
  int wrap4[6];
};

template <int NP>
__device__ __forceinline__ MoveStep move_step(const CollideArgs& A, int m) {
  MoveStep S;
  const size_t half = size_t(NP) * size_t(A.Vp) * sizeof(float);
  S.so = (m & 1) ? unsigned(half) : 0u;
  S.dso = (m & 1) ? 0u : unsigned(half);
  S.fld = raw_rsrc(A.pp, unsigned(2 * half));
  S.tab = raw_rsrc(A.mvtab, unsigned(size_t(NP + 1) * size_t(A.mvext) * sizeof(int)));
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int ax = f >> 1;
    const int ext = ax == 0 ? A.nx : (ax == 1 ? A.ny : A.nz);
    const int stride = ax == 0 ? 1 : (ax == 1 ? A.nx : A.nx * A.ny);
    S.wrap4[f] = (f & 1 ? 4 : -4) * ext * stride;
  }
  return S;
}

// The scatter of tile `tile`, whose accumulators collide_res_acc (or its
// bf16 form) computed from the input half; adds the lane's escape per face
// and light in the box.
template <int NP>
__device__ __forceinline__ void move_epilogue(const CollideArgs& A, const int2* sdesc,
                                              const MoveStep& S, const floatx16 (&acc)[NP / 32],
                                              int tile, double (&esc)[6], double& dom) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int hl = lane >> 5, cl = lane & 31;
  const size_t rowbytes = size_t(A.Vp) * sizeof(float);
  const long long col = (long long)tile * 256 + wave * 32 + cl;
  const unsigned voff = unsigned(size_t(col) * sizeof(float) + size_t(4 * hl) * rowbytes);
  const MoveLane L = move_lane(A, col);
  // light leaving a detector's voxel is kept where the read-out finds it;
  // elsewhere it is only tallied
  const bool det = (A.mvdet[col >> 5] >> (col & 31)) & 1u;
  const bool live = col < A.nvox;
  const unsigned ssv = det ? S.so + voff : kDropOffset;
  if (__any(__builtin_popcount(L.LF) > 1 || det || !live))
    move_tile<NP / 32, true>(sdesc, S.tab, S.fld, acc, L, S.wrap4, ssv, S.dso + voff, live,
                             unsigned(rowbytes), hl, esc, dom);
  else
    move_tile<NP / 32, false>(sdesc, S.tab, S.fld, acc, L, S.wrap4, ssv, S.dso + voff, live,
                              unsigned(rowbytes), hl, esc, dom);
}

// Workgroup sums of the nine tallies (512 threads): absorbed and total to
// part[q * stride + i] (q = 0, 1), escape per face and light in the box to
// spart[q * stride + i] (q = 0..5 faces, 6 in the box).
__device__ __forceinline__ void move_sums(const CollideArgs& A, double absorbed, double total,
                                          const double (&esc)[6], double dom, long long i,
                                          long long stride) {
  __shared__ double red9[9][8];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double v9[9] = {absorbed, total, esc[0], esc[1], esc[2], esc[3], esc[4], esc[5], dom};
  __syncthreads();   // red9 may still be read by the previous call
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const double t = wave_sum(v9[q]);
    if (lane == 0) red9[q][wave] = t;
  }
  __syncthreads();
  if (threadIdx.x < 9) {
    double t = 0.0;
    for (int w = 0; w < 8; ++w) t += red9[threadIdx.x][w];
    const int q = threadIdx.x;
    double* o = q < 2 ? A.part + q * stride + i : A.spart + (q < 8 ? q - 2 : 6) * stride + i;
    *o = t;
  }
}

// P resident in LDS (FP32, or the bf16 hi/lo pair), then this step's
// direction descriptors.  With J.npairs > 0 the kernel also does the step's
// injection (inject_body's arithmetic): each source pair is added by the
// workgroup whose tiles hold its voxel, the only one that reads that column,
// before its first tile.
template <int NP, bool BF16>
__global__ __launch_bounds__(512, 1) void collide_move_kernel(CollideArgs A, InjectArgs J,
                                                              int ntiles) {
  extern __shared__ float Pm[];
  constexpr size_t kPB = BF16 ? 2 * size_t(NP) * (NP + 8) * sizeof(uint16_t)
                              : size_t(NP) * (NP + 4) * sizeof(float);
  int2* sdesc = reinterpret_cast<int2*>(reinterpret_cast<char*>(Pm) + kPB);
  uint16_t* Sh = reinterpret_cast<uint16_t*>(Pm);
  uint16_t* Sl = Sh + NP * (NP + 8);
  if (BF16)
    load_p_bf16_lds<NP>(A.Phi, A.Plo, Sh, Sl);
  else
    load_p_lds<NP>(A.Prow, Pm);
  const int m = *A.step_ctr;
  move_descriptors<NP>(A, sdesc, m);
  const MoveStep S = move_step<NP>(A, A.mvfixed ? 0 : m);
  // a contiguous range of s per workgroup, tile = s * A.mvscramble mod ntiles
  // (a bijection: the multiplier is prime to ntiles), so that the tiles holding
  // edges of the box, which take the per-value face precedence, are spread
  // over the workgroups instead of recurring on the same ones
  const int per = (ntiles + int(gridDim.x) - 1) / int(gridDim.x);
  if (J.npairs > 0) {
    const double qm = m < J.cap ? J.q[m] : 0.0;
    const float share = float(qm / double(J.npairs));
    float* Xin = reinterpret_cast<float*>(reinterpret_cast<char*>(A.pp) + S.so);
    for (int i = threadIdx.x; i < J.npairs; i += blockDim.x) {
      const int d = J.pairs[2 * i], v = J.pairs[2 * i + 1];
      const int s = int((long long)(v >> 8) * A.mvunscramble % ntiles);
      if (s / per == int(blockIdx.x)) Xin[size_t(d) * A.Vp + v] += share;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && m < J.cap)
      J.budget[size_t(m) * 9 + 0] = double(share) * J.npairs;
  }
  __syncthreads();   // descriptors, and the injected values, before the tiles
  CollideArgs B = A;
  B.X = reinterpret_cast<const float*>(reinterpret_cast<const char*>(A.pp) + S.so);
  double absorbed = 0.0, total = 0.0, dom = 0.0;
  double esc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  auto tile_of = [&](int i) {
    const int s = int(blockIdx.x) * per + i;
    return s < ntiles ? int((long long)s * A.mvscramble % ntiles) : -1;
  };
  TileHead H;
  int tile = tile_of(0);
  if (tile >= 0) load_tile_head(B, tile, H);
#pragma unroll 1
  for (int i = 0; i < per && tile >= 0; ++i) {
    const int next = i + 1 < per ? tile_of(i + 1) : -1;
    floatx16 acc[NP / 32];
    if (BF16)
      collide_bf16_res_acc<NP>(B, Sh, Sl, tile, acc, absorbed, total, H, next);
    else
      collide_res_acc<NP>(B, Pm, tile, acc, absorbed, total, H, next);
    move_epilogue<NP>(A, sdesc, S, acc, tile, esc, dom);
    tile = next;
  }
  move_sums(A, absorbed, total, esc, dom, blockIdx.x, gridDim.x);
}

// Column tile and row block of workgroup L of a streamed collision (a 1-D
// grid of ntiles x nrb workgroups).  The nrb row blocks of a column tile read
// the same 256 columns of X.  Workgroups are dispatched to the eight XCDs in
// turn (L mod 8), so the row blocks of a tile get ids L, L + 8, L + 16, ...:
// the same XCD, one after another, and the later ones find X in its L2.
__device__ __forceinline__ void stream_tile(int L, int ntiles, int nrb, int* tile, int* rb) {
  const int G = 8 * nrb;
  const int g = L / G, r = L - g * G;
  const int in_group = ntiles - 8 * g < 8 ? ntiles - 8 * g : 8;
  *tile = 8 * g + r % in_group;
  *rb = r / in_group;
}

// More directions than fit in LDS (NP > 192): the layout of the resident kernel
// (512 threads, 256 voxel columns, lane half h holding the X rows
// 32c + 8(s/4) + 4h + s%4 of row block c, which are the rows of its accumulator
// block when block c lies in the workgroup's row tile), with the workgroup's MT
// rows of P streamed through LDS in 32-column chunks, double-buffered: while
// chunk c feeds the MFMAs, chunk c+1 of P and of X is loaded into registers,
// and it goes to the other LDS buffer before the one barrier per chunk.
// a_v X is added as the X rows of the workgroup's own row tile arrive, so the
// epilogue only stores; the budget partials cover the tile's rows.
template <int MT>
__global__ __launch_bounds__(512, 1) void collide_f32_stream_kernel(CollideArgs A, int ntiles) {
  constexpr int NQ = MT / 32;
  constexpr int KC = 32, LDK = KC + 4;
  constexpr int NPR = (MT * KC / 4 + 511) / 512;   // float4 of P per thread per chunk
  // every thread has NPR float4 when they divide evenly, else all but the last;
  // every slot is filled unconditionally and only the LDS store of a partial
  // slot is guarded (a guarded fill kept preg in scratch)
  constexpr bool kFull = (MT * KC / 4) % 512 == 0;
  extern __shared__ float Pbuf[];                   // [2][MT][LDK]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int hl = lane >> 5, cl = lane & 31;
  const int NC = A.NP / KC;
  int tile, rb;
  stream_tile(int(blockIdx.x), ntiles, A.NP / MT, &tile, &rb);
  const int row0 = rb * MT;
  const size_t rowbytes = size_t(A.Vp) * sizeof(float);
  const long long col = (long long)tile * 256 + wave * 32 + cl;
  const unsigned voff = unsigned(size_t(col) * sizeof(float) + size_t(4 * hl) * rowbytes);
  const char* __restrict__ xb0 = reinterpret_cast<const char*>(A.X);
  const float av = A.a[col], bv = A.b[col];
  auto ld = [&](int c, int s) {
    const char* rb = xb0 + size_t(32 * c + 8 * (s >> 2) + (s & 3)) * rowbytes;
    return *reinterpret_cast<const float*>(rb + voff);
  };
  // P chunk staging, written out in place (no lambda holding preg by
  // reference, which kept it in scratch)
  float4 preg[NPR];
#define TRINITY_STAGE_P(cc)                                                                   \
  _Pragma("unroll") for (int i = 0; i < NPR; ++i) {                                           \
    /* a partial last slot reads element 0 again (in range, not stored) */                    \
    const int e0 = tid + i * 512;                                                             \
    const int e = (kFull || i + 1 < NPR || e0 < MT * KC / 4) ? e0 : 0;                        \
    const int r = e / (KC / 4), k4 = (e - r * (KC / 4)) * 4;                                  \
    preg[i] = *reinterpret_cast<const float4*>(A.Prow + size_t(row0 + r) * A.NP + 32 * (cc) + \
                                               k4);                                           \
  }
#define TRINITY_PUT_P(buf)                                                                    \
  _Pragma("unroll") for (int i = 0; i < NPR; ++i) {                                           \
    const int e = tid + i * 512;                                                              \
    if (kFull || i + 1 < NPR || e < MT * KC / 4) {                                            \
      const int r = e / (KC / 4), k4 = (e - r * (KC / 4)) * 4;                                \
      *reinterpret_cast<float4*>(Pbuf + (buf) * MT * LDK + r * LDK + k4) = preg[i];           \
    }                                                                                         \
  }
  floatx16 acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[q][r] = 0.0f;
  float bcur[16], bnext[16];
  TRINITY_STAGE_P(0)
#pragma unroll
  for (int s = 0; s < 16; ++s) bcur[s] = ld(0, s);
  TRINITY_PUT_P(0)
  __syncthreads();
  double colsum64 = 0.0;
#pragma unroll 1
  for (int c = 0; c < NC; ++c) {
    const int cn = c + 1 < NC ? c + 1 : c;   // the last chunk reloads itself (in bounds, unused)
    TRINITY_STAGE_P(cn)
#pragma unroll
    for (int s = 0; s < 16; ++s) bnext[s] = ld(cn, s);
    const int qc = c - row0 / 32;           // accumulator block of this chunk's rows, if in the tile
    if (qc >= 0 && qc < NQ) {
      float cs = 0.0f;
#pragma unroll
      for (int s = 0; s < 16; ++s) cs += bcur[s];
      colsum64 += double(cs);
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        if (q == qc) {
#pragma unroll
          for (int s = 0; s < 16; ++s) acc[q][s] = fmaf(av, bcur[s], acc[q][s]);
        }
    }
#pragma unroll
    for (int s = 0; s < 16; ++s) bcur[s] *= bv;
    const float* __restrict__ Pl = Pbuf + (c & 1) * MT * LDK + cl * LDK + 4 * hl;
#pragma unroll
    for (int s4 = 0; s4 < 16; s4 += 4) {
      const int kk = 8 * (s4 >> 2);
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const float4 a4 = *reinterpret_cast<const float4*>(Pl + q * 32 * LDK + kk);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.x, bcur[s4 + 0], acc[q], 0, 0, 0);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.y, bcur[s4 + 1], acc[q], 0, 0, 0);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.z, bcur[s4 + 2], acc[q], 0, 0, 0);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.w, bcur[s4 + 3], acc[q], 0, 0, 0);
      }
    }
    if (c + 1 < NC) {
      TRINITY_PUT_P((c + 1) & 1)
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 16; ++s) bcur[s] = bnext[s];
  }
  char* __restrict__ yb0 = reinterpret_cast<char*>(A.Y);
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r)
      *reinterpret_cast<float*>(yb0 + size_t(row0 + q * 32 + 8 * (r >> 2) + (r & 3)) * rowbytes +
                                voff) = acc[q][r];
  block_sums512((1.0 - double(av) - double(bv)) * colsum64, colsum64, A.part + blockIdx.x,
                A.part + gridDim.x + blockIdx.x);
#undef TRINITY_STAGE_P
#undef TRINITY_PUT_P
}

// BF16-split form of collide_f32_stream_kernel: P_hi and P_lo chunks of 32
// columns in LDS, double-buffered, with each chunk's columns stored in the k
// slot order of collide_bf16_res_kernel (slot 16t + 8h + j holds column
// 4h + 8(2t + j/4) + j%4 of the chunk), so each lane's 8 k of a K step are one
// 16-byte read and its X rows are its accumulator rows.
//   Three bf16 products per term: P_hi x_hi + P_hi x_lo + P_lo x_hi, with
// x = b X split into x_hi + x_lo.  The fourth, P_lo x_lo (2^-16 of the term),
// is left out, and so that scattering still conserves the light of every
// incoming direction k, its column total x_lo[k] sum_i P_lo[i][k] is added to
// row k itself (A.plocol[k] = sum_i P_lo[i][k]), as the lane's own rows of X
// arrive together with a_v X.
template <int MT>
__global__ __launch_bounds__(512, 1) void collide_bf16_stream_kernel(CollideArgs A, int ntiles) {
  constexpr int NQ = MT / 32;
  constexpr int KC = 32, LDK = KC + 8;             // bf16 per LDS row
  extern __shared__ uint16_t Sbuf[];               // [2][hi, lo][MT][LDK]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int hl = lane >> 5, cl = lane & 31;
  const int NC = A.NP / KC;
  int tile, rb;
  stream_tile(int(blockIdx.x), ntiles, A.NP / MT, &tile, &rb);
  const int row0 = rb * MT;
  const unsigned rowbytes = unsigned(A.Vp) * 4u;   // < 2^31 / 5 (grid limit)
  const long long col = (long long)tile * 256 + wave * 32 + cl;
  // X through buffer loads: a resource per group of 8 rows (its base in
  // scalar registers), the lane's column and row half in one VGPR offset, the
  // row within the group in the scalar offset
  const unsigned voff = unsigned(col) * 4u + 4u * unsigned(hl) * rowbytes;
  const char* __restrict__ xb0 = reinterpret_cast<const char*>(A.X);
  const float av = A.a[col], bv = A.b[col];
  auto ldc = [&](int c, float (&b)[16]) {
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const __amdgpu_buffer_rsrc_t rs =
          raw_rsrc(xb0 + size_t(32 * c + 8 * g) * rowbytes, 8u * rowbytes);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        b[4 * g + j] =
            __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, int(voff), int(j * rowbytes), 0));
    }
  };
  // P_hi / P_lo staging: thread tid takes row tid / 2 of the chunk and its 16
  // columns 16 (tid & 1) .. +15, read as two 16-byte loads (columns 0-7 and
  // 8-15 of the group, the chunk in the scalar offset) and written as two
  // 16-byte LDS stores in the operand order of the MFMA's k slots: slots 0-7
  // take columns 0-3 and 8-11, slots 8-15 columns 4-7 and 12-15 (the X rows
  // the lane halves hold)
  const __amdgpu_buffer_rsrc_t rph = raw_rsrc(A.Phi, unsigned(A.NP) * unsigned(A.NP) * 2u);
  const __amdgpu_buffer_rsrc_t rpl = raw_rsrc(A.Plo, unsigned(A.NP) * unsigned(A.NP) * 2u);
  const int sr = tid >> 1, sg = 16 * (tid & 1);
  const bool sact = sr < MT;
  const unsigned poff = 2u * unsigned((row0 + (sact ? sr : 0)) * A.NP + sg);
  using u32x4 = unsigned __attribute__((ext_vector_type(4)));
  u32x4 ha, hb, la, lb;
  auto stage = [&](int c) {
    if (!sact) return;
    ha = __builtin_amdgcn_raw_buffer_load_b128(rph, int(poff), 64 * c, 0);
    hb = __builtin_amdgcn_raw_buffer_load_b128(rph, int(poff), 64 * c + 16, 0);
    la = __builtin_amdgcn_raw_buffer_load_b128(rpl, int(poff), 64 * c, 0);
    lb = __builtin_amdgcn_raw_buffer_load_b128(rpl, int(poff), 64 * c + 16, 0);
  };
  auto put = [&](int buf) {
    if (!sact) return;
    uint16_t* Sh = Sbuf + buf * 2 * MT * LDK + sr * LDK + sg;
    uint16_t* Sl = Sh + MT * LDK;
    *reinterpret_cast<u32x4*>(Sh) = u32x4{ha[0], ha[1], hb[0], hb[1]};
    *reinterpret_cast<u32x4*>(Sh + 8) = u32x4{ha[2], ha[3], hb[2], hb[3]};
    *reinterpret_cast<u32x4*>(Sl) = u32x4{la[0], la[1], lb[0], lb[1]};
    *reinterpret_cast<u32x4*>(Sl + 8) = u32x4{la[2], la[3], lb[2], lb[3]};
  };
  floatx16 acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[q][r] = 0.0f;
  float b0[16], b1[16];
  stage(0);
  ldc(0, b0);
  put(0);
  __syncthreads();
  double colsum64 = 0.0;
  // B operands of a chunk: x = b X split into bf16 hi + lo; the next chunk's
  // are formed after the current chunk's MFMAs are issued, before the barrier
  bf16x8 xh[2], xl[2];
  auto split = [&](const float (&bx)[16]) {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float x = bx[8 * t + j] * bv;
        xh[t][j] = static_cast<__bf16>(x);
        xl[t][j] = bf16_rest(x, xh[t][j]);
      }
  };
  split(b0);
#pragma unroll 1
  for (int c = 0; c < NC; ++c) {
    const int cn = c + 1 < NC ? c + 1 : c;   // the last chunk restages itself (in bounds, unused)
    stage(cn);
    if (c + 1 < NC) ldc(c + 1, b1);
    const int qc = c - row0 / 32;           // accumulator block of this chunk's rows, if in the tile
    if (qc >= 0 && qc < NQ) {
      float cs = 0.0f;
#pragma unroll
      for (int s = 0; s < 16; ++s) cs += b0[s];
      colsum64 += double(cs);
      // the chunk's 32 column totals through scalar loads (the table is
      // read-only): the wait for a vector load here would also wait for the
      // next chunk's X loads issued before it; each lane half picks its rows
      typedef const __attribute__((address_space(4))) float* const_f32p;
      const const_f32p pq = (const_f32p)(A.plocol + 32 * c);
      float pv[32];
#pragma unroll
      for (int k = 0; k < 32; ++k)
        pv[k] = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(pq[k])));
      float pc[16];
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int i = 0; i < 4; ++i) pc[4 * g + i] = hl ? pv[8 * g + 4 + i] : pv[8 * g + i];
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        if (q == qc) {
#pragma unroll
          for (int s = 0; s < 16; ++s) {
            acc[q][s] = fmaf(av, b0[s], acc[q][s]);
            acc[q][s] = fmaf(pc[s], static_cast<float>(xl[s >> 3][s & 7]), acc[q][s]);
          }
        }
    }
    const uint16_t* __restrict__ Ph = Sbuf + (c & 1) * 2 * MT * LDK + cl * LDK + 8 * hl;
    const uint16_t* __restrict__ Pl = Ph + MT * LDK;
    // the issuing wave's priority is raised while it feeds the MFMAs, so the
    // other wave of the SIMD does its staging and splitting in the gaps
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const bf16x8 ph = *reinterpret_cast<const bf16x8*>(Ph + q * 32 * LDK + 16 * t);
        const bf16x8 pl = *reinterpret_cast<const bf16x8*>(Pl + q * 32 * LDK + 16 * t);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ph, xh[t], acc[q], 0, 0, 0);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ph, xl[t], acc[q], 0, 0, 0);
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pl, xh[t], acc[q], 0, 0, 0);
      }
    }
    __builtin_amdgcn_s_setprio(0);
    if (c + 1 < NC) split(b1);
    if (c + 1 < NC) put((c + 1) & 1);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 16; ++s) b0[s] = b1[s];
  }
  char* __restrict__ yb0 = reinterpret_cast<char*>(A.Y);
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const __amdgpu_buffer_rsrc_t rs =
          raw_rsrc(yb0 + size_t(row0 + 32 * q + 8 * g) * rowbytes, 8u * rowbytes);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(acc[q][4 * g + j]), rs, int(voff),
                                              int(j * rowbytes), 0);
    }
  block_sums512((1.0 - double(av) - double(bv)) * colsum64, colsum64, A.part + blockIdx.x,
                A.part + gridDim.x + blockIdx.x);
}

// Implicit source (the converged Steps 3-6 of Sec. 2.4): every voxel's column
// solves (I - w1 P) N_c = a N + w0 P N, i.e. with P = V diag(lambda) V^T
//   N_c = V diag(g) V^T N,   g_k = (a + w0 lambda_k) / (1 - w1 lambda_k).
// Resident layout of collide_f32_res_kernel with V in LDS (V[i][k], padded
// pitch): pass 1 forms Z = V^T X in the accumulators (A operand read down a
// column of V, four 4-byte reads), scales row k of Z by g_k, and pass 2 forms
// Y = V Z one 32-row output block at a time.  Z's accumulator rows for block c
// are exactly the k slots of K block c of pass 2 (the row order in which X is
// read), so Z feeds pass 2 from registers.
template <int NP>
__device__ __forceinline__ void collide_implicit_tile(const CollideArgs& A, const float* Vs,
                                                      const float* lamS, int tile,
                                                      double& absorbed, double& total) {
  constexpr int NQ = NP / 32;
  constexpr int LDK = NP + 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int hl = lane >> 5, cl = lane & 31;
  const size_t rowbytes = size_t(A.Vp) * sizeof(float);
  const long long col = (long long)tile * 256 + wave * 32 + cl;
  const unsigned voff = unsigned(size_t(col) * sizeof(float) + size_t(4 * hl) * rowbytes);
  const char* __restrict__ xb0 = reinterpret_cast<const char*>(A.X);
  const float av = A.a[col], w0 = A.w0[col], w1 = A.w1[col], cv = A.cimp[col];
  floatx16 z[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) z[q][r] = 0.0f;
  auto ld = [&](int c, int s) {
    const char* rb = xb0 + size_t(32 * c + 8 * (s >> 2) + (s & 3)) * rowbytes;
    return *reinterpret_cast<const float*>(rb + voff);
  };
  float bcur[16], bnext[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) bcur[s] = ld(0, s);
  double colsum64 = 0.0;
  // pass 1: z = V^T X; A[k_out][i] = V[i][k_out], i the slot's row of X
#pragma unroll 1
  for (int c = 0; c < NQ; ++c) {
    const int cn = c + 1 < NQ ? c + 1 : c;
#pragma unroll
    for (int s = 0; s < 16; ++s) bnext[s] = ld(cn, s);
    float colsum = 0.0f;
#pragma unroll
    for (int s = 0; s < 16; ++s) colsum += bcur[s];
    colsum64 += double(colsum);
#pragma unroll
    for (int s4 = 0; s4 < 16; s4 += 4) {
      const int i0 = 32 * c + 8 * (s4 >> 2) + 4 * hl;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const float* vc = Vs + size_t(i0) * LDK + q * 32 + cl;
        z[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(vc[0], bcur[s4 + 0], z[q], 0, 0, 0);
        z[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(vc[LDK], bcur[s4 + 1], z[q], 0, 0, 0);
        z[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(vc[2 * LDK], bcur[s4 + 2], z[q], 0, 0, 0);
        z[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(vc[3 * LDK], bcur[s4 + 3], z[q], 0, 0, 0);
      }
    }
#pragma unroll
    for (int s = 0; s < 16; ++s) bcur[s] = bnext[s];
  }
  // z[k] *= g_k for the lane's rows k = 32q + 8(r/4) + 4h + r%4
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float lam = lamS[32 * q + 8 * (r >> 2) + 4 * hl + (r & 3)];
      z[q][r] *= (av + w0 * lam) / (1.0f - w1 * lam);
    }
  // pass 2: Y = V z, block by block; K block c of z sits in z[c] in slot order
  const float* __restrict__ Vl = Vs + cl * LDK + 4 * hl;
  char* __restrict__ yb0 = reinterpret_cast<char*>(A.Y);
#pragma unroll 1
  for (int qo = 0; qo < NQ; ++qo) {
    floatx16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    const float* __restrict__ Vq = Vl + qo * 32 * LDK;
#pragma unroll
    for (int c = 0; c < NQ; ++c)
#pragma unroll
      for (int s4 = 0; s4 < 16; s4 += 4) {
        const float4 a4 = *reinterpret_cast<const float4*>(Vq + 32 * c + 8 * (s4 >> 2));
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.x, z[c][s4 + 0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.y, z[c][s4 + 1], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.z, z[c][s4 + 2], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.w, z[c][s4 + 3], acc, 0, 0, 0);
      }
#pragma unroll
    for (int r = 0; r < 16; ++r)
      *reinterpret_cast<float*>(yb0 + size_t(qo * 32 + 8 * (r >> 2) + (r & 3)) * rowbytes +
                                voff) = acc[r];
  }
  absorbed += (1.0 - double(cv)) * colsum64;
  total += colsum64;
}

template <int NP>
__global__ __launch_bounds__(512, 1) void collide_implicit_kernel(CollideArgs A, int ntiles) {
  extern __shared__ float Vsh[];
  float* lamS = Vsh + NP * (NP + 4);
  load_p_lds<NP>(A.V, Vsh);
  for (int i = threadIdx.x; i < NP; i += 512) lamS[i] = A.lam[i];
  __syncthreads();
  double absorbed = 0.0, total = 0.0;
#pragma unroll 1
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
    collide_implicit_tile<NP>(A, Vsh, lamS, tile, absorbed, total);
  block_sums512(absorbed, total, A.part + blockIdx.x, A.part + gridDim.x + blockIdx.x);
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
// f_v = nu_d r_v.  Grid: (row slabs, directions).  Lanes run along x, so every
// wavefront reads and writes contiguous voxels; the upwind row of a y- or
// z-dominant direction is one shifted row, that of an x-dominant direction
// differs lane by lane by at most one row in y and one in z.

namespace {

struct SweepAcc {
  double esc_a = 0, esc_b0 = 0, esc_b1 = 0, esc_c0 = 0, esc_c1 = 0, dom = 0;
};

// The collided field a moving sweep reads for one direction: one field, or,
// when stepping below Courant one, the blend of two past collided fields at
// the retarded time, w_late C^{m+1-n} + w_early C^{m-n}.
struct OneField {
  const float* __restrict__ p;
  __device__ __forceinline__ float operator[](long long i) const { return p[i]; }
  __device__ __forceinline__ float4 q4(long long q) const {
    return reinterpret_cast<const float4*>(p)[q];
  }
};

struct TwoFields {
  const float* __restrict__ late;
  const float* __restrict__ early;
  float wl, we;
  __device__ __forceinline__ float operator[](long long i) const {
    return fmaf(we, early[i], wl * late[i]);
  }
  __device__ __forceinline__ float4 q4(long long q) const {
    const float4 l = reinterpret_cast<const float4*>(late)[q];
    const float4 e = reinterpret_cast<const float4*>(early)[q];
    return make_float4(fmaf(we, e.x, wl * l.x), fmaf(we, e.y, wl * l.y), fmaf(we, e.z, wl * l.z),
                       fmaf(we, e.w, wl * l.w));
  }
};

// Two-level angular grid: the collided row of fine direction i formed as it is
// read, a_v X[i][v] + T[parent(i)][v] share (the same rounding as apply_kernel).
struct TwoLevelRow {
  const float* __restrict__ x;
  const float* __restrict__ t;
  const float* __restrict__ a;
  float share;
  __device__ __forceinline__ float operator[](long long i) const {
    return fmaf(a[i], x[i], t[i] * share);
  }
  __device__ __forceinline__ float4 q4(long long q) const {
    const float4 xv = reinterpret_cast<const float4*>(x)[q];
    const float4 tv = reinterpret_cast<const float4*>(t)[q];
    const float4 av = reinterpret_cast<const float4*>(a)[q];
    return make_float4(fmaf(av.x, xv.x, tv.x * share), fmaf(av.y, xv.y, tv.y * share),
                       fmaf(av.z, xv.z, tv.z * share), fmaf(av.w, xv.w, tv.w * share));
  }
};

// Direction d's rows at the retarded time m + 1 - D_d, D_d = rlag + rphi: slot
// (m + 1 - rlag) mod H with weight 1 - rphi and slot (m - rlag) mod H with
// weight rphi.  Slots of steps before the first are zero (the ring is cleared
// at reset and a slot is written only at its own step).  With rphi = 0 both
// point at the same row.
__device__ __forceinline__ TwoFields retarded_rows(const float* ring, int H, long long slot,
                                                   long long Vp, const DevDir& D, int d, int m) {
  const int sl = ((m + 1 - D.rlag) % H + H) % H;
  const int se = ((m - D.rlag) % H + H) % H;
  TwoFields t;
  t.late = ring + sl * slot + size_t(d) * Vp;
  t.early = D.rphi > 0.0f ? ring + se * slot + size_t(d) * Vp : t.late;
  t.wl = 1.0f - D.rphi;
  t.we = D.rphi;
  return t;
}

// Row d of the collided field at voxel v at the retarded time m + 1 - (lag + phi)
// for a hop of lag whole steps and fraction phi (the voxel's own class).
__device__ __forceinline__ float retarded_value(const float* ring, int H, long long slot,
                                                long long Vp, int d, int m, int lag, float phi,
                                                long long v) {
  const int sl = ((m + 1 - lag) % H + H) % H;
  const float late = ring[sl * slot + size_t(d) * Vp + v];
  if (!(phi > 0.0f)) return late;
  const int se = ((m - lag) % H + H) % H;
  return fmaf(phi, ring[se * slot + size_t(d) * Vp + v], (1.0f - phi) * late);
}

constexpr int kMaxExt = 4096;   // largest grid extent (the C-ABI rejects larger)
#ifndef TRINITY_SWEEP_ROWS
#define TRINITY_SWEEP_ROWS 4
#endif
constexpr int kRows = TRINITY_SWEEP_ROWS;   // rows a thread works on at once

// Rows [rb, re) of direction d with dominant axis AX.  Thread layout: tpr
// threads per row (tpr = min(nx, 256)), rpi = 256 / tpr rows per pass; each
// thread takes kRows rows per iteration and issues all their loads first.
// Phase mode (SPLIT false) is only called for directions that move this step
// (f = 1): a voxel then takes its upwind voxel's value and only light that
// leaves the box needs the voxel's own value.
template <int AX, bool SPLIT, bool FRESNEL>
__device__ __forceinline__ void sweep_rows(const SweepArgs& A, const DevDir& D, int d, int rb,
                                           int re, const int8_t* __restrict__ db,
                                           const int8_t* __restrict__ dc, SweepAcc& acc) {
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const long long sxy = (long long)nx * ny;
  constexpr int BX = AX == 0 ? 1 : 0;   // transverse axes b < c
  constexpr int CX = AX == 2 ? 1 : 2;
  const int ext[3] = {nx, ny, nz};
  const long long str[3] = {1, nx, sxy};
  const int ea = ext[AX], eb = ext[BX], ec = ext[CX];
  const long long sa = str[AX], sb = str[BX], sc = str[CX];
  const float* __restrict__ Yd = A.Y + size_t(d) * A.Vp;
  float* __restrict__ Xd = A.X + size_t(d) * A.Vp;
  const int tpr = nx < kThreads ? nx : kThreads;
  const int rpi = kThreads / tpr;
  const int xs = threadIdx.x % tpr, rsub = threadIdx.x / tpr;
  if (rsub >= rpi) return;
  const int sign = D.sign;
  const float nu = D.nu;
  // (y, z) of this thread's next kRows rows, advanced without division
  int yy[kRows], zz[kRows];
  {
    const int row = rb + rsub;
    zz[0] = row / ny;
    yy[0] = row - zz[0] * ny;
#pragma unroll
    for (int i = 1; i < kRows; ++i) {
      yy[i] = yy[i - 1] + rpi;
      zz[i] = zz[i - 1];
      while (yy[i] >= ny) {
        yy[i] -= ny;
        ++zz[i];
      }
    }
  }
  for (int row0 = rb + rsub; row0 < re; row0 += kRows * rpi) {
    for (int x = xs; x < nx; x += tpr) {
      long long v[kRows], u[kRows];
      int k[kRows], pb[kRows], pc[kRows], dbn[kRows], dcn[kRows];
      bool live[kRows], inflow[kRows];
      float yv[kRows], yu[kRows];
#pragma unroll
      for (int i = 0; i < kRows; ++i) {
        const int row = row0 + i * rpi;
        live[i] = row < re;
        const int z = zz[i], y = yy[i];
        const int pa = AX == 0 ? x : (AX == 1 ? y : z);
        k[i] = sign > 0 ? pa : ea - 1 - pa;
        pb[i] = BX == 0 ? x : y;
        pc[i] = CX == 1 ? y : z;
        v[i] = (long long)row * nx + x;
        const int dbk = db[k[i]], dck = dc[k[i]];
        dbn[i] = db[k[i] + 1];
        dcn[i] = dc[k[i] + 1];
        const int ub = pb[i] - dbk, uc = pc[i] - dck;
        inflow[i] = live[i] && k[i] > 0 && (unsigned)ub < (unsigned)eb && (unsigned)uc < (unsigned)ec;
        u[i] = v[i] - sign * sa - dbk * sb - dck * sc;
        if (FRESNEL && inflow[i]) inflow[i] = !(A.iface[u[i]] && A.nvox[u[i]] != A.nvox[v[i]]);
      }
      // exits: the downwind voxel is outside the box
      int exitf[kRows];   // 0 none, 1 a, 2 b0, 3 b1, 4 c0, 5 c1
#pragma unroll
      for (int i = 0; i < kRows; ++i) {
        int e = 0;
        if (k[i] + 1 >= ea) e = 1;
        else if ((unsigned)(pb[i] + dbn[i]) >= (unsigned)eb) e = dbn[i] > 0 ? 3 : 2;
        else if ((unsigned)(pc[i] + dcn[i]) >= (unsigned)ec) e = dcn[i] > 0 ? 5 : 4;
        exitf[i] = live[i] ? e : 0;
      }
#pragma unroll
      for (int i = 0; i < kRows; ++i) {
        yu[i] = inflow[i] ? Yd[u[i]] : 0.0f;
        const bool need_v = SPLIT || FRESNEL || exitf[i] != 0;
        yv[i] = (live[i] && need_v) ? Yd[v[i]] : 0.0f;
      }
#pragma unroll
      for (int i = 0; i < kRows; ++i) {
        if (!live[i]) continue;
        float fv = 1.0f, fu = 1.0f;
        if (SPLIT) {
          fv = nu * A.r[v[i]];
          fu = inflow[i] ? nu * A.r[u[i]] : 0.0f;
        }
        const float out = SPLIT ? fmaf(fu, yu[i], (1.0f - fv) * yv[i]) : yu[i];
        Xd[v[i]] = out;
        acc.dom += double(out);
        const float mv = fv * yv[i];
        switch (exitf[i]) {
          case 1: acc.esc_a += double(mv); break;
          case 2: acc.esc_b0 += double(mv); break;
          case 3: acc.esc_b1 += double(mv); break;
          case 4: acc.esc_c0 += double(mv); break;
          case 5: acc.esc_c1 += double(mv); break;
          default:
            if (FRESNEL && A.iface[v[i]]) {
              const long long w = v[i] + sign * sa + dbn[i] * sb + dcn[i] * sc;
              if (A.nvox[w] != A.nvox[v[i]]) {
                A.icptF[size_t(A.islot[v[i]]) * A.ndir + d] = mv;
                acc.dom += double(mv);
              }
            }
        }
      }
    }
#pragma unroll
    for (int i = 0; i < kRows; ++i) {
      yy[i] += kRows * rpi;
      while (yy[i] >= ny) {
        yy[i] -= ny;
        ++zz[i];
      }
    }
  }
}

// Phase mode, a moving direction whose dominant axis is y or z, any nx: the
// voxels of rows [rb, re) in flat order, kThreads apart, two per thread per
// pass with all loads issued before the stores, so that every lane works
// whatever the row length (one, three, four or eight per pass were slower on
// the 101^3 x 3072 retarded sweep).  Same tallies, in the same order of precedence, as
// the row paths.
template <int AX, class Src>
__device__ __forceinline__ void sweep_phase_flat(const SweepArgs& A, const Src& Yd,
                                                 const DevDir& D, int d, int rb, int re,
                                                 const int8_t* __restrict__ db,
                                                 const int8_t* __restrict__ dc, SweepAcc& acc) {
  static_assert(AX == 1 || AX == 2, "rows run along x");
  constexpr int CX = AX == 2 ? 1 : 2;
  constexpr int U = 2;
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const int ea = AX == 1 ? ny : nz;
  const int ec = CX == 1 ? ny : nz;
  const int sa = AX == 1 ? nx : nx * ny;
  const int sc = CX == 1 ? nx : nx * ny;
  float* __restrict__ Xd = A.X + size_t(d) * A.Vp;
  const int sign = D.sign;
  const int vb = rb * nx, ve = re * nx;
  // passes start on a 128-byte line (32 voxels) at or before the block's first
  // voxel, so a wave's 64 voxels are two whole lines; slots before vb belong
  // to the block before and are skipped
  const int gs = vb & ~31;
  const int drow = kThreads / nx, dxs = kThreads - drow * nx;
  // slot j of a pass takes flat index g0 + j kThreads: its (x, y, z)
  int xs[U], yys[U], zzs[U];
  {
    const int g = gs + threadIdx.x;
    const int row = g / nx;
    xs[0] = g - row * nx;
    zzs[0] = row / ny;
    yys[0] = row - zzs[0] * ny;
#pragma unroll
    for (int j = 1; j < U; ++j) {
      xs[j] = xs[j - 1] + dxs;
      yys[j] = yys[j - 1] + drow;
      zzs[j] = zzs[j - 1];
      if (xs[j] >= nx) { xs[j] -= nx; ++yys[j]; }
      while (yys[j] >= ny) { yys[j] -= ny; ++zzs[j]; }
    }
  }
  const int drowU = U * kThreads / nx, dxU = U * kThreads - drowU * nx;
  for (int g0 = gs + threadIdx.x; g0 < ve; g0 += U * kThreads) {
    float out[U];
    int kk[U], dbn[U], dcn[U];
    bool live[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int v = g0 + j * kThreads;
      live[j] = v >= vb && v < ve;
      const int pa = AX == 1 ? yys[j] : zzs[j];
      const int pc = CX == 1 ? yys[j] : zzs[j];
      kk[j] = sign > 0 ? pa : ea - 1 - pa;
      const int kc = live[j] ? kk[j] : 0;   // slots past the end read in-range tables
      const int dbk = db[kc], dck = dc[kc];
      dbn[j] = db[kc + 1];
      dcn[j] = dc[kc + 1];
      const bool in = live[j] && kk[j] > 0 && (unsigned)(pc - dck) < (unsigned)ec &&
                      (unsigned)(xs[j] - dbk) < (unsigned)nx;
      out[j] = in ? Yd[v - sign * sa - dck * sc - dbk] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      if (!live[j]) continue;
      const int v = g0 + j * kThreads;
      const int pc = CX == 1 ? yys[j] : zzs[j];
      // the field is not read again in this step: stream it past the caches
      __builtin_nontemporal_store(out[j], Xd + v);
      acc.dom += double(out[j]);
      if (kk[j] + 1 >= ea) {
        acc.esc_a += double(Yd[v]);
      } else if ((unsigned)(xs[j] + dbn[j]) >= (unsigned)nx) {
        if (dbn[j] > 0) acc.esc_b1 += double(Yd[v]); else acc.esc_b0 += double(Yd[v]);
      } else if ((unsigned)(pc + dcn[j]) >= (unsigned)ec) {
        if (dcn[j] > 0) acc.esc_c1 += double(Yd[v]); else acc.esc_c0 += double(Yd[v]);
      }
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      xs[j] += dxU;
      int adv = drowU;
      if (xs[j] >= nx) { xs[j] -= nx; ++adv; }
      yys[j] += adv;
      while (yys[j] >= ny) { yys[j] -= ny; ++zzs[j]; }
    }
  }
}

// Phase mode, a moving direction whose dominant axis is y or z, on a grid with
// nx a multiple of 4: every lane moves four consecutive voxels of a row as one
// 16-byte load and store.  The source row is the upwind row, displaced along x
// by the plane-to-plane shift s in {-1, 0, 1}; the one value a lane needs from
// the next four voxels over comes from its neighbour lane (or, at the edge of
// the wave, from memory).  Same tallies, in the same order of precedence, as
// the scalar path.
template <int AX, class Src>
__device__ __forceinline__ void sweep_phase_vec(const SweepArgs& A, const Src& Ysrc,
                                                const DevDir& D, int d, int rb, int re,
                                                const int8_t* __restrict__ db,
                                                const int8_t* __restrict__ dc, SweepAcc& acc) {
  static_assert(AX == 1 || AX == 2, "rows run along x");
  constexpr int CX = AX == 2 ? 1 : 2;
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const int ea = AX == 1 ? ny : nz;
  const int ec = CX == 1 ? ny : nz;
  const int tq = nx >> 2;                              // float4 per row
  const int sa4 = AX == 1 ? tq : tq * ny;              // plane stride in float4
  const int sc4 = CX == 1 ? tq : tq * ny;
  float4* __restrict__ Xd = reinterpret_cast<float4*>(A.X + size_t(d) * A.Vp);
  const int sign = D.sign;
  const int lane = threadIdx.x & 63;
  const int ge = re * tq;
  // flat float4 index g = row * tq + q, advanced by kThreads per pass
  int g = rb * tq + threadIdx.x;
  int row = g / tq, q = g - row * tq;
  int zz = row / ny, yy = row - zz * ny;
  const int drow = kThreads / tq, dq = kThreads - drow * tq;
  for (; g < ge; g += kThreads) {
    const int pa = AX == 1 ? yy : zz;
    const int pc = CX == 1 ? yy : zz;
    const int k = sign > 0 ? pa : ea - 1 - pa;
    const int dbk = db[k], dck = dc[k], dbn = db[k + 1], dcn = dc[k + 1];
    const bool rowin = k > 0 && (unsigned)(pc - dck) < (unsigned)ec;
    const int u = g - sign * sa4 - dck * sc4;
    const float4 y = rowin ? Ysrc.q4(u) : make_float4(0.f, 0.f, 0.f, 0.f);
    // the neighbour lane holds the next four voxels of the same row (q > 0 / q < tq - 1)
    const float prev_w = __shfl_up(y.w, 1);
    const float next_x = __shfl_down(y.x, 1);
    float4 o = y;
    if (dbk > 0) {
      float w = 0.f;
      if (rowin && q > 0) w = lane > 0 ? prev_w : Ysrc[4 * u - 1];
      o = make_float4(w, y.x, y.y, y.z);
    } else if (dbk < 0) {
      float x = 0.f;
      if (rowin && q < tq - 1) x = lane < 63 ? next_x : Ysrc[4 * u + 4];
      o = make_float4(y.y, y.z, y.w, x);
    }
    Xd[g] = o;
    acc.dom += (double(o.x) + double(o.y)) + (double(o.z) + double(o.w));
    // light that leaves: through the exit plane, then the x sides, then the c sides
    const bool last = k + 1 >= ea;
    const bool bx = !last && ((dbn > 0 && q == tq - 1) || (dbn < 0 && q == 0));
    const bool cexit = !last && (unsigned)(pc + dcn) >= (unsigned)ec;
    if (last || bx || cexit) {
      const float4 s4 = Ysrc.q4(g);
      if (last) {
        acc.esc_a += (double(s4.x) + double(s4.y)) + (double(s4.z) + double(s4.w));
      } else {
        float e0 = s4.x, e3 = s4.w;
        if (bx && dbn > 0) { acc.esc_b1 += double(s4.w); e3 = 0.f; }
        if (bx && dbn < 0) { acc.esc_b0 += double(s4.x); e0 = 0.f; }
        if (cexit) {
          const double t = (double(e0) + double(s4.y)) + (double(s4.z) + double(e3));
          if (dcn > 0) acc.esc_c1 += t; else acc.esc_c0 += t;
        }
      }
    }
    q += dq;
    int adv = drow;
    if (q >= tq) { q -= tq; ++adv; }
    yy += adv;
    while (yy >= ny) { yy -= ny; ++zz; }
  }
}

// Split mode with index-class bytes.  A voxel keeps (1 - f_v) of its light and
// takes f_u of its upwind voxel's; the path ratio r comes from the class byte
// through a table in LDS.  Light never crosses between classes on the lattice:
// where the upwind voxel's class differs nothing flows in, and a voxel whose
// downwind voxel has another class hands its moving share to the interception
// buffer (Eq. 13-14) instead.
//
// Every value of Y is read twice, as a voxel's own value and as its downwind
// neighbour's upwind value.  The rows of a direction are therefore taken in
// band order: bands of TB rows across one transverse axis, walked plane by
// plane along the other, and a workgroup takes a contiguous range of (band,
// plane) items.  A row's upwind row was then read at most one item earlier
// (or is read one item later) and is still in the L2 cache, so HBM delivers
// each value once.

// Row (y, z) holds only background-class voxels, none starting an interception.
__device__ __forceinline__ bool bg_row(const uint32_t* __restrict__ rbits, int row) {
  return row < kMaxRowBits && ((rbits[row >> 5] >> (row & 31)) & 1u);
}

// Dominant axis y or z, nx a multiple of 4: four voxels of a row per lane, as
// one 16-byte load and store; the upwind row is displaced along x by the shift
// s in {-1, 0, 1}, and the one value a lane needs from the next four voxels
// over comes from its neighbour lane (or, at the edge of the wave, from memory).
// Bands run across the non-dominant transverse axis c and are walked along the
// dominant axis in the direction of propagation.
template <int AX, bool FRESNEL>
__device__ __forceinline__ void sweep_split_vec(const SweepArgs& A, const DevDir& D, int d,
                                                int blk, int nblk,
                                                const int8_t* __restrict__ db,
                                                const int8_t* __restrict__ dc,
                                                const float* __restrict__ srt,
                                                const uint32_t* __restrict__ rbits,
                                                SweepAcc& acc) {
  static_assert(AX == 1 || AX == 2, "rows run along x");
  constexpr int CX = AX == 2 ? 1 : 2;
  const int nx = A.nx, ny = A.ny;
  const unsigned bg4 = A.bgcls * 0x01010101u;
  const int ns = AX == 1 ? ny : A.nz;   // planes along the dominant axis
  const int nf = CX == 1 ? ny : A.nz;   // rows across c
  const int tq = nx >> 2;
  const int sa4 = AX == 1 ? tq : tq * ny;
  const int sc4 = CX == 1 ? tq : tq * ny;
  const float4* __restrict__ Yd = reinterpret_cast<const float4*>(A.Y + size_t(d) * A.Vp);
  float4* __restrict__ Xd = reinterpret_cast<float4*>(A.X + size_t(d) * A.Vp);
  const float* __restrict__ Ys = A.Y + size_t(d) * A.Vp;
  const unsigned* __restrict__ M4 = reinterpret_cast<const unsigned*>(A.mat);
  const int sign = D.sign;
  const float nu = D.nu;
  const int lane = threadIdx.x & 63;
  // band of TB rows: about two float4 per thread per item (at most four when
  // one row alone exceeds that, nx <= 4096)
  int TB = 2 * kThreads / tq;
  if (TB < 1) TB = 1;
  if (TB > nf) TB = nf;
  const int per = TB * tq;
  constexpr int EMAX = 4;
  int fo[EMAX], qq[EMAX];
#pragma unroll
  for (int j = 0; j < EMAX; ++j) {
    const int e = threadIdx.x + j * kThreads;
    fo[j] = e / tq;
    qq[j] = e - fo[j] * tq;
  }
  const int nb = (nf + TB - 1) / TB;
  const long long T = (long long)nb * ns;   // at most 4096^2 items
  const int i0 = int(T * blk / nblk), i1 = int(T * (blk + 1) / nblk);
  for (int i = i0; i < i1; ++i) {
    const int band = i / ns, k = i - band * ns;
    const int pa = sign > 0 ? k : ns - 1 - k;
    const int dbk = db[k], dck = dc[k], dbn = db[k + 1], dcn = dc[k + 1];
    const bool last = k + 1 >= ns;
#pragma unroll
    for (int j = 0; j < EMAX; ++j) {
      if (j * kThreads >= per) break;
      const int pc = band * TB + fo[j];
      const int q = qq[j];
      const bool act = threadIdx.x + j * kThreads < per && pc < nf;
      const int y = AX == 2 ? pc : pa, z = AX == 2 ? pa : pc;
      const int g = (z * ny + y) * tq + q;
      const bool rowin = act && k > 0 && (unsigned)(pc - dck) < (unsigned)nf;
      const int u = g - sign * sa4 - dck * sc4;
      float4 yv = make_float4(0.f, 0.f, 0.f, 0.f), yu = yv;
      unsigned mv = 0, mu = 0;
      // class bytes: the background class for rows the bitmap marks, else per voxel
      const int row = z * ny + y;
      const int urow = row - sign * (AX == 1 ? 1 : ny) - dck * (CX == 1 ? 1 : ny);
      if (act) {
        yv = Yd[g];
        mv = bg_row(rbits, row) ? bg4 : M4[g];
      }
      if (rowin) {
        yu = Yd[u];
        mu = bg_row(rbits, urow) ? bg4 : M4[u];
      }
      // the neighbour lane holds the next four voxels of the same row
      const float prev_w = __shfl_up(yu.w, 1);
      const float next_x = __shfl_down(yu.x, 1);
      const unsigned prev_m = __shfl_up(mu, 1) >> 24;
      const unsigned next_m = __shfl_down(mu, 1) & 0xffu;
      if (!act) continue;
      float su[4] = {yu.x, yu.y, yu.z, yu.w};
      unsigned cu[4] = {mu & 0xffu, (mu >> 8) & 0xffu, (mu >> 16) & 0xffu, mu >> 24};
      bool in[4] = {rowin, rowin, rowin, rowin};
      if (dbk > 0) {
        float w = 0.f;
        unsigned cw = 0;
        const bool have = rowin && q > 0;
        if (have) {
          w = lane > 0 ? prev_w : Ys[4 * u - 1];
          cw = lane > 0 ? prev_m : A.mat[4 * u - 1];
        }
        su[3] = su[2]; su[2] = su[1]; su[1] = su[0]; su[0] = w;
        cu[3] = cu[2]; cu[2] = cu[1]; cu[1] = cu[0]; cu[0] = cw;
        in[0] = have;
      } else if (dbk < 0) {
        float w = 0.f;
        unsigned cw = 0;
        const bool have = rowin && q < tq - 1;
        if (have) {
          w = lane < 63 ? next_x : Ys[4 * u + 4];
          cw = lane < 63 ? next_m : A.mat[4 * u + 4];
        }
        su[0] = su[1]; su[1] = su[2]; su[2] = su[3]; su[3] = w;
        cu[0] = cu[1]; cu[1] = cu[2]; cu[2] = cu[3]; cu[3] = cw;
        in[3] = have;
      }
      const float sv[4] = {yv.x, yv.y, yv.z, yv.w};
      float o[4], mvv[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const unsigned cv = (mv >> (8 * t)) & 0xffu;
        const float fv = nu * srt[cv & 0x7fu];
        bool inj = in[t];
        if (FRESNEL) inj = inj && ((cu[t] ^ cv) & 0x7fu) == 0;
        const float fu = inj ? nu * srt[cu[t] & 0x7fu] : 0.0f;
        o[t] = fmaf(fu, su[t], (1.0f - fv) * sv[t]);
        mvv[t] = fv * sv[t];
      }
      // X is not read again in this step: stream it past the caches
      const f32x4 ov = {o[0], o[1], o[2], o[3]};
      __builtin_nontemporal_store(ov, reinterpret_cast<f32x4*>(Xd + g));
      acc.dom += (double(o[0]) + double(o[1])) + (double(o[2]) + double(o[3]));
      // light that leaves: through the exit plane, then the x sides, then the c sides
      if (last) {
        acc.esc_a += (double(mvv[0]) + double(mvv[1])) + (double(mvv[2]) + double(mvv[3]));
        continue;
      }
      const bool cexit = (unsigned)(pc + dcn) >= (unsigned)nf;
      const bool b1 = dbn > 0 && q == tq - 1, b0 = dbn < 0 && q == 0;
      if (b1) { acc.esc_b1 += double(mvv[3]); mvv[3] = 0.f; }
      if (b0) { acc.esc_b0 += double(mvv[0]); mvv[0] = 0.f; }
      if (cexit) {
        const double t = (double(mvv[0]) + double(mvv[1])) + (double(mvv[2]) + double(mvv[3]));
        if (dcn > 0) acc.esc_c1 += t; else acc.esc_c0 += t;
      } else if (FRESNEL && (mv & 0x80808080u)) {
        // an interface voxel among the four: compare with its downwind voxel
        const int vb = 4 * g;
        const int wofs = sign * 4 * sa4 + dbn + dcn * 4 * sc4;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          if (!((mv >> (8 * t)) & 0x80u)) continue;
          if ((t == 3 && b1) || (t == 0 && b0)) continue;   // left through an x side
          const unsigned cw = A.mat[vb + t + wofs];
          if (((cw ^ (mv >> (8 * t))) & 0x7fu) != 0) {
            A.icptF[size_t(A.islot[vb + t]) * A.ndir + d] = mvv[t];
            acc.dom += double(mvv[t]);
          }
        }
      }
    }
  }
}

// Phase mode, a moving x-dominant direction, in the band order of the split
// paths: a lane's plane, shifts and exit face are fixed, bands of 4 x rpi rows
// across z are walked along y, and the upwind rows a wave reads in pieces
// (they differ lane by lane by a row in y or z) are still in L2 when the
// neighbouring rows' waves read the rest of their cache lines.
template <class Src>
__device__ __forceinline__ void sweep_phase_band0(const SweepArgs& A, const Src& Yd,
                                                  const DevDir& D, int d, int blk, int nblk,
                                                  const int8_t* __restrict__ db,
                                                  const int8_t* __restrict__ dc, SweepAcc& acc) {
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const int nxy = nx * ny;
  float* __restrict__ Xd = A.X + size_t(d) * A.Vp;
  const int tpr = nx < kThreads ? nx : kThreads;
  const int rpi = kThreads / tpr;
  const int xs = threadIdx.x % tpr, rsub = threadIdx.x / tpr;
  if (rsub >= rpi) return;
  const int sign = D.sign;
  constexpr int RB = 4;
  const int TB = RB * rpi;
  const int nb = (nz + TB - 1) / TB;
  const long long T = (long long)nb * ny;
  const int i0 = int(T * blk / nblk), i1 = int(T * (blk + 1) / nblk);
  for (int x = xs; x < nx; x += tpr) {
    const int k = sign > 0 ? x : nx - 1 - x;
    const int dbk = db[k], dck = dc[k], dbn = db[k + 1], dcn = dc[k + 1];
    const bool exit_a = k + 1 >= nx;
    const int uoff = -sign - dbk * nx - dck * nxy;
    for (int i = i0; i < i1; ++i) {
      const int band = i / ny, y = i - band * ny;
      const bool yin = k > 0 && (unsigned)(y - dbk) < (unsigned)ny;
      const bool yexit = (unsigned)(y + dbn) >= (unsigned)ny;
      int v[RB], zz[RB];
      bool live[RB];
      float out[RB];
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        zz[r] = band * TB + rsub + r * rpi;
        live[r] = zz[r] < nz;
        v[r] = (zz[r] * ny + y) * nx + x;
        const bool in = live[r] && yin && (unsigned)(zz[r] - dck) < (unsigned)nz;
        out[r] = in ? Yd[v[r] + uoff] : 0.0f;
      }
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        if (!live[r]) continue;
        Xd[v[r]] = out[r];
        acc.dom += double(out[r]);
        if (exit_a) {
          acc.esc_a += double(Yd[v[r]]);
        } else if (yexit) {
          if (dbn > 0) acc.esc_b1 += double(Yd[v[r]]); else acc.esc_b0 += double(Yd[v[r]]);
        } else if ((unsigned)(zz[r] + dcn) >= (unsigned)nz) {
          if (dcn > 0) acc.esc_c1 += double(Yd[v[r]]); else acc.esc_c0 += double(Yd[v[r]]);
        }
      }
    }
  }
}

// x-dominant: lanes run across planes, so each lane's plane index, shifts and
// exit face are fixed and only the row (y, z) changes.  Bands of 4 x rpi rows
// across z are walked along y, four rows per lane per item with all loads
// issued before the stores.
template <bool FRESNEL>
__device__ __forceinline__ void sweep_split_rows0(const SweepArgs& A, const DevDir& D, int d,
                                                  int blk, int nblk,
                                                  const int8_t* __restrict__ db,
                                                  const int8_t* __restrict__ dc,
                                                  const float* __restrict__ srt,
                                                  const uint32_t* __restrict__ rbits,
                                                  SweepAcc& acc) {
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const int nxy = nx * ny;
  const float* __restrict__ Yd = A.Y + size_t(d) * A.Vp;
  float* __restrict__ Xd = A.X + size_t(d) * A.Vp;
  const uint8_t* __restrict__ M = A.mat;
  const int tpr = nx < kThreads ? nx : kThreads;
  const int rpi = kThreads / tpr;
  const int xs = threadIdx.x % tpr, rsub = threadIdx.x / tpr;
  if (rsub >= rpi) return;
  const int sign = D.sign;
  const float nu = D.nu;
  constexpr int RB = 4;
  const int TB = RB * rpi;
  const int nb = (nz + TB - 1) / TB;
  const long long T = (long long)nb * ny;
  const int i0 = int(T * blk / nblk), i1 = int(T * (blk + 1) / nblk);
  for (int x = xs; x < nx; x += tpr) {
    const int k = sign > 0 ? x : nx - 1 - x;
    const int dbk = db[k], dck = dc[k], dbn = db[k + 1], dcn = dc[k + 1];
    const bool exit_a = k + 1 >= nx;
    const int uoff = -sign - dbk * nx - dck * nxy;
    const int woff = sign + dbn * nx + dcn * nxy;
    for (int i = i0; i < i1; ++i) {
      const int band = i / ny, y = i - band * ny;
      const bool yin = k > 0 && (unsigned)(y - dbk) < (unsigned)ny;
      const bool yexit = (unsigned)(y + dbn) >= (unsigned)ny;
      int v[RB], zz[RB];
      bool live[RB], in[RB];
      float yv[RB], yu[RB];
      unsigned cv[RB], cu[RB];
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        zz[r] = band * TB + rsub + r * rpi;
        live[r] = zz[r] < nz;
        v[r] = (zz[r] * ny + y) * nx + x;
        in[r] = live[r] && yin && (unsigned)(zz[r] - dck) < (unsigned)nz;
        yv[r] = live[r] ? Yd[v[r]] : 0.0f;
        yu[r] = in[r] ? Yd[v[r] + uoff] : 0.0f;
        // class bytes: the background class for rows the bitmap marks
        const int row = zz[r] * ny + y, urow = row - dbk - dck * ny;
        cv[r] = !live[r] ? 0u : (bg_row(rbits, row) ? A.bgcls : M[v[r]]);
        cu[r] = !in[r] ? 0u : (bg_row(rbits, urow) ? A.bgcls : M[v[r] + uoff]);
      }
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        if (!live[r]) continue;
        const float fv = nu * srt[cv[r] & 0x7fu];
        bool inf = in[r];
        if (FRESNEL) inf = inf && ((cu[r] ^ cv[r]) & 0x7fu) == 0;
        const float fu = inf ? nu * srt[cu[r] & 0x7fu] : 0.0f;
        const float out = fmaf(fu, yu[r], (1.0f - fv) * yv[r]);
        __builtin_nontemporal_store(out, Xd + v[r]);
        acc.dom += double(out);
        const float mv = fv * yv[r];
        if (exit_a) {
          acc.esc_a += double(mv);
        } else if (yexit) {
          if (dbn > 0) acc.esc_b1 += double(mv); else acc.esc_b0 += double(mv);
        } else if ((unsigned)(zz[r] + dcn) >= (unsigned)nz) {
          if (dcn > 0) acc.esc_c1 += double(mv); else acc.esc_c0 += double(mv);
        } else if (FRESNEL && (cv[r] & 0x80u)) {
          if (((M[v[r] + woff] ^ cv[r]) & 0x7fu) != 0) {
            A.icptF[size_t(A.islot[v[r]]) * A.ndir + d] = mv;
            acc.dom += double(mv);
          }
        }
      }
    }
  }
}

}  // namespace

// Phase mode, direction d does not move at this step: the collided field of
// rows [rb, re) passes through.
template <class Src>
__device__ __forceinline__ void sweep_still(const SweepArgs& A, const Src& Y, int d, int rb,
                                            int re, SweepAcc& acc) {
  float4* __restrict__ Xd = reinterpret_cast<float4*>(A.X + size_t(d) * A.Vp);
  const long long v0 = (long long)rb * A.nx, v1 = (long long)re * A.nx;
  // whole float4s inside [v0, v1) are copied as vectors, the ragged ends one by one
  const long long q0 = (v0 + 3) / 4, q1 = v1 / 4;
  for (long long q = q0 + threadIdx.x; q < q1; q += kThreads) {
    const float4 y = Y.q4(q);
    Xd[q] = y;
    acc.dom += (double(y.x) + double(y.y)) + (double(y.z) + double(y.w));
  }
  float* Xs = A.X + size_t(d) * A.Vp;
  for (long long v = v0 + threadIdx.x; v < v1; v += kThreads) {
    if (v >= 4 * q0 && v < 4 * q1) continue;
    const float y = Y[v];
    Xs[v] = y;
    acc.dom += double(y);
  }
}

// Every photon of direction d moves one plane: 16-byte rows for y- and
// z-dominant directions on grids with nx a multiple of 4, else rows of single
// voxels, or, x-dominant, lanes across planes in band order.
template <class Src>
__device__ __forceinline__ void sweep_moving(const SweepArgs& A, const Src& Y, const DevDir& D,
                                             int d, int blk, int nblk, int rb, int re,
                                             int8_t (&sdelta)[2][kMaxExt + 2], SweepAcc& acc) {
  if (D.axis != 0 && (A.nx & 3) == 0 && D.unitb) {
    if (D.axis == 2)
      sweep_phase_vec<2>(A, Y, D, d, rb, re, sdelta[0], sdelta[1], acc);
    else
      sweep_phase_vec<1>(A, Y, D, d, rb, re, sdelta[0], sdelta[1], acc);
  } else if (D.axis == 2) {
    sweep_phase_flat<2>(A, Y, D, d, rb, re, sdelta[0], sdelta[1], acc);
  } else if (D.axis == 1) {
    sweep_phase_flat<1>(A, Y, D, d, rb, re, sdelta[0], sdelta[1], acc);
  } else {
    sweep_phase_band0(A, Y, D, d, blk, nblk, sdelta[0], sdelta[1], acc);
  }
}

// The 7 partial sums of block blk of direction d (escape per face scaled by
// esc_scale, light in the box) to A.part[q * ndir * nblk + d * nblk + blk].
__device__ __forceinline__ void store_sweep_partials(const SweepArgs& A, const DevDir& D, int d,
                                                     int blk, int nblk, const SweepAcc& acc,
                                                     double esc_scale = 1.0) {
  double face[6];
  const int fa = 2 * D.axis + (D.sign > 0 ? 1 : 0);
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    double s = 0;
    if (f == fa) s += acc.esc_a;
    if (f == 2 * D.bax) s += acc.esc_b0;
    if (f == 2 * D.bax + 1) s += acc.esc_b1;
    if (f == 2 * D.cax) s += acc.esc_c0;
    if (f == 2 * D.cax + 1) s += acc.esc_c1;
    face[f] = s * esc_scale;
  }
  const double vals[7] = {face[0], face[1], face[2], face[3], face[4], face[5], acc.dom};
  block_sums<7>(vals, A.part + (long long)d * nblk + blk, (long long)A.ndir * nblk);
}

// Block blk of nblk row slabs of direction d; writes the block's 7 partial sums
// (escape per face, light in the box) to A.part[q * ndir * nblk + d * nblk + blk].
// FAST: every direction takes one of the class-byte split paths (x-dominant
// lanes or 16-byte rows); the generic row path is then left out of the kernel,
// which keeps its register count, and so its occupancy, that of the fast paths.
template <bool SPLIT, bool FRESNEL, bool FAST = false>
__device__ __forceinline__ void sweep_block(const SweepArgs& A, int d, int blk, int nblk,
                                            int8_t (&sdelta)[2][kMaxExt + 2],
                                            float* srt = nullptr, uint32_t* rbits = nullptr) {
  const DevDir D = A.dirs[d];
  const int m = *A.step_ctr;
  const float fph = SPLIT ? 1.0f : phase_move(D.nu64, m);
  const int R = A.ny * A.nz;
  const int rb = int((long long)R * blk / nblk);
  const int re = int((long long)R * (blk + 1) / nblk);
  SweepAcc acc;
  if (fph == 0.0f) {
    sweep_still(A, OneField{A.Y + size_t(d) * A.Vp}, d, rb, re, acc);
  } else {
    const int ea = D.axis == 0 ? A.nx : (D.axis == 1 ? A.ny : A.nz);
    for (int i = threadIdx.x; i <= ea; i += kThreads) {
      sdelta[0][i] = A.delta[(size_t(d) * 2 + 0) * A.dstride + i];
      sdelta[1][i] = A.delta[(size_t(d) * 2 + 1) * A.dstride + i];
    }
    const bool vec = D.axis != 0 && (A.nx & 3) == 0 && D.unitb;
    const bool smat = FAST || (SPLIT && A.mat != nullptr && srt != nullptr && rbits != nullptr);
    const bool svec = smat && vec;
    if (smat && threadIdx.x < 128) srt[threadIdx.x] = A.rtab[threadIdx.x];
    if (smat) {
      const int R = A.ny * A.nz;
      const int nw = ((R < kMaxRowBits ? R : kMaxRowBits) + 31) >> 5;
      for (int i = threadIdx.x; i < nw; i += kThreads) rbits[i] = A.rowbits[i];
    }
    __syncthreads();
    if (FAST) {
      if (D.axis == 0)
        sweep_split_rows0<FRESNEL>(A, D, d, blk, nblk, sdelta[0], sdelta[1], srt, rbits, acc);
      else if (D.axis == 2)
        sweep_split_vec<2, FRESNEL>(A, D, d, blk, nblk, sdelta[0], sdelta[1], srt, rbits, acc);
      else
        sweep_split_vec<1, FRESNEL>(A, D, d, blk, nblk, sdelta[0], sdelta[1], srt, rbits, acc);
    } else if (smat && D.axis == 0) {
      sweep_split_rows0<FRESNEL>(A, D, d, blk, nblk, sdelta[0], sdelta[1], srt, rbits, acc);
    } else if (svec) {
      if (D.axis == 2)
        sweep_split_vec<2, FRESNEL>(A, D, d, blk, nblk, sdelta[0], sdelta[1], srt, rbits, acc);
      else
        sweep_split_vec<1, FRESNEL>(A, D, d, blk, nblk, sdelta[0], sdelta[1], srt, rbits, acc);
    } else if (!SPLIT) {
      sweep_moving(A, OneField{A.Y + size_t(d) * A.Vp}, D, d, blk, nblk, rb, re, sdelta, acc);
    } else if (D.axis == 2) {
      sweep_rows<2, SPLIT, FRESNEL>(A, D, d, rb, re, sdelta[0], sdelta[1], acc);
    } else if (D.axis == 1) {
      sweep_rows<1, SPLIT, FRESNEL>(A, D, d, rb, re, sdelta[0], sdelta[1], acc);
    } else {
      sweep_rows<0, SPLIT, FRESNEL>(A, D, d, rb, re, sdelta[0], sdelta[1], acc);
    }
  }
  store_sweep_partials(A, D, d, blk, nblk, acc);
  __syncthreads();   // LDS (shift tables, partial sums) is reused by the next block of work
}

template <bool SPLIT, bool FRESNEL, bool FAST>
__global__ __launch_bounds__(kThreads) void sweep_kernel(SweepArgs A) {
  __shared__ int8_t sdelta[2][kMaxExt + 2];
  __shared__ float srt[128];
  __shared__ uint32_t rbits[SPLIT ? kMaxRowBits / 32 : 1];
  sweep_block<SPLIT, FRESNEL, FAST>(A, blockIdx.y, blockIdx.x, gridDim.x, sdelta, srt, rbits);
}

// The split fast paths held to 64 registers, eight waves per SIMD: at 68-70
// registers (seven waves) the 128^3 x 768 sweep took 3.13 ms, at 64 (a 12-byte
// spill) 2.87 ms.
template <bool FRESNEL>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(8, 8)))
void sweep_fast_kernel(SweepArgs A) {
  __shared__ int8_t sdelta[2][kMaxExt + 2];
  __shared__ float srt[128];
  __shared__ uint32_t rbits[kMaxRowBits / 32];
  sweep_block<true, FRESNEL, true>(A, blockIdx.y, blockIdx.x, gridDim.x, sdelta, srt, rbits);
}

// Retarded stepping below Courant one (Sec. 2.1, the upwind value at the
// retarded time t - dr/c): every direction moves each step, and a voxel takes
// its upwind voxel's collided value at step m + 1 - D_d, blended from two
// history slots.  Light leaving the box crosses the face at its content over
// D_d per step.
// Retarded stepping with a varying refractive index.  The hop from voxel u
// along d lasts D[d][u] = lag + phi steps by u's index class, so each voxel v
// takes the blend of its upwind voxel u at u's own retarded time.  A hop into
// a voxel of another index is intercepted: the light that reached the
// interface goes to A.icptF and the gather returns it as reflected and
// refracted content (Eq. 13-14).  Escape and interception tallies count the
// flux blend / D[d][v]; light in the box counts the content written, plus the
// content the gather will make of the intercepted light (A.icptW).  Voxels of
// a block in flat order, one per thread per pass.
__global__ __launch_bounds__(kThreads) void sweep_retarded_het_kernel(SweepArgs A) {
  __shared__ int8_t sdelta[2][kMaxExt + 2];
  __shared__ int slag[128];
  __shared__ float sphi[128], sinvD[128];
  const int d = blockIdx.y, blk = blockIdx.x, nblk = gridDim.x;
  const DevDir D = A.dirs[d];
  const int m = *A.step_ctr;
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const int ea = D.axis == 0 ? nx : (D.axis == 1 ? ny : nz);
  const int eb = D.bax == 0 ? nx : (D.bax == 1 ? ny : nz);
  const int ec = D.cax == 0 ? nx : (D.cax == 1 ? ny : nz);
  for (int i = threadIdx.x; i <= ea; i += kThreads) {
    sdelta[0][i] = A.delta[(size_t(d) * 2 + 0) * A.dstride + i];
    sdelta[1][i] = A.delta[(size_t(d) * 2 + 1) * A.dstride + i];
  }
  for (int i = threadIdx.x; i < 128; i += kThreads) {
    slag[i] = A.rlagc[d * 128 + i];
    sphi[i] = A.rphic[d * 128 + i];
    sinvD[i] = A.rinvDc[d * 128 + i];
  }
  __syncthreads();
  const long long sa = D.axis == 0 ? 1 : (D.axis == 1 ? nx : (long long)nx * ny);
  const long long sb = D.bax == 0 ? 1 : (D.bax == 1 ? nx : (long long)nx * ny);
  const long long sc = D.cax == 0 ? 1 : (D.cax == 1 ? nx : (long long)nx * ny);
  const float* __restrict__ ring = A.ring;
  float* __restrict__ Xd = A.X + size_t(d) * A.Vp;
  const long long V = A.V;
  const long long vb = V * blk / nblk, ve = V * (blk + 1) / nblk;
  SweepAcc acc;
  for (long long v = vb + threadIdx.x; v < ve; v += kThreads) {
    const int x = int(v % nx), y = int((v / nx) % ny), z = int(v / ((long long)nx * ny));
    const int pa = D.axis == 0 ? x : (D.axis == 1 ? y : z);
    const int pb = D.bax == 0 ? x : (D.bax == 1 ? y : z);
    const int pc = D.cax == 0 ? x : (D.cax == 1 ? y : z);
    const int k = D.sign > 0 ? pa : ea - 1 - pa;
    const int dbk = sdelta[0][k], dck = sdelta[1][k];
    const int dbn = sdelta[0][k + 1], dcn = sdelta[1][k + 1];
    const uint8_t cv = A.mat[v];
    // inflow from the upwind voxel, unless that hop is intercepted
    float out = 0.0f;
    const int ub = pb - dbk, uc = pc - dck;
    if (k > 0 && (unsigned)ub < (unsigned)eb && (unsigned)uc < (unsigned)ec) {
      const long long u = v - D.sign * sa - dbk * sb - dck * sc;
      const uint8_t cu = A.mat[u];
      if (!((cu & 0x80) && A.nvox[u] != A.nvox[v])) {
        const int c = cu & 0x7f;
        out = retarded_value(ring, A.H, A.slot, A.Vp, d, m, slag[c], sphi[c], u);
      }
    }
    Xd[v] = out;
    acc.dom += double(out);
    // what leaves this voxel: through a face, or into a voxel of another index
    int e = 0;   // 0 none, 1 a, 2 b0, 3 b1, 4 c0, 5 c1
    if (k + 1 >= ea) e = 1;
    else if ((unsigned)(pb + dbn) >= (unsigned)eb) e = dbn > 0 ? 3 : 2;
    else if ((unsigned)(pc + dcn) >= (unsigned)ec) e = dcn > 0 ? 5 : 4;
    const bool icpt = e == 0 && (cv & 0x80) &&
                      A.nvox[v + D.sign * sa + dbn * sb + dcn * sc] != A.nvox[v];
    if (e != 0 || icpt) {
      const int c = cv & 0x7f;
      const float r = retarded_value(ring, A.H, A.slot, A.Vp, d, m, slag[c], sphi[c], v);
      const double fl = double(r * sinvD[c]);
      switch (e) {
        case 1: acc.esc_a += fl; break;
        case 2: acc.esc_b0 += fl; break;
        case 3: acc.esc_b1 += fl; break;
        case 4: acc.esc_c0 += fl; break;
        case 5: acc.esc_c1 += fl; break;
        default: {
          const size_t sl = size_t(A.islot[v]) * A.ndir + d;
          A.icptF[sl] = r;
          acc.dom += double(r * A.icptW[sl]);
        }
      }
    }
  }
  store_sweep_partials(A, D, d, blk, nblk, acc, 1.0);
}

__global__ __launch_bounds__(kThreads) void sweep_retarded_kernel(SweepArgs A) {
  __shared__ int8_t sdelta[2][kMaxExt + 2];
  const int d = blockIdx.y, blk = blockIdx.x, nblk = gridDim.x;
  const DevDir D = A.dirs[d];
  const int m = *A.step_ctr;
  const int ea = D.axis == 0 ? A.nx : (D.axis == 1 ? A.ny : A.nz);
  for (int i = threadIdx.x; i <= ea; i += kThreads) {
    sdelta[0][i] = A.delta[(size_t(d) * 2 + 0) * A.dstride + i];
    sdelta[1][i] = A.delta[(size_t(d) * 2 + 1) * A.dstride + i];
  }
  __syncthreads();
  const int R = A.ny * A.nz;
  const int rb = int((long long)R * blk / nblk);
  const int re = int((long long)R * (blk + 1) / nblk);
  SweepAcc acc;
  sweep_moving(A, retarded_rows(A.ring, A.H, A.slot, A.Vp, D, d, m), D, d, blk, nblk, rb, re,
               sdelta, acc);
  store_sweep_partials(A, D, d, blk, nblk, acc, double(D.rinvD));
}

// Two-level angular grid, phase mode: the sweep of fine direction d reads the
// collided value a X + T[parent(d)] share of the field of this step's parity
// and writes the other field, so the collided field is never stored.  Blocks
// take the directions in the order dorder, the children of each coarse bin
// together, so that a row of T is read from HBM about once.
__global__ __launch_bounds__(kThreads) void sweep_twolevel_kernel(SweepArgs A) {
  __shared__ int8_t sdelta[2][kMaxExt + 2];
  int d, blk, nblk;
  if (A.tlbpd > 0) {
    // XCD-ordered: id L runs on XCD L mod 8; on it, for each coarse bin, each
    // of the XCD's row blocks takes the bin's children in turn
    const int L = int(blockIdx.x), xcd = L & 7, j = L >> 3;
    const int nbx = A.tlbpd >> 3;
    const int per_bin = nbx * A.tlnk;
    const int J = j / per_bin, rem = j - J * per_bin;
    const int kb = rem / A.tlnk, c = rem - kb * A.tlnk;
    d = A.dorder[J * A.tlnk + c];
    blk = xcd + 8 * kb;
    nblk = A.tlbpd;
  } else {
    d = A.dorder[blockIdx.y];
    blk = blockIdx.x;
    nblk = gridDim.x;
  }
  const DevDir D = A.dirs[d];
  const int m = *A.step_ctr;
  SweepArgs B = A;
  B.X = (m & 1) ? A.pp0 : A.pp1;
  const TwoLevelRow Y{((m & 1) ? A.pp1 : A.pp0) + size_t(d) * A.Vp,
                      A.tlT + size_t(A.tlparent[d]) * A.Vp, A.tla, A.tlshare};
  const int R = A.ny * A.nz;
  const int rb = int((long long)R * blk / nblk);
  const int re = int((long long)R * (blk + 1) / nblk);
  SweepAcc acc;
  if (phase_move(D.nu64, m) == 0.0f) {
    sweep_still(B, Y, d, rb, re, acc);
  } else {
    const int ea = D.axis == 0 ? A.nx : (D.axis == 1 ? A.ny : A.nz);
    for (int i = threadIdx.x; i <= ea; i += kThreads) {
      sdelta[0][i] = A.delta[(size_t(d) * 2 + 0) * A.dstride + i];
      sdelta[1][i] = A.delta[(size_t(d) * 2 + 1) * A.dstride + i];
    }
    __syncthreads();
    sweep_moving(B, Y, D, d, blk, nblk, rb, re, sdelta, acc);
  }
  store_sweep_partials(A, D, d, blk, nblk, acc);
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

// Per-step tallies.  Workgroup q sums quantity q over the kernels' per-workgroup
// partials in a fixed order (q = 0 absorbed, 1 in the box, 2..7 escape through
// faces 0..5); workgroup 0 also sums the light leaving through each detector
// patch.  The last workgroup to finish writes the budget of step m, checks it
// and advances the step counter.  Deterministic: same inputs, same bits.
// Direction d's share of a detector record at voxel v in step m.
__device__ __forceinline__ double det_term(const ReduceArgs& A, int d, int v, int m) {
  const DevDir D = A.dirs[d];
  if (A.ring && A.rlagc) {
    // varying index: the voxel's class fixes its hop's steps, fraction and 1/D
    const int k = d * 128 + (A.mat[v] & 0x7f);
    return double(A.rinvDc[k] * retarded_value(A.ring, A.H, A.slot, A.Vp, d, m, A.rlagc[k],
                                               A.rphic[k], v));
  }
  if (A.ring) return double(D.rinvD * retarded_rows(A.ring, A.H, A.slot, A.Vp, D, d, m)[v]);
  if (A.tlT) {
    const float* x = (m & 1) ? A.pp1 : A.pp0;
    const TwoLevelRow Y{x + size_t(d) * A.Vp, A.tlT + size_t(A.tlparent[d]) * A.Vp, A.tla,
                        A.tlshare};
    return double(phase_move(D.nu64, m) * Y[v]);
  }
  // with the moves in the collision, the light that left is in the input
  // field of this step, at the voxel it left from
  const float* Y = A.mvfused ? ((m & 1) ? A.pp1 : A.pp0) : A.Y;
  const float f = A.split ? D.nu * A.r[v] : phase_move(D.nu64, m);
  return double(f * Y[size_t(d) * A.Vp + v]);
}

constexpr int kDetTerms = 2048;

__device__ __forceinline__ void reduce_part(const ReduceArgs& A, int q, int nq) {
  __shared__ double red[kThreads];
  __shared__ bool last;
  const int tid = threadIdx.x;
  const int m = *A.step_ctr;
  const bool ok = m < A.cap;
  const double* src;
  long long n;
  if (q == 0) {
    src = A.cpart;
    n = A.cnwg;
  } else {
    src = A.spart + (long long)(q == 1 ? 6 : q - 2) * A.snwg;
    n = A.snwg;
  }
  // eight loads in flight per thread, summed in a fixed order
  double s = 0;
  for (long long i0 = tid; i0 < n; i0 += 8 * kThreads) {
    double v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const long long i = i0 + (long long)j * kThreads;
      v[j] = i < n ? src[i] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) s += v[j];
  }
  red[tid] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) A.scratch[q] = red[0];
  if (q == 0) {
    // detector k's record is the sum, in pair order, of its pairs' terms; up
    // to kDetTerms pairs the terms are formed one pair per thread first
    __shared__ double term[kDetTerms];
    const int npairs = A.ndet > 0 ? A.det_first[A.ndet] : 0;
    const bool staged = npairs <= kDetTerms;
    if (staged) {
      for (int p = tid; p < npairs; p += kThreads)
        term[p] = det_term(A, A.det_pairs[2 * p + 1], A.det_vox[A.det_pairs[2 * p]], m);
      __syncthreads();
    }
    for (int k = tid; k < A.ndet; k += kThreads) {
      double sd = 0;
      const int v = A.det_vox[k];
      for (int p = A.det_first[k]; p < A.det_first[k + 1]; ++p)
        sd += staged ? term[p] : det_term(A, A.det_pairs[2 * p + 1], v, m);
      if (ok) A.det_steps[size_t(k) * A.cap + m] = sd;
    }
  }
  __threadfence();
  __syncthreads();
  if (tid == 0) last = atomicAdd(A.done, 1) == nq - 1;
  __syncthreads();
  if (!last || tid != 0) return;
  __threadfence();
  double res[8];
  for (int i = 0; i < 8; ++i)
    res[i] = __hip_atomic_load(A.scratch + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (ok) {
    double* b = A.budget + size_t(m) * 9;
    b[1] = res[0];
    b[2] = res[1];
    for (int f = 0; f < 6; ++f) b[3 + f] = res[2 + f];
    bool finite = true;
    for (int i = 0; i < 9; ++i) finite = finite && isfinite(b[i]);
    if (!finite) atomicOr(A.flag, 1);
  } else {
    atomicOr(A.flag, 2);
  }
  *A.done = 0;
  __threadfence();
  *A.step_ctr = m + 1;
}

__global__ __launch_bounds__(kThreads) void reduce_kernel(ReduceArgs A) {
  reduce_part(A, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// Batched server kernels.  Each walks a device-resident work list over all
// live request slots and runs the same per-tile / per-block device code as the
// single-medium kernels, so a request's result does not depend on what else
// is in the batch.  Slots whose request has no steps left are skipped.

__device__ __forceinline__ bool req_running(const ReqDev& r) {
  return r.live && *r.swp.step_ctr < r.nsteps;
}

__global__ void srv_inject_kernel(const ReqDev* R) {
  const ReqDev& r = R[blockIdx.x];
  if (!req_running(r) || r.inj.npairs == 0) return;
  const InjectArgs A = r.inj;
  inject_body(A);
}

// A request with the phase moves in the collision (col.pp set) takes the
// fused path per tile (this step's descriptors for its directions in LDS after
// P); the others store the collided field for the sweep items.
template <int NP>
__global__ __launch_bounds__(512, 1) void srv_collide_kernel(const ReqDev* R, const int2* items,
                                                             const int* counts,
                                                             const float* Prow) {
  extern __shared__ float Ps[];
  int2* sdesc = reinterpret_cast<int2*>(Ps + NP * (NP + 4));
  load_p_lds<NP>(Prow, Ps);
  __syncthreads();
  const int n = counts[0];
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int slot = __builtin_amdgcn_readfirstlane(items[it].x);
    const int tile = __builtin_amdgcn_readfirstlane(items[it].y);
    const ReqDev& r = R[slot];
    if (!req_running(r)) continue;
    const CollideArgs A = r.col;
    double ab = 0.0, tot = 0.0;
    if (A.pp) {
      const int m = *A.step_ctr;
      __syncthreads();   // the previous item's scatter has read the descriptors
      move_descriptors<NP>(A, sdesc, m);
      __syncthreads();
      const MoveStep S = move_step<NP>(A, m);
      CollideArgs B = A;
      B.X = reinterpret_cast<const float*>(reinterpret_cast<const char*>(A.pp) + S.so);
      double dom = 0.0;
      double esc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      floatx16 acc[NP / 32];
      collide_res_acc<NP>(B, Ps, tile, acc, ab, tot);
      move_epilogue<NP>(A, sdesc, S, acc, tile, esc, dom);
      move_sums(A, ab, tot, esc, dom, tile, r.ntiles);
    } else {
      collide_res_tile<NP>(A, Ps, tile, ab, tot);
      block_sums512(ab, tot, A.part + tile, A.part + r.ntiles + tile);
    }
  }
}

__global__ __launch_bounds__(kThreads) void srv_sweep_kernel(const ReqDev* R, const int4* items,
                                                             const int* counts) {
  __shared__ int8_t sdelta[2][kMaxExt + 2];
  const int n = counts[1];
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int slot = __builtin_amdgcn_readfirstlane(items[it].x);
    const int d = __builtin_amdgcn_readfirstlane(items[it].y);
    const int blk = __builtin_amdgcn_readfirstlane(items[it].z);
    const ReqDev& r = R[slot];
    if (!req_running(r)) continue;
    const SweepArgs A = r.swp;
    sweep_block<false, false>(A, d, blk, r.bpd, sdelta);
  }
}

__global__ __launch_bounds__(kThreads) void srv_reduce_kernel(const ReqDev* R) {
  const ReqDev& r = R[blockIdx.y];
  if (!req_running(r)) return;
  const ReduceArgs A = r.red;
  reduce_part(A, blockIdx.x, 8);
}

// ---------------------------------------------------------------------------
// Adjoint of the phase-mode step (transposes of the sweep, the detector
// read-out and the collision), for gradients of a detector loss.

// mu[d][v] = T_m^T lam: the photons of v went to its downwind voxel w (if the
// direction moved at step m and w is inside the box), so v's adjoint is w's.
__global__ __launch_bounds__(kThreads) void adj_sweep_kernel(AdjArgs A, int m) {
  const int d = blockIdx.y;
  const DevDir D = A.dirs[d];
  const float f = phase_move(D.nu64, m);
  const float* __restrict__ L = A.lam + size_t(d) * A.Vp;
  float* __restrict__ M = A.mu + size_t(d) * A.Vp;
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const int ea = pick(D.axis, nx, ny, nz), eb = pick(D.bax, nx, ny, nz), ec = pick(D.cax, nx, ny, nz);
  const long long sxy = (long long)nx * ny;
  const long long sa = D.axis == 0 ? 1 : (D.axis == 1 ? nx : sxy);
  const long long sb = D.bax == 0 ? 1 : (D.bax == 1 ? nx : sxy);
  const long long sc = D.cax == 0 ? 1 : (D.cax == 1 ? nx : sxy);
  const int8_t* db = A.delta + (size_t(d) * 2 + 0) * A.dstride;
  const int8_t* dc = A.delta + (size_t(d) * 2 + 1) * A.dstride;
  // rows (y, z) of this block, x across the threads: one division per row
  const int R = ny * nz;
  const int rb = int((long long)R * blockIdx.x / gridDim.x);
  const int re = int((long long)R * (blockIdx.x + 1) / gridDim.x);
  const int tpr = nx < kThreads ? nx : kThreads;
  const int rpi = kThreads / tpr;
  const int rsub = threadIdx.x / tpr, xs = threadIdx.x - rsub * tpr;
  if (rsub >= rpi) return;
  for (int row = rb + rsub; row < re; row += rpi) {
    const int z = row / ny, y = row - z * ny;
    const long long v0 = (long long)row * nx;
    if (f == 0.0f) {
      for (int x = xs; x < nx; x += tpr) M[v0 + x] = L[v0 + x];
      continue;
    }
    for (int x = xs; x < nx; x += tpr) {
      const int pa = pick(D.axis, x, y, z), pb = pick(D.bax, x, y, z), pc = pick(D.cax, x, y, z);
      const int k = D.sign > 0 ? pa : ea - 1 - pa;
      float out = 0.0f;
      if (k + 1 < ea) {
        const int dbn = db[k + 1], dcn = dc[k + 1];
        if ((unsigned)(pb + dbn) < (unsigned)eb && (unsigned)(pc + dcn) < (unsigned)ec)
          out = L[v0 + x + D.sign * sa + dbn * sb + dcn * sc];
      }
      M[v0 + x] = out;
    }
  }
}

// mu[d][v_k] += f_d(m) seed[k][m] for every (detector k, direction d) pair.
// One pair per thread; two detectors on one voxel and face share (direction,
// voxel) targets, hence the atomic add.
__global__ void adj_detector_kernel(AdjArgs A, int m) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < A.ndet_pairs;
       p += gridDim.x * blockDim.x) {
    const int k = A.det_pairs[2 * p], d = A.det_pairs[2 * p + 1];
    const float f = phase_move(A.dirs[d].nu64, m);
    const int v = A.det_vox[k];
    atomicAdd(A.mu + size_t(d) * A.Vp + v, f * float(A.seed[size_t(k) * A.steps + m]));
  }
}

// Transposed collision on LDS-resident P^T (same tiling as the forward kernel):
// z = P^T mu per voxel, lam_out = a mu + b z, and the voxel's gradient sums.
template <int NP>
__global__ __launch_bounds__(512, 1) void adj_collide_kernel(AdjArgs A, int ntiles) {
  constexpr int NQ = NP / 32;
  constexpr int LDK = NP + 4;
  extern __shared__ float Ps[];
  load_p_lds<NP>(A.PT, Ps);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int hl = lane >> 5, cl = lane & 31;
  const size_t rowbytes = size_t(A.Vp) * sizeof(float);
  const float* __restrict__ Pl = Ps + cl * LDK + 4 * hl;
#pragma unroll 1
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long col = (long long)tile * 256 + wave * 32 + cl;
    const unsigned voff = unsigned(size_t(col) * sizeof(float) + size_t(4 * hl) * rowbytes);
    const char* __restrict__ mb0 = reinterpret_cast<const char*>(A.mu);
    floatx16 acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[q][r] = 0.0f;
    // the rows of chunk c + 1 are loaded while chunk c feeds the MFMAs (the
    // last chunk reloads itself: in bounds, unused); the lane's rows of the
    // forward field x are loaded once, in the accumulator layout, so that
    // dL/da (mu x) is summed as the mu rows arrive and dL/db (z x) in the
    // epilogue without reading x again
    float bcur[16], bnext[16];
    const char* __restrict__ xb0 = reinterpret_cast<const char*>(A.xs);
    floatx16 xr[NQ];
    double ga = 0.0;
#pragma unroll
    for (int s = 0; s < 16; ++s)
      bcur[s] = *reinterpret_cast<const float*>(
          mb0 + size_t(8 * (s >> 2) + (s & 3)) * rowbytes + voff);
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int s = 0; s < 16; ++s)
        xr[q][s] = *reinterpret_cast<const float*>(
            xb0 + size_t(32 * q + 8 * (s >> 2) + (s & 3)) * rowbytes + voff);
#pragma unroll 1
    for (int c = 0; c < NQ; ++c) {
      const int cn = c + 1 < NQ ? c + 1 : c;
#pragma unroll
      for (int s = 0; s < 16; ++s)
        bnext[s] = *reinterpret_cast<const float*>(
            mb0 + size_t(32 * cn + 8 * (s >> 2) + (s & 3)) * rowbytes + voff);
      {
        float fa = 0.0f;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
          if (q == c) {
#pragma unroll
            for (int s = 0; s < 16; ++s) fa = fmaf(bcur[s], xr[q][s], fa);
          }
        ga += double(fa);
      }
#pragma unroll
      for (int s4 = 0; s4 < 16; s4 += 4) {
        const int kk = 32 * c + 8 * (s4 >> 2);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const float4 a4 = *reinterpret_cast<const float4*>(Pl + q * 32 * LDK + kk);
          acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.x, bcur[s4 + 0], acc[q], 0, 0, 0);
          acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.y, bcur[s4 + 1], acc[q], 0, 0, 0);
          acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.z, bcur[s4 + 2], acc[q], 0, 0, 0);
          acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.w, bcur[s4 + 3], acc[q], 0, 0, 0);
        }
      }
#pragma unroll
      for (int s = 0; s < 16; ++s) bcur[s] = bnext[s];
    }
    const float av = A.a[col], bv = A.b[col];
    char* __restrict__ lb0 = reinterpret_cast<char*>(A.lam_out);
    double gb = 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      float fb = 0.0f;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const size_t off = size_t(q * 32 + 8 * (r >> 2) + (r & 3)) * rowbytes + voff;
        const float mu = *reinterpret_cast<const float*>(mb0 + off);
        const float z = acc[q][r];
        *reinterpret_cast<float*>(lb0 + off) = av * mu + bv * z;
        fb = fmaf(z, xr[q][r], fb);
      }
      gb += double(fb);
    }
    ga += __shfl_xor(ga, 32, 64);
    gb += __shfl_xor(gb, 32, 64);
    if (hl == 0 && col < A.V) {
      A.ga[col] += ga;
      A.gb[col] += gb;
    }
  }
}

// Adjoint step m with the moves in its epilogue.  mu_m (the seeds of step m
// included) is half m & 1 of M.pp.  The transposed collision gives
// lam_m = a mu_m + b P^T mu_m and the voxel's gradient sums (as
// adj_collide_kernel), then lam_m goes through the transposed moves of step
// m - 1 into the other half: mu_{m-1}[v] = lam_m[w], w the voxel v's photons
// moved to at step m - 1, or 0 when they left the box.  That map is the
// inverse of the forward moves on the box taken periodically, so it is written
// as the forward scatter along reversed move tables (M.mvtab: for a voxel at
// coordinate p of d's dominant axis, the offset back to the plane the forward
// ray came from; a value that leaves writes a zero to the voxel whose forward
// downwind lies outside).  At m = 0 there is no earlier step and nothing is
// moved.  M.mvdet must be all zero (no detector keeps its value here).
template <int NP>
__global__ __launch_bounds__(512, 1) void adj_collide_move_kernel(AdjArgs A, CollideArgs M,
                                                                  int ntiles, int m) {
  constexpr int NQ = NP / 32;
  constexpr int LDK = NP + 4;
  extern __shared__ float Ps[];
  int2* sdesc = reinterpret_cast<int2*>(Ps + size_t(NP) * LDK);
  load_p_lds<NP>(A.PT, Ps);
  move_descriptors<NP>(M, sdesc, m > 0 ? m - 1 : 0);
  __syncthreads();
  const MoveStep S = move_step<NP>(M, m);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int hl = lane >> 5, cl = lane & 31;
  const size_t rowbytes = size_t(A.Vp) * sizeof(float);
  const float* __restrict__ Pl = Ps + cl * LDK + 4 * hl;
  const char* __restrict__ mb0 = reinterpret_cast<const char*>(M.pp) + S.so;
  const char* __restrict__ xb0 = reinterpret_cast<const char*>(A.xs);
#pragma unroll 1
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long col = (long long)tile * 256 + wave * 32 + cl;
    const unsigned voff = unsigned(size_t(col) * sizeof(float) + size_t(4 * hl) * rowbytes);
    floatx16 acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[q][r] = 0.0f;
    // z = P^T mu: the rows of chunk c + 1 are loaded while chunk c feeds the
    // MFMAs (the last chunk reloads itself: in bounds, unused)
    float bcur[16], bnext[16];
#pragma unroll
    for (int s = 0; s < 16; ++s)
      bcur[s] = *reinterpret_cast<const float*>(
          mb0 + size_t(8 * (s >> 2) + (s & 3)) * rowbytes + voff);
#pragma unroll 1
    for (int c = 0; c < NQ; ++c) {
      const int cn = c + 1 < NQ ? c + 1 : c;
#pragma unroll
      for (int s = 0; s < 16; ++s)
        bnext[s] = *reinterpret_cast<const float*>(
            mb0 + size_t(32 * cn + 8 * (s >> 2) + (s & 3)) * rowbytes + voff);
#pragma unroll
      for (int s4 = 0; s4 < 16; s4 += 4) {
        const int kk = 32 * c + 8 * (s4 >> 2);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const float4 a4 = *reinterpret_cast<const float4*>(Pl + q * 32 * LDK + kk);
          acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.x, bcur[s4 + 0], acc[q], 0, 0, 0);
          acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.y, bcur[s4 + 1], acc[q], 0, 0, 0);
          acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.z, bcur[s4 + 2], acc[q], 0, 0, 0);
          acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4.w, bcur[s4 + 3], acc[q], 0, 0, 0);
        }
      }
#pragma unroll
      for (int s = 0; s < 16; ++s) bcur[s] = bnext[s];
    }
    // the gradient sums mu x and z x, and lam = a mu + b z in place of z,
    // block by block with the next block's mu and x rows in flight
    const float av = A.a[col], bv = A.b[col];
    double ga = 0.0, gb = 0.0;
    float mc[16], xc[16], mn[16], xn[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const size_t off = size_t(8 * (r >> 2) + (r & 3)) * rowbytes + voff;
      mc[r] = *reinterpret_cast<const float*>(mb0 + off);
      xc[r] = *reinterpret_cast<const float*>(xb0 + off);
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      if (q + 1 < NQ) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const size_t off = size_t((q + 1) * 32 + 8 * (r >> 2) + (r & 3)) * rowbytes + voff;
          mn[r] = *reinterpret_cast<const float*>(mb0 + off);
          xn[r] = *reinterpret_cast<const float*>(xb0 + off);
        }
      }
      float fa = 0.0f, fb = 0.0f;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float z = acc[q][r];
        fa = fmaf(mc[r], xc[r], fa);
        fb = fmaf(z, xc[r], fb);
        acc[q][r] = av * mc[r] + bv * z;
      }
      ga += double(fa);
      gb += double(fb);
      if (q + 1 < NQ) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          mc[r] = mn[r];
          xc[r] = xn[r];
        }
      }
    }
    ga += __shfl_xor(ga, 32, 64);
    gb += __shfl_xor(gb, 32, 64);
    if (hl == 0 && col < A.V) {
      A.ga[col] += ga;
      A.gb[col] += gb;
    }
    if (m > 0) {
      double esc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, dom = 0.0;
      move_epilogue<NP>(M, sdesc, S, acc, tile, esc, dom);
    }
  }
}

// The step counter, advanced without the tallies (the adjoint's recompute).
__global__ void advance_step_kernel(int* ctr) {
  if (threadIdx.x == 0) *ctr = *ctr + 1;
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
size_t stream_lds(int bf16split) {
  return bf16split ? 2 * 2 * size_t(MT) * (32 + 8) * sizeof(uint16_t)
                   : 2 * size_t(MT) * (32 + 4) * sizeof(float);
}

template <int MT>
hipError_t launch_collide_mt(const CollideArgs& a, const Field& f, int bf16split, hipStream_t s) {
  const int ntiles = int(f.Vp / 256);
  dim3 grid(unsigned(ntiles * (f.NP / MT)));
  if (bf16split)
    hipLaunchKernelGGL(collide_bf16_stream_kernel<MT>, grid, dim3(512), stream_lds<MT>(1), s, a,
                       ntiles);
  else
    hipLaunchKernelGGL(collide_f32_stream_kernel<MT>, grid, dim3(512), stream_lds<MT>(0), s, a,
                       ntiles);
  return hipGetLastError();
}

template <int MT>
hipError_t prepare_stream_mt(int bf16split) {
  const void* k = bf16split ? reinterpret_cast<const void*>(&collide_bf16_stream_kernel<MT>)
                            : reinterpret_cast<const void*>(&collide_f32_stream_kernel<MT>);
  return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                             int(stream_lds<MT>(bf16split)));
}

int resident_blocks() {
  static int n = 0;
  if (n == 0) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
      cus = 256;
    n = cus;
  }
  return n;
}

template <int NP>
size_t res_lds(int bf16split) {
  return bf16split ? 2 * size_t(NP) * (NP + 8) * sizeof(uint16_t)
                   : size_t(NP) * (NP + 4) * sizeof(float);
}

template <int NP>
hipError_t prepare_res(int bf16split) {
  const void* k = bf16split ? reinterpret_cast<const void*>(&collide_bf16_res_kernel<NP>)
                            : reinterpret_cast<const void*>(&collide_f32_res_kernel<NP>);
  return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                             int(res_lds<NP>(bf16split)));
}

template <int NP>
hipError_t launch_res(const CollideArgs& a, const Field& f, int bf16split, hipStream_t s) {
  const size_t lds = res_lds<NP>(bf16split);
  const int ntiles = int(f.Vp / 256);
  const int nb = ntiles < resident_blocks() ? ntiles : resident_blocks();
  if (bf16split)
    hipLaunchKernelGGL(collide_bf16_res_kernel<NP>, dim3(unsigned(nb)), dim3(512), lds, s, a,
                       ntiles);
  else
    hipLaunchKernelGGL(collide_f32_res_kernel<NP>, dim3(unsigned(nb)), dim3(512), lds, s, a,
                       ntiles);
  return hipGetLastError();
}

bool use_resident(const Field& f, int) {
  return f.NP <= 192;
}

}  // namespace

hipError_t prepare_collide(const Field& f, int bf16split) {
  if (!use_resident(f, bf16split)) {
    switch (collide_mt(f.NP)) {
      case 256: return prepare_stream_mt<256>(bf16split);
      case 224: return prepare_stream_mt<224>(bf16split);
      case 192: return prepare_stream_mt<192>(bf16split);
      case 160: return prepare_stream_mt<160>(bf16split);
      case 128: return prepare_stream_mt<128>(bf16split);
      case 96: return prepare_stream_mt<96>(bf16split);
      case 64: return prepare_stream_mt<64>(bf16split);
      default: return prepare_stream_mt<32>(bf16split);
    }
  }
  switch (f.NP) {
    case 32: return prepare_res<32>(bf16split);
    case 64: return prepare_res<64>(bf16split);
    case 96: return prepare_res<96>(bf16split);
    case 128: return prepare_res<128>(bf16split);
    case 160: return prepare_res<160>(bf16split);
    default: return prepare_res<192>(bf16split);
  }
}

int collide_nwg(const Field& f, int bf16split) {
  if (use_resident(f, bf16split)) {
    const int ntiles = int(f.Vp / 256);
    return ntiles < resident_blocks() ? ntiles : resident_blocks();
  }
  return int(f.Vp / 256) * (f.NP / collide_mt(f.NP));
}

hipError_t launch_collide(const CollideArgs& a, const Field& f, int bf16split, int, hipStream_t s) {
  if (use_resident(f, bf16split)) {
    switch (f.NP) {
      case 32: return launch_res<32>(a, f, bf16split, s);
      case 64: return launch_res<64>(a, f, bf16split, s);
      case 96: return launch_res<96>(a, f, bf16split, s);
      case 128: return launch_res<128>(a, f, bf16split, s);
      case 160: return launch_res<160>(a, f, bf16split, s);
      default: return launch_res<192>(a, f, bf16split, s);
    }
  }
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

namespace {
template <int NP>
const void* move_kernel(int bf16split) {
  return bf16split ? reinterpret_cast<const void*>(&collide_move_kernel<NP, true>)
                   : reinterpret_cast<const void*>(&collide_move_kernel<NP, false>);
}
template <int NP>
size_t move_lds(int bf16split) {
  return res_lds<NP>(bf16split) + size_t(NP) * sizeof(int2);
}
template <int NP>
hipError_t prepare_move_np(int bf16split) {
  return hipFuncSetAttribute(move_kernel<NP>(bf16split),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(move_lds<NP>(bf16split)));
}
template <int NP>
hipError_t launch_move_np(const CollideArgs& a, const InjectArgs& j, const Field& f,
                          int bf16split, hipStream_t s) {
  const int ntiles = int(f.Vp / 256);
  const int nb = ntiles < resident_blocks() ? ntiles : resident_blocks();
  if (bf16split)
    hipLaunchKernelGGL((collide_move_kernel<NP, true>), dim3(unsigned(nb)), dim3(512),
                       move_lds<NP>(bf16split), s, a, j, ntiles);
  else
    hipLaunchKernelGGL((collide_move_kernel<NP, false>), dim3(unsigned(nb)), dim3(512),
                       move_lds<NP>(bf16split), s, a, j, ntiles);
  return hipGetLastError();
}
}  // namespace

// The epilogue addresses both fields through one buffer resource, with 32-bit
// offsets below the drop offset 2^31.
bool use_collide_move(const Field& f) {
  return use_resident(f, 0) && (long long)(2 * f.NP + 32) * f.Vp * 4 < (1LL << 31) && f.nx <= 1023 &&
         f.ny <= 1023 && f.nz <= 1023;
}

hipError_t prepare_collide_move(const Field& f, int bf16split) {
  switch (f.NP) {
    case 32: return prepare_move_np<32>(bf16split);
    case 64: return prepare_move_np<64>(bf16split);
    case 96: return prepare_move_np<96>(bf16split);
    case 128: return prepare_move_np<128>(bf16split);
    case 160: return prepare_move_np<160>(bf16split);
    default: return prepare_move_np<192>(bf16split);
  }
}

hipError_t launch_collide_move(const CollideArgs& a, const InjectArgs& j, const Field& f,
                               int bf16split, hipStream_t s) {
  if (!use_collide_move(f)) return hipErrorInvalidValue;
  switch (f.NP) {
    case 32: return launch_move_np<32>(a, j, f, bf16split, s);
    case 64: return launch_move_np<64>(a, j, f, bf16split, s);
    case 96: return launch_move_np<96>(a, j, f, bf16split, s);
    case 128: return launch_move_np<128>(a, j, f, bf16split, s);
    case 160: return launch_move_np<160>(a, j, f, bf16split, s);
    default: return launch_move_np<192>(a, j, f, bf16split, s);
  }
}

namespace {
template <int NP>
size_t implicit_lds() {
  return (size_t(NP) * (NP + 4) + NP) * sizeof(float);
}
template <int NP>
hipError_t prepare_implicit_np() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&collide_implicit_kernel<NP>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(implicit_lds<NP>()));
}
template <int NP>
hipError_t launch_implicit_np(const CollideArgs& a, const Field& f, hipStream_t s) {
  const int ntiles = int(f.Vp / 256);
  const int nb = ntiles < resident_blocks() ? ntiles : resident_blocks();
  hipLaunchKernelGGL(collide_implicit_kernel<NP>, dim3(unsigned(nb)), dim3(512), implicit_lds<NP>(),
                     s, a, ntiles);
  return hipGetLastError();
}
}  // namespace

namespace {
template <int NP>
size_t hop_lds() {
  return (size_t(NP) * (NP + 4) + 3 * NP) * sizeof(float);
}
template <int NP>
hipError_t prepare_hop_np() {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&collide_hop_kernel<NP, false>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     int(hop_lds<NP>()));
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&collide_hop_kernel<NP, true>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(hop_lds<NP>()));
}
template <int NP>
hipError_t launch_hop_np(const CollideArgs& a, const Field& f, hipStream_t s) {
  const int ntiles = int(f.Vp / 256);
  const int nb = ntiles < resident_blocks() ? ntiles : resident_blocks();
  if (a.flux)
    hipLaunchKernelGGL((collide_hop_kernel<NP, true>), dim3(unsigned(nb)), dim3(512),
                       hop_lds<NP>(), s, a, ntiles);
  else
    hipLaunchKernelGGL((collide_hop_kernel<NP, false>), dim3(unsigned(nb)), dim3(512),
                       hop_lds<NP>(), s, a, ntiles);
  return hipGetLastError();
}
}  // namespace

hipError_t prepare_collide_hop(const Field& f) {
  switch (f.NP) {
    case 32: return prepare_hop_np<32>();
    case 64: return prepare_hop_np<64>();
    case 96: return prepare_hop_np<96>();
    case 128: return prepare_hop_np<128>();
    case 160: return prepare_hop_np<160>();
    case 192: return prepare_hop_np<192>();
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_collide_hop(const CollideArgs& a, const Field& f, hipStream_t s) {
  switch (f.NP) {
    case 32: return launch_hop_np<32>(a, f, s);
    case 64: return launch_hop_np<64>(a, f, s);
    case 96: return launch_hop_np<96>(a, f, s);
    case 128: return launch_hop_np<128>(a, f, s);
    case 160: return launch_hop_np<160>(a, f, s);
    case 192: return launch_hop_np<192>(a, f, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_sweep_twolevel(const SweepArgs& a, const Field& f, int bpd, hipStream_t s) {
  if (a.tlbpd > 0)
    hipLaunchKernelGGL(sweep_twolevel_kernel, dim3(unsigned(bpd) * unsigned(f.ndir)),
                       dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL(sweep_twolevel_kernel, dim3(unsigned(bpd), unsigned(f.ndir)),
                       dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sweep_retarded_het(const SweepArgs& a, const Field& f, int bpd, hipStream_t s) {
  hipLaunchKernelGGL(sweep_retarded_het_kernel, dim3(unsigned(bpd), unsigned(f.ndir)),
                     dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sweep_retarded(const SweepArgs& a, const Field& f, int bpd, hipStream_t s) {
  hipLaunchKernelGGL(sweep_retarded_kernel, dim3(unsigned(bpd), unsigned(f.ndir)),
                     dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t prepare_collide_implicit(const Field& f) {
  switch (f.NP) {
    case 32: return prepare_implicit_np<32>();
    case 64: return prepare_implicit_np<64>();
    case 96: return prepare_implicit_np<96>();
    case 128: return prepare_implicit_np<128>();
    case 160: return prepare_implicit_np<160>();
    case 192: return prepare_implicit_np<192>();
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_collide_implicit(const CollideArgs& a, const Field& f, hipStream_t s) {
  switch (f.NP) {
    case 32: return launch_implicit_np<32>(a, f, s);
    case 64: return launch_implicit_np<64>(a, f, s);
    case 96: return launch_implicit_np<96>(a, f, s);
    case 128: return launch_implicit_np<128>(a, f, s);
    case 160: return launch_implicit_np<160>(a, f, s);
    case 192: return launch_implicit_np<192>(a, f, s);
    default: return hipErrorInvalidValue;
  }
}

int sweep_blocks_per_dir(const Field& f, int retarded) {
  // about 6144 voxels (24 per thread) or more per workgroup, at least one row,
  // and no more than about 32768 workgroups in all (each leaves 7 partial
  // sums): enough rounds of resident workgroups that the last, partly filled
  // round costs little.  The retarded sweep, which reads two history slots
  // per direction, takes up to 98304: with more, shorter workgroups per
  // direction the resident ones cover fewer directions at once, which on
  // 101^3 voxels x 3072 directions took the sweep from 11.9 to 9.6 ms (with
  // its streaming stores)
  long long b = f.V / 6144;
  const long long rows = (long long)f.ny * f.nz;
  const long long most = retarded ? 98304 : 32768;
  const long long cap = most / f.ndir > 1 ? most / f.ndir : 1;
  if (b > cap) b = cap;
  if (b > rows) b = rows;
  return int(b < 1 ? 1 : b);
}

hipError_t launch_sweep(const SweepArgs& a, const Field& f, int split, int fresnel, int bpd,
                        hipStream_t s, int fast_split_ok) {
  dim3 grid(unsigned(bpd), unsigned(f.ndir));
  // split mode: fast kernel when every direction has a class-byte path
  const bool fast = split && a.mat != nullptr && fast_split_ok;
  if (split && fresnel && fast)
    hipLaunchKernelGGL((sweep_fast_kernel<true>), grid, dim3(kThreads), 0, s, a);
  else if (split && fresnel)
    hipLaunchKernelGGL((sweep_kernel<true, true, false>), grid, dim3(kThreads), 0, s, a);
  else if (split && fast)
    hipLaunchKernelGGL((sweep_fast_kernel<false>), grid, dim3(kThreads), 0, s, a);
  else if (split)
    hipLaunchKernelGGL((sweep_kernel<true, false, false>), grid, dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL((sweep_kernel<false, false, false>), grid, dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gather(const GatherArgs& a, hipStream_t s) {
  if (a.ntgt == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_kernel, dim3(unsigned((a.ntgt + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(reduce_kernel, dim3(8), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

namespace {
template <int NP>
hipError_t prepare_srv() {
  const size_t lds = size_t(NP) * (NP + 4) * sizeof(float) + size_t(NP) * sizeof(int2);
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&srv_collide_kernel<NP>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
}

template <int NP>
hipError_t launch_srv_collide(const ReqDev* reqs, const int* citems, const int* counts,
                              const float* Prow, hipStream_t s) {
  const size_t lds = size_t(NP) * (NP + 4) * sizeof(float) + size_t(NP) * sizeof(int2);
  hipLaunchKernelGGL(srv_collide_kernel<NP>, dim3(unsigned(resident_blocks())), dim3(512), lds, s,
                     reqs, reinterpret_cast<const int2*>(citems), counts, Prow);
  return hipGetLastError();
}
}  // namespace

hipError_t prepare_server(int NP) {
  switch (NP) {
    case 32: return prepare_srv<32>();
    case 64: return prepare_srv<64>();
    case 96: return prepare_srv<96>();
    case 128: return prepare_srv<128>();
    case 160: return prepare_srv<160>();
    case 192: return prepare_srv<192>();
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_server_step(const ReqDev* reqs, int nslots, const int* citems,
                              const int* sitems, const int* counts, const float* Prow, int NP,
                              hipStream_t s) {
  hipLaunchKernelGGL(srv_inject_kernel, dim3(unsigned(nslots)), dim3(64), 0, s, reqs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (NP) {
    case 32: e = launch_srv_collide<32>(reqs, citems, counts, Prow, s); break;
    case 64: e = launch_srv_collide<64>(reqs, citems, counts, Prow, s); break;
    case 96: e = launch_srv_collide<96>(reqs, citems, counts, Prow, s); break;
    case 128: e = launch_srv_collide<128>(reqs, citems, counts, Prow, s); break;
    case 160: e = launch_srv_collide<160>(reqs, citems, counts, Prow, s); break;
    case 192: e = launch_srv_collide<192>(reqs, citems, counts, Prow, s); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(srv_sweep_kernel, dim3(unsigned(4 * resident_blocks())), dim3(kThreads), 0, s,
                     reqs, reinterpret_cast<const int4*>(sitems), counts);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(srv_reduce_kernel, dim3(8, unsigned(nslots)), dim3(kThreads), 0, s, reqs);
  return hipGetLastError();
}

namespace {
template <int NP>
hipError_t prepare_adj() {
  const size_t lds = size_t(NP) * (NP + 4) * sizeof(float);
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&adj_collide_kernel<NP>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
}
template <int NP>
hipError_t launch_adj_collide(const AdjArgs& a, hipStream_t s) {
  const size_t lds = size_t(NP) * (NP + 4) * sizeof(float);
  const int ntiles = int(a.Vp / 256);
  const int nb = ntiles < resident_blocks() ? ntiles : resident_blocks();
  hipLaunchKernelGGL(adj_collide_kernel<NP>, dim3(unsigned(nb)), dim3(512), lds, s, a, ntiles);
  return hipGetLastError();
}
}  // namespace

namespace {
template <int NP>
size_t adj_move_lds() {
  return size_t(NP) * (NP + 4) * sizeof(float) + size_t(NP) * sizeof(int2);
}
template <int NP>
hipError_t prepare_adj_move() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&adj_collide_move_kernel<NP>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(adj_move_lds<NP>()));
}
template <int NP>
hipError_t launch_adj_move_np(const AdjArgs& a, const CollideArgs& mv, int m, hipStream_t s) {
  const int ntiles = int(a.Vp / 256);
  const int nb = ntiles < resident_blocks() ? ntiles : resident_blocks();
  hipLaunchKernelGGL(adj_collide_move_kernel<NP>, dim3(unsigned(nb)), dim3(512),
                     adj_move_lds<NP>(), s, a, mv, ntiles, m);
  return hipGetLastError();
}
}  // namespace

hipError_t prepare_adjoint_move(int NP) {
  switch (NP) {
    case 32: return prepare_adj_move<32>();
    case 64: return prepare_adj_move<64>();
    case 96: return prepare_adj_move<96>();
    case 128: return prepare_adj_move<128>();
    case 160: return prepare_adj_move<160>();
    case 192: return prepare_adj_move<192>();
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_adjoint_move_step(const AdjArgs& a, const CollideArgs& mv, int m,
                                    hipStream_t s) {
  hipError_t e;
  switch (a.NP) {
    case 32: e = launch_adj_move_np<32>(a, mv, m, s); break;
    case 64: e = launch_adj_move_np<64>(a, mv, m, s); break;
    case 96: e = launch_adj_move_np<96>(a, mv, m, s); break;
    case 128: e = launch_adj_move_np<128>(a, mv, m, s); break;
    case 160: e = launch_adj_move_np<160>(a, mv, m, s); break;
    case 192: e = launch_adj_move_np<192>(a, mv, m, s); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess || m == 0 || a.ndet_pairs == 0) return e;
  // the seeds of step m - 1 into mu_{m-1}
  AdjArgs d = a;
  d.mu = mv.pp + ((m - 1) & 1) * size_t(a.NP) * size_t(a.Vp);
  hipLaunchKernelGGL(adj_detector_kernel, dim3(unsigned((a.ndet_pairs + 255) / 256)), dim3(256),
                     0, s, d, m - 1);
  return hipGetLastError();
}

hipError_t launch_adjoint_seeds(const AdjArgs& a, int m, hipStream_t s) {
  if (a.ndet_pairs == 0) return hipSuccess;
  hipLaunchKernelGGL(adj_detector_kernel, dim3(unsigned((a.ndet_pairs + 255) / 256)), dim3(256),
                     0, s, a, m);
  return hipGetLastError();
}

hipError_t launch_advance_step(int* ctr, hipStream_t s) {
  hipLaunchKernelGGL(advance_step_kernel, dim3(1), dim3(64), 0, s, ctr);
  return hipGetLastError();
}

hipError_t prepare_adjoint(int NP) {
  switch (NP) {
    case 32: return prepare_adj<32>();
    case 64: return prepare_adj<64>();
    case 96: return prepare_adj<96>();
    case 128: return prepare_adj<128>();
    case 160: return prepare_adj<160>();
    case 192: return prepare_adj<192>();
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_adjoint_step(const AdjArgs& a, int m, hipStream_t s) {
  const int bpd = (a.V + kThreads * 16 - 1) / (kThreads * 16);
  hipLaunchKernelGGL(adj_sweep_kernel, dim3(unsigned(bpd < 64 ? bpd : 64), unsigned(a.ndir)),
                     dim3(kThreads), 0, s, a, m);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.ndet_pairs > 0) {
    hipLaunchKernelGGL(adj_detector_kernel, dim3(unsigned((a.ndet_pairs + 255) / 256)),
                       dim3(256), 0, s, a, m);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  switch (a.NP) {
    case 32: return launch_adj_collide<32>(a, s);
    case 64: return launch_adj_collide<64>(a, s);
    case 96: return launch_adj_collide<96>(a, s);
    case 128: return launch_adj_collide<128>(a, s);
    case 160: return launch_adj_collide<160>(a, s);
    case 192: return launch_adj_collide<192>(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_energy(const float* X, long long Vp, int ndir, int V, float* E, hipStream_t s) {
  hipLaunchKernelGGL(energy_kernel, dim3(unsigned((V + 255) / 256)), dim3(256), 0, s, X, Vp, ndir,
                     V, E);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Workspace of the allocation-free step: the per-workgroup FP64 partial sums
// of the collision and transport kernels, the tally kernel's per-step sums and
// its finished-workgroup counter, in one file-scope device array.  Each GPU
// the library runs on holds its own copy for the life of the process; host
// code reaches it only through the address hipGetSymbolAddress returns on that
// device (the array's name is a host-side stand-in, not a device address).
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_address(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

namespace {
__global__ void zero_fill_kernel(double* p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = 0.0;
}
}  // namespace

hipError_t launch_zero_fill(double* p, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long long blocks = (n + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(zero_fill_kernel, dim3(unsigned(blocks < 1024 ? blocks : 1024)),
                     dim3(kThreads), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace trinity
