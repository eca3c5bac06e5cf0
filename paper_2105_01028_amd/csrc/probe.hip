// Matrix-core rate probe: back-to-back independent MFMAs on register operands,
// with no memory traffic inside the loop.  It measures what the two MFMA
// shapes the collision kernels use actually deliver on the GPU at hand (clock
// under load included), the ceiling to set their achieved rates against
// beside the datasheet peaks.
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace trinity {
namespace {

typedef float probe_f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 probe_bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kProbeChains = 8;   // independent accumulators per wavefront

// 512 threads (two wavefronts per SIMD, as in the collision kernels), each
// wavefront issuing kProbeChains independent accumulations per iteration.
// The operands depend on the thread so nothing folds; one float per thread
// is written so nothing is removed.
template <int KIND>
__global__ __launch_bounds__(512, 1) void mfma_probe_kernel(float* out, int iters, float seed) {
  probe_f32x16 acc[kProbeChains];
#pragma unroll
  for (int q = 0; q < kProbeChains; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[q][r] = 0.0f;
  const float a = seed * float(threadIdx.x + 1), b = seed * 0.5f;
  probe_bf16x8 ah, bh;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    ah[j] = static_cast<__bf16>(a + float(j));
    bh[j] = static_cast<__bf16>(b - float(j));
  }
#pragma unroll 1
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int q = 0; q < kProbeChains; ++q) {
      if (KIND == 0)
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[q], 0, 0, 0);
      else
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[q], 0, 0, 0);
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int q = 0; q < kProbeChains; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) s += acc[q][r];
  out[size_t(blockIdx.x) * blockDim.x + threadIdx.x] = s;
}

}  // namespace
}  // namespace trinity

using namespace trinity;

extern "C" tr_status tr_probe_mfma(int kind, int iters, int blocks, double* tflops,
                                   double* ms) {
  if (kind != TR_PROBE_MFMA_F32 && kind != TR_PROBE_MFMA_BF16)
    return fail(TR_EINVAL, "kind must be TR_PROBE_MFMA_F32 or TR_PROBE_MFMA_BF16");
  // bounds that keep a launch to about two minutes at most
  if (iters < 1 || iters > (1 << 20) || blocks < 1 || blocks > (1 << 16))
    return fail(TR_EINVAL, "iters must be in 1..2^20 and blocks in 1..2^16");
  if (!tflops || !ms) return fail(TR_EINVAL, "null output");
  float* out = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&out, size_t(blocks) * 512 * sizeof(float));
  if (e == hipSuccess) e = hipStreamCreate(&st);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  // one launch to warm up, then the timed one
  for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
    if (rep == 1) e = hipEventRecord(e0, st);
    if (e != hipSuccess) break;
    if (kind == TR_PROBE_MFMA_F32)
      hipLaunchKernelGGL(mfma_probe_kernel<0>, dim3(unsigned(blocks)), dim3(512), 0, st, out,
                         iters, 1e-3f);
    else
      hipLaunchKernelGGL(mfma_probe_kernel<1>, dim3(unsigned(blocks)), dim3(512), 0, st, out,
                         iters, 1e-3f);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  if (e1) (void)hipEventDestroy(e1);
  if (e0) (void)hipEventDestroy(e0);
  if (st) (void)hipStreamDestroy(st);
  if (out) (void)hipFree(out);
  if (e != hipSuccess) return fail(TR_EDEVICE, std::string("mfma probe: ") + hipGetErrorString(e));
  // FLOP per MFMA per wavefront: 2 M N K (32 x 32 x 2 FP32, 32 x 32 x 16 bf16)
  const double per = kind == TR_PROBE_MFMA_F32 ? 2.0 * 32 * 32 * 2 : 2.0 * 32 * 32 * 16;
  const double flop = per * kProbeChains * double(iters) * 8.0 * double(blocks);
  *ms = double(t);
  *tflops = t > 0.0f ? flop / (double(t) * 1e-3) / 1e12 : 0.0;
  return TR_OK;
}
