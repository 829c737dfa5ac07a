// Measurement probes: the achievable HBM copy rate and the achievable
// matrix-core rate of this device, timed by the caller, so that roofline
// fractions can be stated against measured ceilings beside the data-sheet
// peaks. They compute nothing of the method.
#include "internal.h"

namespace gfd {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// dst = src, 16-byte vector loads and stores, grid-stride
__global__ __launch_bounds__(256) void k_copy16(const float4 *__restrict__ src,
                                                float4 *__restrict__ dst, int64_t n16) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
  int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    const float4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    dst[i] = a;
    dst[i + stride] = b;
    dst[i + 2 * stride] = c;
    dst[i + 3 * stride] = d;
  }
  for (; i < n16; i += stride) dst[i] = src[i];
}

// iters x 8 independent FP64 MFMA chains per wavefront; one value per lane
// written so that nothing is optimised away
__global__ __launch_bounds__(256) void k_mfma_f64(double *__restrict__ out, int iters, double a) {
  d4 acc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) acc[c] = d4{0.0, 0.0, 0.0, 0.0};
  const double b = a * (1.0 + threadIdx.x * 1e-9);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_mfma_bf16(float *__restrict__ out, int iters, float a) {
  f4 acc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) acc[c] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  bf8 x, y;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    x[e] = static_cast<__bf16>(a);
    y[e] = static_cast<__bf16>(a * (1.0f + threadIdx.x * 1e-3f));
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, acc[c], 0, 0, 0);
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < 8; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x] = s;
}

}  // namespace
}  // namespace gfd

using namespace gfd;

extern "C" {

int gpaw_probe_copy(const void *src, void *dst, int64_t bytes, void *stream) {
  if (!src || !dst || bytes < 0 || bytes % 16 != 0)
    return fail(GPAW_EINVAL, "gpaw_probe_copy: non-NULL buffers and a multiple of 16 bytes");
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 != 0)
    return fail(GPAW_EINVAL, "gpaw_probe_copy: buffers must be 16-byte aligned");
  const int64_t n16 = bytes / 16;
  if (n16 == 0) return GPAW_OK;
  k_copy16<<<4096, 256, 0, static_cast<hipStream_t>(stream)>>>(
      static_cast<const float4 *>(src), static_cast<float4 *>(dst), n16);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? GPAW_OK : hip_fail(e, "gpaw_probe_copy");
}

int gpaw_probe_mfma(int32_t kind, void *out, int32_t workgroups, int32_t iters, void *stream) {
  if (!out || workgroups < 1 || iters < 1 || (kind != 0 && kind != 1))
    return fail(GPAW_EINVAL, "gpaw_probe_mfma: kind 0 (FP64) or 1 (BF16), out, workgroups, iters");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (kind == 0)
    k_mfma_f64<<<workgroups, 256, 0, st>>>(static_cast<double *>(out), iters, 1.0000001);
  else
    k_mfma_bf16<<<workgroups, 256, 0, st>>>(static_cast<float *>(out), iters, 1.0f);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? GPAW_OK : hip_fail(e, "gpaw_probe_mfma");
}

}  // extern "C"
