// Probe of the gfx950 matrix instructions the kernels rely on (test
// infrastructure): one wavefront multiplies a 16 x K by a K x 16 tile with
// v_mfma_f32_16x16x4f32 or v_mfma_f64_16x16x4f64, K/4 instructions
// accumulating, and writes the four accumulator registers of every lane as
// they are (out[q * 64 + lane] = register q of lane), so the host can check
// both the values and the register layout.
#include <hip/hip_runtime.h>

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

// A: [16][K] row-major, B: [K][16] row-major, K a multiple of 4 (<= 1024)
__global__ void __launch_bounds__(64) k_probe_f32(const float *A, const float *B, int K,
                                                  float *out) {
  const int lane = threadIdx.x;
  f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < K; k0 += 4) {
    const float a = A[(lane & 15) * K + k0 + (lane >> 4)];
    const float b = B[(k0 + (lane >> 4)) * 16 + (lane & 15)];
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
  }
  for (int q = 0; q < 4; ++q) out[q * 64 + lane] = acc[q];
}

__global__ void __launch_bounds__(64) k_probe_f64(const double *A, const double *B, int K,
                                                  double *out) {
  const int lane = threadIdx.x;
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += 4) {
    const double a = A[(lane & 15) * K + k0 + (lane >> 4)];
    const double b = B[(k0 + (lane >> 4)) * 16 + (lane & 15)];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  for (int q = 0; q < 4; ++q) out[q * 64 + lane] = acc[q];
}

// Device pointers; returns 0 on success, -1 on a bad K, else the HIP error.
extern "C" int mfma_probe_f32(const float *A, const float *B, int K, float *out, void *stream) {
  if (K < 4 || K > 1024 || (K & 3)) return -1;
  hipLaunchKernelGGL(k_probe_f32, dim3(1), dim3(64), 0, (hipStream_t)stream, A, B, K, out);
  return (int)hipGetLastError();
}

extern "C" int mfma_probe_f64(const double *A, const double *B, int K, double *out,
                              void *stream) {
  if (K < 4 || K > 1024 || (K & 3)) return -1;
  hipLaunchKernelGGL(k_probe_f64, dim3(1), dim3(64), 0, (hipStream_t)stream, A, B, K, out);
  return (int)hipGetLastError();
}
