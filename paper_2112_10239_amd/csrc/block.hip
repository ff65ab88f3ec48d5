// A dense five-qubit block (a 32 x 32 complex unitary, e.g. several layers of
// gates on five qubits fused into one matrix) applied to qubits 0..4 of a
// complex64 state, on the matrix cores or on the vector ALUs.  Measurement
// kernels: they settle whether fused dense blocks on MFMA would beat the
// factored single-qubit rotations of the pass kernel (they do not: a dense
// block costs 256 flops per amplitude, a stage of four factored rotations 12
// VALU instructions).
//
// With the state as a matrix Psi of 2^(n-5) rows of 32 amplitudes (the five
// low index bits vary along a row), the block is Psi <- Psi U^T.  In real
// form, a row is psi64 = [Re psi_0..31, Im psi_0..31] and psi64 <- psi64 W with
// the 64 x 64 real matrix W = [[Re U^T, Im U^T], [-Im U^T, Re U^T]].
#include "kernels.h"

namespace qsim {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));

// One wave per 32 rows (1024 amplitudes): OUT (32 x 64) = PSI (32 x 64) W with
// v_mfma_f32_32x32x2f32 (A 32 x 2: lane l holds A[l % 32][l / 32]; B 2 x 32:
// lane l holds B[l / 32][l % 32]; D 32 x 32: lane l, element v holds
// D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32]).  The K dimension (64) is taken in
// 32 steps of 2; step s gives lane group g = l / 32 the real-form column
// krow(s, g) = g 16 + s (s < 16, real parts) or 32 + g 16 + s - 16 (imaginary
// parts), so each lane reads 16 contiguous amplitudes of its row.  wb holds W
// in B order: wb[(t 32 + s) 64 + l] = W[krow(s, l / 32)][t 32 + l % 32] for the
// real (t = 0) and imaginary (t = 1) output halves.
__global__ __launch_bounds__(256) void k_block5_mfma(float2* __restrict__ psi, const float* __restrict__ wb,
                                                    int64_t rows) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t row0 = wave * 32;
  if (row0 >= rows) return;  // rows is a multiple of 32: whole waves only
  const int g = lane >> 5, r = lane & 31;
  float b[2][32];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int s = 0; s < 32; ++s) b[t][s] = wb[(t * 32 + s) * 64 + lane];
  float2* rowp = psi + ((row0 + r) << 5) + g * 16;
  float2 a[16];
#pragma unroll
  for (int k = 0; k < 16; k += 2) {
    const float4 v = *reinterpret_cast<const float4*>(rowp + k);
    a[k] = make_float2(v.x, v.y);
    a[k + 1] = make_float2(v.z, v.w);
  }
  f32x16 acc0 = {0}, acc1 = {0};
#pragma unroll
  for (int s = 0; s < 32; ++s) {
    const float av = s < 16 ? a[s].x : a[s - 16].y;
    acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(av, b[0][s], acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(av, b[1][s], acc1, 0, 0, 0);
  }
  // every lane of the wave has read its rows (the MFMA operands) before any store
  float2* out = psi + (row0 << 5) + r;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int i = 8 * (v >> 2) + 4 * g + (v & 3);
    out[(int64_t)i << 5] = make_float2(acc0[v], acc1[v]);
  }
}

// The same block on the vector ALUs: one thread per row, the row's 32
// amplitudes in registers, U (complex, row-major) through scalar loads.
__global__ __launch_bounds__(256) void k_block5_valu(float2* __restrict__ psi, const float* __restrict__ u,
                                                    int64_t rows) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= rows) return;
  float2* rowp = psi + (row << 5);
  float2 x[32];
#pragma unroll
  for (int k = 0; k < 32; k += 2) {
    const float4 v = *reinterpret_cast<const float4*>(rowp + k);
    x[k] = make_float2(v.x, v.y);
    x[k + 1] = make_float2(v.z, v.w);
  }
  // scalar loads: every lane uses the same entries
  const __attribute__((address_space(4))) float* uc = (const __attribute__((address_space(4))) float*)(uintptr_t)u;
#pragma unroll 2
  for (int j = 0; j < 32; j += 2) {
    float y0r = 0, y0i = 0, y1r = 0, y1i = 0;
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      const float ar = uc[(j * 32 + i) * 2], ai = uc[(j * 32 + i) * 2 + 1];
      const float br = uc[((j + 1) * 32 + i) * 2], bi = uc[((j + 1) * 32 + i) * 2 + 1];
      y0r = __builtin_fmaf(ar, x[i].x, y0r);
      y0r = __builtin_fmaf(-ai, x[i].y, y0r);
      y0i = __builtin_fmaf(ar, x[i].y, y0i);
      y0i = __builtin_fmaf(ai, x[i].x, y0i);
      y1r = __builtin_fmaf(br, x[i].x, y1r);
      y1r = __builtin_fmaf(-bi, x[i].y, y1r);
      y1i = __builtin_fmaf(br, x[i].y, y1i);
      y1i = __builtin_fmaf(bi, x[i].x, y1i);
    }
    *reinterpret_cast<float4*>(rowp + j) = make_float4(y0r, y0i, y1r, y1i);
    // the outputs j, j+1 overwrite inputs already held in registers
  }
}

}  // namespace

hipError_t launch_block5(void* psi, int64_t rows, const float* d_w, int method, hipStream_t stream) {
  if (rows <= 0) return hipSuccess;
  if (method == 0) {
    if (rows % 32) return hipErrorInvalidValue;
    const int64_t waves = rows / 32;
    const int64_t blocks = (waves + 3) / 4;
    hipLaunchKernelGGL(k_block5_mfma, dim3((unsigned)blocks), dim3(256), 0, stream, reinterpret_cast<float2*>(psi),
                       d_w, rows);
  } else {
    hipLaunchKernelGGL(k_block5_valu, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, stream,
                       reinterpret_cast<float2*>(psi), d_w, rows);
  }
  return hipGetLastError();
}

}  // namespace qsim
