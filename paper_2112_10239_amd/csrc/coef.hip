// Coefficient rows built on the device from a parameter buffer in device
// memory, so a caller whose parameters live on the GPU (an optimiser step in
// torch, say) never copies them to the host.  One thread per (row, slot)
// computes the slot's 2x2 matrix in fp64 from its source gates (the same
// definitions as the host rows, coefmath.h) and rounds it once into the
// state's precision; a factored group's block and the product-start block are
// written by their first slot from the member slots' matrices.
#include "coefmath.h"
#include "kernels.h"

namespace qsim {
namespace {

__device__ cm::M2 slot_matrix(const CoefSlot* slots, const int32_t* srcs, const CoefGate* gates, const double* th,
                              int s) {
  const CoefSlot sl = slots[s];
  cm::M2 M = cm::eye();
  for (int k = 0; k < sl.src_cnt; ++k) {
    const CoefGate& g = gates[srcs[sl.src_off + k]];
    const double t = (g.param >= 0 && th) ? th[g.param] : g.angle;
    M = cm::mul(cm::gate_m2(g.kind, t, g.mat), M);
  }
  return sl.inverse ? cm::adjoint(M) : M;
}

template <class T>
__global__ __launch_bounds__(256) void k_build_coef(const CoefSlot* __restrict__ slots, int nslots,
                                                    const int32_t* __restrict__ srcs,
                                                    const CoefGate* __restrict__ gates,
                                                    const double* __restrict__ theta, int64_t theta_stride, int rows,
                                                    T* __restrict__ out, int64_t row_stride) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)rows * nslots) return;
  const int64_t row = idx / nslots;
  const int s = (int)(idx % nslots);
  const double* th = theta ? theta + row * theta_stride : nullptr;
  T* o = out + row * row_stride + (int64_t)s * 8;
  const CoefSlot sl = slots[s];
  if (sl.kind == CK_TAB) {
    if (sl.gen != 0) return;
    cm::M2 mm[4];
    int has[4] = {0, 0, 0, 0};
    const int r = sl.q < 4 ? sl.q : 4;
    for (int j = 0; j < r && j < sl.src_cnt; ++j) {
      const int m = srcs[sl.src_off + j];
      if (m >= 0) {
        mm[j] = slot_matrix(slots, srcs, gates, th, m);
        has[j] = 1;
      }
    }
    double blk[cm::kTabScalars];
    cm::tab_block(mm, has, r, blk);
    for (int e = 0; e < cm::kTabScalars; ++e) {
      if (e == 68 || e == 69) cm::put_raw(&o[e], (uint32_t)blk[e]);
      else o[e] = (T)blk[e];
    }
    return;
  }
  if (sl.kind == CK_INITF) {
    if (sl.gen != 0) return;
    const int n = sl.q;
    const int nsc = 8 * ((4 * n + 7) / 8);
    for (int e = 0; e < nsc; ++e) o[e] = 0;
    for (int q = 0; q < n && q < sl.src_cnt; ++q) {
      const int m = srcs[sl.src_off + q];
      cm::C f0 = cm::mk(1), f1 = cm::mk(0);
      if (m >= 0) {
        const cm::M2 M = slot_matrix(slots, srcs, gates, th, m);
        f0 = M.a[0][0];
        f1 = M.a[1][0];
      }
      o[4 * q] = (T)f0.re;
      o[4 * q + 1] = (T)f0.im;
      o[4 * q + 2] = (T)f1.re;
      o[4 * q + 3] = (T)f1.im;
    }
    return;
  }
  const cm::M2 M = slot_matrix(slots, srcs, gates, th, s);
  for (int k = 0; k < 8; ++k) o[k] = 0;
  if (sl.kind == CK_RY) {
    o[0] = (T)M.a[0][0].re;
    o[1] = (T)M.a[1][0].re;
  } else if (sl.kind == CK_PHASE) {
    o[0] = (T)M.a[0][0].re;
    o[1] = (T)M.a[0][0].im;
    o[2] = (T)M.a[1][1].re;
    o[3] = (T)M.a[1][1].im;
  } else {
    o[0] = (T)M.a[0][0].re;
    o[1] = (T)M.a[0][0].im;
    o[2] = (T)M.a[0][1].re;
    o[3] = (T)M.a[0][1].im;
    o[4] = (T)M.a[1][0].re;
    o[5] = (T)M.a[1][0].im;
    o[6] = (T)M.a[1][1].re;
    o[7] = (T)M.a[1][1].im;
  }
}

}  // namespace

hipError_t launch_build_coef(const CoefSlot* slots, int nslots, const int32_t* srcs, const CoefGate* gates,
                             const double* theta, int64_t theta_stride, int rows, void* out, int64_t row_stride,
                             int c128, hipStream_t stream) {
  const int64_t total = (int64_t)rows * nslots;
  if (total == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((total + 255) / 256);
  if (c128)
    hipLaunchKernelGGL(k_build_coef<double>, dim3(blocks), dim3(256), 0, stream, slots, nslots, srcs, gates, theta,
                       theta_stride, rows, reinterpret_cast<double*>(out), row_stride);
  else
    hipLaunchKernelGGL(k_build_coef<float>, dim3(blocks), dim3(256), 0, stream, slots, nslots, srcs, gates, theta,
                       theta_stride, rows, reinterpret_cast<float*>(out), row_stride);
  return hipGetLastError();
}

}  // namespace qsim
