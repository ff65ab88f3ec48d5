// Launch wrappers for the gfx950 kernels (host side).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "qsim_types.h"

namespace qsim {

// Arguments of one dense pass over a batch of states.
struct PassLaunch {
  const PassDesc* d_pass;   // device copy of the pass descriptor
  const PassDesc* h_pass;   // host copy (for n, m, r, flags)
  const StageDesc* d_stages;
  const DevOp* d_ops;
  void* A;                  // psi, [rows][2^n] complex
  void* B;                  // lambda (dual passes) or nullptr
  int64_t row_stride;       // amplitudes per row
  const void* coef;         // [rows][coef_row_stride] scalars
  int64_t coef_row_stride;
  double* meas;             // [rows][n_meas][tiles]
  int n_meas;
  double* grad;             // [rows][n_gslots][tiles]
  int n_gslots;
  int rows;
  int c128;                 // 0: complex64, 1: complex128
  int dual;                 // 0: psi only, 1: psi and lambda
  int prefetch = 1;         // next-tile register prefetch where the variant has one
};

hipError_t launch_pass(const PassLaunch& L, hipStream_t stream);

// One workgroup per cone (or per small circuit); cones[order[b]] for block b.
struct ConeLaunch {
  const ConeDesc* d_cones;
  const int32_t* d_order;
  int n_cones;
  const PassDesc* d_passes;
  const StageDesc* d_stages;
  const DevOp* d_ops;
  void* scratch;            // cone states with more than m qubits
  const void* coef;         // slots of all cones
  double* out;              // [n_out] measurement per cone
  double* grad;             // dual cones: [gradient slots], written by the slot's cone
  int m_max;                // largest tile of any cone pass
  int r;
  int c128;
  int dual;                 // 1: forward, lambda = P psi and adjoint sweep per cone
};

hipError_t launch_cones(const ConeLaunch& L, hipStream_t stream);

// Many requests' passes in one launch; all items share precision, r and dual.
hipError_t launch_pass_multi(const PassItem* d_items, int n_items, int64_t total_tiles, int m_max, int r, int c128,
                             int dual, hipStream_t stream);

// out[row] = add + sum_k part[row * per_row + k], in a fixed order.
hipError_t launch_reduce_rows(const double* part, int rows, int64_t per_row, double add, double* out,
                              hipStream_t stream);
// grad[row * n_params + p] = sum over slots s of p (CSR param_slots) of slot_total[row * n_slots + s].
hipError_t launch_grad_scatter(const double* slot_total, int rows, int n_slots, const int32_t* p_off,
                               const int32_t* p_slots, int n_params, double* grad, hipStream_t stream);

// tval[t] = coef[t] * prod_{k in [off[t], off[t+1])} fval[fac[k]] (in k order).
hipError_t launch_term_products(const double* fval, const int32_t* off, const int32_t* fac, const double* coef, int T,
                                double* tval, hipStream_t stream);

// w[f] = sum over terms t containing factor f (CSR f_off/f_terms) of
// t_coef[t] * prod of fval over t's other factors: d<H>/d<P_f>.
hipError_t launch_factor_weights(const double* fval, const int32_t* f_off, const int32_t* f_terms,
                                 const int32_t* t_off, const int32_t* t_fac, const double* t_coef, int F, double* w,
                                 hipStream_t stream);
// grad[p] = sum over slots s of p (CSR) of w[g_cone[s]] * g[s], in CSR order.
hipError_t launch_weighted_scatter(const double* g, const int32_t* g_cone, const double* w, const int32_t* p_off,
                                   const int32_t* p_slots, int n_params, double* grad, hipStream_t stream);

// Reduced density matrices rho_b = M_b M_b^dagger, M_b[i][k] = psi_b[off_i[i] + off_k(k)]
// with off_k(k) = klo[k & (2^lo_bits - 1)] + khi[k >> lo_bits]; rho row-major [batch][N][N].
struct DensityLaunch {
  const void* psi;          // [batch][row_stride] complex amplitudes
  int64_t row_stride;
  int batch;
  const int64_t* off_i;     // [N] amplitude offsets of the kept-qubit index
  const int64_t* klo;       // [2^lo_bits] offsets of the low traced bits
  const int64_t* khi;       // [K >> lo_bits] offsets of the high traced bits
  int lo_bits;
  int N;                    // 2^m
  int64_t K;                // 2^(n-m)
  void* rho;
  int c128;
};
hipError_t launch_density(const DensityLaunch& L, hipStream_t stream);

// Coefficient rows [rows][row_stride] (scalars of the state's precision) built on
// the device: slot s of row b from the slot table and the gates, with parameters
// theta[b * theta_stride + param] (device float64; may be null without
// parameterised gates).
hipError_t launch_build_coef(const CoefSlot* slots, int nslots, const int32_t* srcs, const CoefGate* gates,
                             const double* theta, int64_t theta_stride, int rows, void* out, int64_t row_stride,
                             int c128, hipStream_t stream);

// A dense 32 x 32 complex block on qubits 0..4 of complex64 states, rows = states *
// 2^(n-5) rows of 32 amplitudes, in place.  method 0: fp32 matrix cores, w = the
// 64 x 64 real form in MFMA operand order (4096 floats; rows a multiple of 32);
// method 1: vector ALUs, w = the complex matrix row-major (2048 floats).
hipError_t launch_block5(void* psi, int64_t rows, const float* w, int method, hipStream_t stream);

// Plain copy of n16 16-byte words (reference HBM stream).
hipError_t launch_copy(const void* src, void* dst, uint64_t n16, hipStream_t stream);

// Dynamic LDS bytes for a pass kernel with tile size 2^m.
size_t pass_lds_bytes(int m, int c128, int dual);
int max_lds_bytes();

}  // namespace qsim
