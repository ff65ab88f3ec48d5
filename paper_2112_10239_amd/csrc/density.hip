// Reduced density matrix of a pure state on the matrix cores.
//
// Viewing the state as a matrix M with rows indexed by the kept qubits (i)
// and columns by the traced-out ones (k), the partial trace is the Hermitian
// product rho = M M^dagger (paper, Sec. 2: a partial trace is a contraction
// of the state tensor with its conjugate over the traced modes).  With
// M = Mr + i Mi:
//   Re rho = Mr Mr^T + Mi Mi^T,   Im rho = Mi Mr^T - Mr Mi^T,
// four real products with a shared reduction over k, run as 16x16x4 MFMA
// steps (fp32 for complex64 states, fp64 for complex128).
//
// Tiling: a workgroup of four waves owns a (32*WB) x (32*WB) output tile of
// the lower triangle (tile row >= tile column); each wave owns a
// (16*WB) x (16*WB) corner of it as WB x WB blocks of 16 x 16, and writes
// each element below the diagonal both at (i, j) and, conjugated, at (j, i)
// (the mirror block transposed through LDS, so both writes are row segments).
// Operands come straight from HBM/L2 (each amplitude of a k-slice is read by
// the tiles of its row and column); the next k-slice is loaded before the
// current one is multiplied.
#include <cmath>

#include "kernels.h"

namespace qsim {
namespace {

template <class T>
struct Mfma;

template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 step(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // result item v of lane group q = l / 16 is row 4 q + v
  static __device__ __forceinline__ int row(int q, int v) { return 4 * q + v; }
};

template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 step(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // the fp64 variant interleaves the rows: item v of lane group q is row 4 v + q
  static __device__ __forceinline__ int row(int q, int v) { return 4 * v + q; }
};

template <class T>
struct Amp2;
template <>
struct Amp2<float> {
  typedef float type __attribute__((ext_vector_type(2)));
};
template <>
struct Amp2<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};

// MFMA 16x16x4 operand/result layout (per lane l of the wave):
//   A operand: element (row l % 16, k l / 16); B operand: (k l / 16, col l % 16);
//   result v = 0..3: element (row Mfma<T>::row(l / 16, v), col l % 16).
template <class T, int WB>
__global__ __launch_bounds__(256) void k_density(const T* __restrict__ psi, int64_t row_stride,
                                                 const int64_t* __restrict__ off_i,
                                                 const int64_t* __restrict__ klo,
                                                 const int64_t* __restrict__ khi, int lo_bits, int N, int64_t K,
                                                 T* __restrict__ rho) {
  using V = typename Mfma<T>::v4;
  using A2 = typename Amp2<T>::type;
  constexpr int TB = 32 * WB;
  // lower-triangular tile t -> (ti, tj), ti >= tj, t = ti (ti + 1) / 2 + tj
  const int64_t t = blockIdx.x;
  int64_t ti = (int64_t)((std::sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  while (ti * (ti + 1) / 2 > t) --ti;
  const int64_t tj = t - ti * (ti + 1) / 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int64_t i0 = ti * TB + (wave >> 1) * 16 * WB, j0 = tj * TB + (wave & 1) * 16 * WB;
  const A2* A = reinterpret_cast<const A2*>(psi) + (int64_t)blockIdx.y * row_stride;
  int64_t oi[WB], oj[WB];
  bool vi[WB], vj[WB];
#pragma unroll
  for (int b = 0; b < WB; ++b) {
    const int64_t i = i0 + 16 * b + r16, j = j0 + 16 * b + r16;
    vi[b] = i < N;
    vj[b] = j < N;
    oi[b] = vi[b] ? off_i[i] : 0;
    oj[b] = vj[b] ? off_i[j] : 0;
  }
  V cr[WB][WB], ci[WB][WB];
#pragma unroll
  for (int a = 0; a < WB; ++a)
#pragma unroll
    for (int b = 0; b < WB; ++b) {
      cr[a][b] = V{0, 0, 0, 0};
      ci[a][b] = V{0, 0, 0, 0};
    }
  const int64_t lomask = ((int64_t)1 << lo_bits) - 1;
  A2 x[WB], y[WB];
  auto fetch = [&](int64_t k0) __attribute__((always_inline)) {
    const int64_t k = k0 + kq;
    const bool vk = k < K;
    const int64_t ok = vk ? klo[k & lomask] + khi[k >> lo_bits] : 0;
#pragma unroll
    for (int b = 0; b < WB; ++b) {
      x[b] = (vk && vi[b]) ? A[ok + oi[b]] : A2{0, 0};
      y[b] = (vk && vj[b]) ? A[ok + oj[b]] : A2{0, 0};
    }
  };
  fetch(0);
  for (int64_t k0 = 0; k0 < K; k0 += 4) {
    A2 xc[WB], yc[WB];
#pragma unroll
    for (int b = 0; b < WB; ++b) {
      xc[b] = x[b];
      yc[b] = y[b];
    }
    if (k0 + 4 < K) fetch(k0 + 4);
#pragma unroll
    for (int a = 0; a < WB; ++a)
#pragma unroll
      for (int b = 0; b < WB; ++b) {
        cr[a][b] = Mfma<T>::step(xc[a].x, yc[b].x, cr[a][b]);
        cr[a][b] = Mfma<T>::step(xc[a].y, yc[b].y, cr[a][b]);
        ci[a][b] = Mfma<T>::step(xc[a].y, yc[b].x, ci[a][b]);
        ci[a][b] = Mfma<T>::step(-xc[a].x, yc[b].y, ci[a][b]);
      }
  }
  // Each pair (i > j) is written from one value, at (i, j) and conjugated at
  // (j, i); the diagonal keeps its real part (its imaginary part is zero up to
  // rounding).  The upper half of a diagonal tile is left to the mirror writes.
  // The mirror writes go through a per-wave 16 x 16 block in LDS (rows padded to
  // 17), so both writes store 16 consecutive entries of a row per 16 lanes.
  __shared__ A2 tb[4][16][17];
  A2* out = reinterpret_cast<A2*>(rho) + (int64_t)blockIdx.y * N * N;
#pragma unroll
  for (int a = 0; a < WB; ++a)
#pragma unroll
    for (int b = 0; b < WB; ++b) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int il = Mfma<T>::row(kq, v);
        const int64_t i = i0 + 16 * a + il, j = j0 + 16 * b + r16;
        if (i < N && j < N && i >= j) {
          if (i == j) out[i * N + i] = A2{cr[a][b][v], T(0)};
          else out[i * N + j] = A2{cr[a][b][v], ci[a][b][v]};
        }
        tb[wave][r16][il] = A2{cr[a][b][v], -ci[a][b][v]};  // (j, i) = conj of (i, j)
      }
      // a wave's LDS operations complete in order: its reads below see its writes
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int jl = (lane >> 4) + 4 * s4, il = lane & 15;
        const int64_t i = i0 + 16 * a + il, j = j0 + 16 * b + jl;
        const A2 val = tb[wave][jl][il];
        if (i < N && j < N && i > j) out[j * N + i] = val;
      }
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // reads done before the next block's writes
    }
}

template <class T, int WB>
hipError_t launch_density_t(const DensityLaunch& L, hipStream_t stream) {
  constexpr int TB = 32 * WB;
  const int64_t nt = (L.N + TB - 1) / TB;
  const int64_t tiles = nt * (nt + 1) / 2;
  hipLaunchKernelGGL((k_density<T, WB>), dim3((unsigned)tiles, (unsigned)L.batch), dim3(256), 0, stream,
                     reinterpret_cast<const T*>(L.psi), L.row_stride, L.off_i, L.klo, L.khi, L.lo_bits, L.N, L.K,
                     reinterpret_cast<T*>(L.rho));
  return hipGetLastError();
}

}  // namespace

hipError_t launch_density(const DensityLaunch& L, hipStream_t stream) {
  if (L.N <= 0 || L.K <= 0 || L.batch <= 0 || L.batch > 65535) return hipErrorInvalidValue;
  if (L.c128) return launch_density_t<double, 2>(L, stream);
  return L.N >= 2048 ? launch_density_t<float, 4>(L, stream) : launch_density_t<float, 2>(L, stream);
}

}  // namespace qsim
