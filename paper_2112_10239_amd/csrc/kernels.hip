// gfx950 kernels: tiled gate passes over a dense state, batched light cones,
// and deterministic reductions.
//
// Gate application is bandwidth-bound for 1- and 2-qubit gates (a few flops
// per 16 bytes moved), so a pass is organised around moving every amplitude
// through HBM exactly once: a workgroup owns a tile of 2^m amplitudes (the
// amplitudes that agree on the n-m non-local index bits), holds it in
// registers (2^r per thread) and in LDS (one exchange per change of register
// bits), applies every op the planner put in the pass, and writes the tile
// back.  The first and the storing stage keep the six lowest index bits in
// the lanes, so each wave moves 512 contiguous bytes per access.  Diagonal
// gates, CNOT controls and measurement signs read any index bit: register
// bits are compile-time per register, thread bits come from the lane's local
// index, tile bits from the tile's base index.
//
// Expectation values (paper, Sec. 1 and Sec. 3) are reduced in the same
// passes: per-thread sums in the state's precision over the thread's
// registers, fp64 across threads, one fp64 partial per tile, then a
// fixed-order cross-tile reduction, so results do not depend on scheduling.
#include <cstdlib>
#include <map>
#include <mutex>
#include <type_traits>

#include "kernels.h"

namespace qsim {
namespace {

template <class T>
struct __attribute__((aligned(2 * sizeof(T)))) cpx {
  T x, y;
};

// One amplitude per lane in a single 8- or 16-byte access.
template <class T>
struct Vec2;
template <>
struct Vec2<float> {
  typedef float type __attribute__((ext_vector_type(2)));
};
template <>
struct Vec2<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};

template <class T>
__device__ __forceinline__ cpx<T> ld_amp(const cpx<T>* p) {
  const typename Vec2<T>::type v = *reinterpret_cast<const typename Vec2<T>::type*>(p);
  cpx<T> r;
  r.x = v.x;
  r.y = v.y;
  return r;
}

template <class T>
__device__ __forceinline__ void st_amp(cpx<T>* p, const cpx<T>& a) {
  typename Vec2<T>::type v;
  v.x = a.x;
  v.y = a.y;
  *reinterpret_cast<typename Vec2<T>::type*>(p) = v;
}

// LDS amplitude slots addressed by their full 32-bit LDS byte address.  The
// pass kernels keep the tile at the start of dynamic LDS and have no static
// LDS (checked at launch), so the tile starts at LDS address 0 and an offset
// below the tile size can be XORed into a slot address.
template <class T>
using lds_vec2 = __attribute__((address_space(3))) typename Vec2<T>::type;

template <class T>
__device__ __forceinline__ cpx<T> ld_lds(uint32_t addr) {
  const typename Vec2<T>::type v = *reinterpret_cast<const lds_vec2<T>*>((size_t)addr);
  cpx<T> r;
  r.x = v.x;
  r.y = v.y;
  return r;
}

template <class T>
__device__ __forceinline__ void st_lds(uint32_t addr, const cpx<T>& a) {
  typename Vec2<T>::type v;
  v.x = a.x;
  v.y = a.y;
  *reinterpret_cast<lds_vec2<T>*>((size_t)addr) = v;
}

template <class T>
__device__ __forceinline__ uint32_t lds_addr(cpx<T>* p) {
  return (uint32_t)(size_t)(__attribute__((address_space(3))) char*)(reinterpret_cast<char*>(p));
}

// Pass, stage and op descriptors and gate coefficients are read-only while a
// kernel runs and the same for every wave of a workgroup.  Reading them through
// the constant address space gives scalar loads, which stay out of the vector
// memory pipeline and do not wait behind the HBM loads of a prefetched tile.
template <class T>
using kptr = const __attribute__((address_space(4))) T*;

template <class T>
__device__ __forceinline__ kptr<T> kc(const T* p) {
  return (kptr<T>)(uintptr_t)p;
}

// Scalar loads are dword-granular: 8- and 16-bit descriptor fields are read
// through their aligned dword.
__device__ __forceinline__ uint32_t kb(kptr<uint8_t> p) {
  const uintptr_t a = (uintptr_t)p;
  return (*(kptr<uint32_t>)(a & ~(uintptr_t)3) >> (8 * (a & 3))) & 0xffu;
}

__device__ __forceinline__ uint32_t kh(kptr<uint16_t> p) {
  const uintptr_t a = (uintptr_t)p;
  return (*(kptr<uint32_t>)(a & ~(uintptr_t)3) >> (8 * (a & 2))) & 0xffffu;
}

// A dword-aligned descriptor array read once as NW scalar dwords; elements are
// then extracted with constant shifts (indices are compile-time in unrolled loops).
template <int NW>
struct KWords {
  uint32_t w[NW];
  __device__ __forceinline__ explicit KWords(const void __attribute__((address_space(4))) * p) {
#pragma unroll
    for (int i = 0; i < NW; ++i) w[i] = *((kptr<uint32_t>)p + i);
  }
  __device__ __forceinline__ uint32_t u8(int k) const { return (w[k >> 2] >> (8 * (k & 3))) & 0xffu; }
  __device__ __forceinline__ uint32_t u16(int k) const { return (w[k >> 1] >> (16 * (k & 1))) & 0xffffu; }
};

template <int N>
using IC = std::integral_constant<int, N>;

template <int R, int J = 0, class F>
__device__ __forceinline__ void for_bit(int j, F&& f) {
  if constexpr (J < R) {
    if (j == J) f(IC<J>{});
    else for_bit<R, J + 1>(j, f);
  }
}

template <int NR, int M = 1, class F>
__device__ __forceinline__ void for_mask(uint32_t mask, F&& f) {
  if constexpr (M < NR) {
    if (mask == (uint32_t)M) f(IC<M>{});
    else for_mask<NR, M + 1>(mask, f);
  }
}

struct BitSel {
  uint32_t kind, idx, val;
};

__device__ __forceinline__ BitSel mkbit(uint32_t kind, uint32_t idx, uint32_t tl, uint64_t base) {
  BitSel b{kind, idx, 0u};
  if (kind == BK_THREAD) b.val = (tl >> idx) & 1u;
  else if (kind == BK_TILE) b.val = (uint32_t)(base >> idx) & 1u;
  return b;
}

__device__ __forceinline__ uint32_t bitv(const BitSel& b, int i) {
  return b.kind == BK_REG ? (((uint32_t)i >> b.idx) & 1u) : b.val;
}

// Value of lane partner(l) under a DPP pattern (rows of 16 lanes; lanes of
// rows outside ROWS get 0).  Patterns used: quad_perm [1,0,3,2] (0xB1) and
// [2,3,0,1] (0x4E), row_half_mirror (0x141), row_mirror (0x140), and the row
// broadcasts of lane 15 (0x142) and lane 31 (0x143).
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ float dpp_f32(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROWS, 0xf, false));
}
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROWS, 0xf, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Sum over the 64 lanes of a wave, returned as a wave-uniform value: within
// rows of 16 lanes by DPP (pairs of lanes, quads, half rows, rows), then lane
// 15 of each row into the next row and lane 31 into the upper half, which
// leaves the total in lane 63.  No LDS traffic and a short dependency chain.
// A fixed order: the result does not depend on scheduling.
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_f32<0xB1>(v);
  v += dpp_f32<0x4E>(v);
  v += dpp_f32<0x141>(v);
  v += dpp_f32<0x140>(v);
  v += dpp_f32<0x142, 0xa>(v);
  v += dpp_f32<0x143, 0xc>(v);
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  v += dpp_f64<0x141>(v);
  v += dpp_f64<0x140>(v);
  v += dpp_f64<0x142, 0xa>(v);
  v += dpp_f64<0x143, 0xc>(v);
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 63);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

template <class T>
__device__ __forceinline__ T sgn(int odd) {
  return odd ? T(-1) : T(1);
}

// ---------------------------------------------------------------------------
// register-level ops
// ---------------------------------------------------------------------------

template <class T, int R, int J>
__device__ __forceinline__ void ap_u(cpx<T>* a, kptr<T> u, const BitSel& c) {
  const T u00r = u[0], u00i = u[1], u01r = u[2], u01i = u[3];
  const T u10r = u[4], u10i = u[5], u11r = u[6], u11i = u[7];
  const bool ctl = c.kind != BK_NONE;
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    if (i & (1 << J)) continue;
    const int i1 = i | (1 << J);
    const cpx<T> x0 = a[i], x1 = a[i1];
    cpx<T> y0, y1;
    y0.x = u00r * x0.x - u00i * x0.y + u01r * x1.x - u01i * x1.y;
    y0.y = u00r * x0.y + u00i * x0.x + u01r * x1.y + u01i * x1.x;
    y1.x = u10r * x0.x - u10i * x0.y + u11r * x1.x - u11i * x1.y;
    y1.y = u10r * x0.y + u10i * x0.x + u11r * x1.y + u11i * x1.x;
    if (ctl) {
      const bool on = bitv(c, i) != 0u;
      a[i] = on ? y0 : x0;
      a[i1] = on ? y1 : x1;
    } else {
      a[i] = y0;
      a[i1] = y1;
    }
  }
}

template <class T, int R, int J>
__device__ __forceinline__ void ap_ry(cpx<T>* a, kptr<T> u, const BitSel& c) {
  const T cs = u[0], sn = u[1];
  const bool ctl = c.kind != BK_NONE;
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    if (i & (1 << J)) continue;
    const int i1 = i | (1 << J);
    const cpx<T> x0 = a[i], x1 = a[i1];
    cpx<T> y0, y1;
    y0.x = cs * x0.x - sn * x1.x;
    y0.y = cs * x0.y - sn * x1.y;
    y1.x = sn * x0.x + cs * x1.x;
    y1.y = sn * x0.y + cs * x1.y;
    if (ctl) {
      const bool on = bitv(c, i) != 0u;
      a[i] = on ? y0 : x0;
      a[i1] = on ? y1 : x1;
    } else {
      a[i] = y0;
      a[i1] = y1;
    }
  }
}

template <class T, int R, int J>
__device__ __forceinline__ void ap_x(cpx<T>* a, const BitSel& c) {
  const bool ctl = c.kind != BK_NONE;
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    if (i & (1 << J)) continue;
    const int i1 = i | (1 << J);
    const cpx<T> x0 = a[i], x1 = a[i1];
    const bool on = !ctl || bitv(c, i) != 0u;
    a[i] = on ? x1 : x0;
    a[i1] = on ? x0 : x1;
  }
}

// Real factor T = [[1, -k], [k, 1]] of a factored rotation on register bit J
// (|k| <= 1; the diagonal factors are in the tables): one multiply-add per
// output component.
template <class T, int R, int J>
__device__ __forceinline__ void ap_tan(cpx<T>* a, T k) {
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    if (i & (1 << J)) continue;
    const int i1 = i | (1 << J);
    const cpx<T> x0 = a[i], x1 = a[i1];
    a[i].x = x0.x - k * x1.x;
    a[i].y = x0.y - k * x1.y;
    a[i1].x = x1.x + k * x0.x;
    a[i1].y = x1.y + k * x0.y;
  }
}

// Diagonal over the register index: a[i] *= d[i] (complex, one per register value).
template <class T, int R>
__device__ __forceinline__ void ap_table(cpx<T>* a, kptr<T> d) {
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    const T dr = d[2 * i], di = d[2 * i + 1];
    const cpx<T> x = a[i];
    a[i].x = dr * x.x - di * x.y;
    a[i].y = dr * x.y + di * x.x;
  }
}

// The same with a real table (imaginary parts zero): one real product per component.
template <class T, int R>
__device__ __forceinline__ void ap_table_real(cpx<T>* a, kptr<T> d) {
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    const T dr = d[2 * i];
    a[i].x = dr * a[i].x;
    a[i].y = dr * a[i].y;
  }
}

template <class T, int R>
__device__ __forceinline__ void ap_phase(cpx<T>* a, kptr<T> d, const BitSel& b) {
  const T d0r = d[0], d0i = d[1], d1r = d[2], d1i = d[3];
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    const bool one = bitv(b, i) != 0u;
    const T dr = one ? d1r : d0r, di = one ? d1i : d0i;
    const cpx<T> x = a[i];
    a[i].x = dr * x.x - di * x.y;
    a[i].y = dr * x.y + di * x.x;
  }
}

template <int R>
__device__ __forceinline__ constexpr uint32_t reg_pattern_all() {
  return R >= 5 ? 0xFFFFFFFFu : ((1u << (1 << R)) - 1u);
}

template <class T, int R>
__device__ __forceinline__ void ap_cz(cpx<T>* a, const BitSel& b1, const BitSel& b2) {
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    const bool neg = (bitv(b1, i) & bitv(b2, i)) != 0u;
    a[i].x = neg ? -a[i].x : a[i].x;
    a[i].y = neg ? -a[i].y : a[i].y;
  }
}

// Register indices i (of 2^R) with bit j set, as a bit mask over i; all of them.
template <int R>
__device__ __forceinline__ uint32_t reg_pattern(uint32_t j) {
  constexpr uint32_t pat[5] = {0xAAAAAAAAu, 0xCCCCCCCCu, 0xF0F0F0F0u, 0xFF00FF00u, 0xFFFF0000u};
  return pat[j] & reg_pattern_all<R>();
}

// a_i *= -1 where bit i of S is set (the sign bits of both components)
template <class T, int R>
__device__ __forceinline__ void ap_signs(cpx<T>* a, uint32_t S) {
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    const bool neg = ((S >> i) & 1u) != 0u;
    a[i].x = neg ? -a[i].x : a[i].x;
    a[i].y = neg ? -a[i].y : a[i].y;
  }
}

// sum_i (-1)^{parity(i & rz)} p_i with p_i = |a_i|^2
template <class T, int R>
__device__ __forceinline__ T meas_zp(const T* p, uint32_t rz) {
  T s = 0;
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) s += sgn<T>(__popc((uint32_t)i & rz) & 1) * p[i];
  return s;
}

// Re( i^ph * (-1)^par * sum_y (-1)^{parity(y & rz)} conj(a_{y^F}) a_y ).  The two
// members of a pair (y, y^F) contribute g z + g' conj(z) with z = conj(a_{y^F}) a_y,
// and g' = g or -g for every pair alike, so each pair costs one real product.
template <class T, int R, int F>
__device__ __forceinline__ double meas_f(const cpx<T>* a, uint32_t rz, uint32_t par, uint32_t ph) {
  const bool same = !(__popc((uint32_t)F & rz) & 1);
  T acc = 0;
  if (same) {
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
      const int k = i ^ F;
      if (i < k) acc += sgn<T>(__popc((uint32_t)i & rz) & 1) * (a[k].x * a[i].x + a[k].y * a[i].y);
    }
  } else {
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
      const int k = i ^ F;
      if (i < k) acc += sgn<T>(__popc((uint32_t)i & rz) & 1) * (a[k].x * a[i].y - a[k].y * a[i].x);
    }
  }
  double vr = same ? 2.0 * (double)acc : 0.0, vi = same ? 0.0 : 2.0 * (double)acc;
  if (par) {
    vr = -vr;
    vi = -vi;
  }
  return ph == 0 ? vr : ph == 1 ? -vi : ph == 2 ? -vr : vi;
}

// b_i += c (-1)^{z(i)} a_i
template <class T, int R>
__device__ __forceinline__ void h_z(const cpx<T>* a, cpx<T>* b, T c, uint32_t rz, uint32_t par) {
  const T cc = par ? -c : c;
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    const T g = cc * sgn<T>(__popc((uint32_t)i & rz) & 1);
    b[i].x += g * a[i].x;
    b[i].y += g * a[i].y;
  }
}

// b_i += c i^ph (-1)^{z(i^F)} a_{i^F}
template <class T, int R, int F>
__device__ __forceinline__ void h_f(const cpx<T>* a, cpx<T>* b, T c, uint32_t rz, uint32_t par, uint32_t ph) {
  const T cc = par ? -c : c;
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    const int k = i ^ F;
    const T g = cc * sgn<T>(__popc((uint32_t)k & rz) & 1);
    const T xr = a[k].x, xi = a[k].y;
    const T pr = ph == 0 ? xr : ph == 1 ? -xi : ph == 2 ? -xr : xi;
    const T pi = ph == 0 ? xi : ph == 1 ? xr : ph == 2 ? -xi : -xr;
    b[i].x += g * pr;
    b[i].y += g * pi;
  }
}

// Im sum_i conj(b_i) (P a)_i for P = X, Y on register bit J, or Z on a bit.
// Probes accumulate as chains of multiply-adds (one per real product).
template <class T>
__device__ __forceinline__ T fma_t(T x, T y, T z) {
  if constexpr (sizeof(T) == 4) return __builtin_fmaf(x, y, z);
  else return __builtin_fma(x, y, z);
}

template <class T, int R, int J>
__device__ __forceinline__ T grad_x(const cpx<T>* a, const cpx<T>* b) {
  T s = 0;
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    const cpx<T> p = a[i ^ (1 << J)];
    s = fma_t<T>(b[i].x, p.y, s);
    s = fma_t<T>(-b[i].y, p.x, s);
  }
  return s;
}

template <class T, int R, int J>
__device__ __forceinline__ T grad_y(const cpx<T>* a, const cpx<T>* b) {
  // (Y a)_i = -i (-1)^{bit_J(i)} a_{i^J};  Im(conj(b) * (-i) * a') = -Re(conj(b) a')
  T s = 0;
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    const cpx<T> p = a[i ^ (1 << J)];
    const T sg = ((i >> J) & 1) ? T(1) : T(-1);
    s = fma_t<T>(sg * b[i].x, p.x, s);
    s = fma_t<T>(sg * b[i].y, p.y, s);
  }
  return s;
}

template <class T, int R>
__device__ __forceinline__ T grad_z(const cpx<T>* a, const cpx<T>* b, const BitSel& bit) {
  T s = 0;
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    const T im = b[i].x * a[i].y - b[i].y * a[i].x;
    s += bitv(bit, i) ? -im : im;
  }
  return s;
}

// ---------------------------------------------------------------------------
// one tile of one pass
// ---------------------------------------------------------------------------

// Workgroup barrier for LDS traffic only: waits for this wave's LDS operations,
// not for its outstanding HBM loads, so a prefetch of the next tile stays in
// flight across the exchanges of the current one.
__device__ __forceinline__ void lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

template <class T, int R, bool DUAL>
struct TileRegs {
  cpx<T> a[1 << R];
  cpx<T> b[DUAL ? (1 << R) : 1];
};

// Physical index bits of the non-local qubits of a pass (uniform, scalar work).
__device__ __forceinline__ uint64_t nonlocal_mask(kptr<PassDesc> P) {
  const int nn = P->n - P->m;
  uint64_t M = 0;
  for (int k = 0; k < nn; ++k) M |= 1ull << kb(&P->npos[k]);
  return M;
}

// The bits of x deposited, lowest first, at the set bits of M.
__device__ __forceinline__ uint64_t deposit(uint64_t x, uint64_t M) {
  uint64_t r = 0;
  for (uint64_t m = M; m && x; m &= m - 1, x >>= 1)
    if (x & 1) r |= m & (~m + 1);
  return r;
}

// Physical index of a tile's first amplitude: the tile number deposited at the
// non-local positions.  Walking tiles by a fixed stride d, the next base is
// ((base | ~M) + deposit(d, M)) & M: the carries skip the local positions.
__device__ __forceinline__ uint64_t next_base(uint64_t base, uint64_t M, uint64_t dstep) {
  return ((base | ~M) + dstep) & M;
}

// Thread-local part of stage S's local index (thread bits deposited into tb).
template <int R>
__device__ __forceinline__ uint32_t thread_local_index(kptr<StageDesc> S, int m, int tid) {
  // tid's bit k is the local index bit tb[k]; bits past the tile are dropped
  const KWords<kMaxLocal / 4> tb(S->tb);
  uint32_t tl = 0;
#pragma unroll
  for (int k = 0; k < kMaxLocal - R; ++k)
    if (k < m - R) tl |= (((uint32_t)tid >> k) & 1u) << tb.u8(k);
  return tl;
}

// Global offsets (physical index bits) of stage S: per-thread part and per-register-bit parts.
template <int R>
__device__ __forceinline__ uint64_t stage_gaddr(kptr<PassDesc> P, kptr<StageDesc> S, int tid, uint64_t base,
                                                uint64_t* gr) {
  const int m = P->m;
  const KWords<kMaxLocal / 4> tp(S->tpos);
  const KWords<2> rp(S->rpos);
  uint64_t gt = base;
#pragma unroll
  for (int k = 0; k < kMaxLocal - R; ++k)
    if (k < m - R) gt |= (uint64_t)((uint32_t)(tid >> k) & 1u) << tp.u8(k);
#pragma unroll
  for (int j = 0; j < R; ++j) gr[j] = 1ull << rp.u8(j);
  return gt;
}

// Global offsets of the stage that stores: through the pass's exit permutation
// (destination offsets of the thread bits, lane bits per lane and wave bits and
// the tile's affine terms uniform, and of the register bits) when it has one.
template <int R>
__device__ __forceinline__ uint64_t store_gaddr(kptr<PassDesc> P, kptr<StageDesc> S, int tid, uint64_t base,
                                                uint64_t* gr) {
  if (P->exit_perm) {
    const int m = P->m;
    const uint32_t wv = __builtin_amdgcn_readfirstlane((uint32_t)tid >> 6);
    uint64_t gl = 0, gu = base;
#pragma unroll
    for (int k = 0; k < kMaxLocal - R; ++k)
      if (k < m - R) {
        const uint64_t c = *((kptr<uint64_t>)&P->xcol[0] + k);
        if (k < 6) gl ^= ((uint32_t)(tid >> k) & 1u) ? c : 0ull;
        else gu ^= ((wv >> (k - 6)) & 1u) ? c : 0ull;
      }
    const int na = P->n_xaff;
    for (int j = 0; j < na; ++j)
      if ((base >> kb(&P->xaff_pos[j])) & 1ull) gu ^= *((kptr<uint64_t>)&P->xaff[0] + j);
#pragma unroll
    for (int j = 0; j < R; ++j) gr[j] = *((kptr<uint64_t>)&P->xreg[0] + j);
    return gl ^ gu;
  }
  return stage_gaddr<R>(P, S, tid, base, gr);
}

// Product start state of a tile (first pass of a plan with leading single-qubit
// gates folded in): prod_q (U_q|0>)_{x_q}.  The factor of the tile's non-local
// bits and the thread's bits is computed out of line (once per tile of the first
// pass only, its registers outside the pass kernel's allocation); the register
// factors are multiplied in by doubling at the call.
template <class T, int R>
__device__ __attribute__((noinline)) cpx<T> init_thread_factor(kptr<PassDesc> P, kptr<StageDesc> S0, uint64_t base,
                                                               kptr<T> f) {
  const int m = P->m;
  const int tid = threadIdx.x;
  T cr = 1, ci = 0;
  const int nn = P->n - m;
  for (int k = 0; k < nn; ++k) {
    const int q = (int)kb(&P->npos[k]);
    const int o = 4 * q + 2 * (int)((base >> q) & 1ull);
    const T fr = f[o], fi = f[o + 1];
    const T xr = cr * fr - ci * fi;
    ci = cr * fi + ci * fr;
    cr = xr;
  }
  const KWords<kMaxLocal / 4> tp(S0->tpos);
#pragma unroll
  for (int k = 0; k < kMaxLocal - R; ++k)
    if (k < m - R) {
      const int q = (int)tp.u8(k);
      const bool one = ((tid >> k) & 1) != 0;
      const T fr = one ? f[4 * q + 2] : f[4 * q], fi = one ? f[4 * q + 3] : f[4 * q + 1];
      const T xr = cr * fr - ci * fi;
      ci = cr * fi + ci * fr;
      cr = xr;
    }
  cpx<T> c;
  c.x = cr;
  c.y = ci;
  return c;
}

// First stage of a tile: load a (and b) from HBM, or generate |0...0>.  Lanes
// past the tile (tiles of fewer than 64 threads' worth of amplitudes) read a
// valid slot of their tile too; tile_run zeroes them.
template <class T, int R, bool DUAL>
__device__ __forceinline__ void tile_load(kptr<PassDesc> P, kptr<StageDesc> S0, const cpx<T>* __restrict__ A,
                                          const cpx<T>* __restrict__ B, uint64_t base, TileRegs<T, R, DUAL>& t,
                                          kptr<T> coef) {
  constexpr int NR = 1 << R;
  const int m = P->m, flags = P->flags;
  const int tid = threadIdx.x;
  const bool ld_a = (flags & PF_LOAD_A) != 0, ld_b = DUAL && (flags & PF_LOAD_B) != 0;
  cpx<T> z;
  z.x = 0;
  z.y = 0;
  if (ld_a || ld_b) {
    uint64_t gr[R];
    uint64_t gt;
    if (P->entry_perm) {
      // registers read from their sources under the inverse of the entry
      // permutation: source offsets XOR over the thread's bits (lane bits per
      // lane, wave bits and the tile's affine terms uniform) and register bits
      const uint32_t wv = __builtin_amdgcn_readfirstlane((uint32_t)tid >> 6);
      uint64_t gl = 0, gu = base;
#pragma unroll
      for (int k = 0; k < kMaxLocal - R; ++k)
        if (k < m - R) {
          const uint64_t c = *((kptr<uint64_t>)&P->ecol[0] + k);
          if (k < 6) gl ^= ((uint32_t)(tid >> k) & 1u) ? c : 0ull;
          else gu ^= ((wv >> (k - 6)) & 1u) ? c : 0ull;
        }
      const int na = P->n_eaff;
      for (int j = 0; j < na; ++j)
        if ((base >> kb(&P->eaff_pos[j])) & 1ull) gu ^= *((kptr<uint64_t>)&P->eaff[0] + j);
      gt = gl ^ gu;
#pragma unroll
      for (int j = 0; j < R; ++j) gr[j] = *((kptr<uint64_t>)&P->ereg[0] + j);
    } else {
      gt = stage_gaddr<R>(P, S0, tid, base, gr);
    }
    auto addr = [&](int i) __attribute__((always_inline)) {
      uint64_t g = gt;
#pragma unroll
      for (int j = 0; j < R; ++j)
        if ((i >> j) & 1) g ^= gr[j];
      return g;
    };
    if (ld_a) {
#pragma unroll
      for (int i = 0; i < NR; ++i) t.a[i] = ld_amp(A + addr(i));
    } else {
#pragma unroll
      for (int i = 0; i < NR; ++i) t.a[i] = z;
    }
    if constexpr (DUAL) {
      if (ld_b) {
#pragma unroll
        for (int i = 0; i < NR; ++i) t.b[i] = ld_amp(B + addr(i));
      } else {
#pragma unroll
        for (int i = 0; i < NR; ++i) t.b[i] = z;
      }
    }
  } else if ((flags & PF_INIT) && P->init_fac) {
    const kptr<T> f = coef + (int64_t)P->init_slot * 8;
    const cpx<T> c = init_thread_factor<T, R>(P, S0, base, f);
    const bool active = tid < (1 << (m - R));
    t.a[0].x = active ? c.x : T(0);
    t.a[0].y = active ? c.y : T(0);
    const KWords<2> rp(S0->rpos);
#pragma unroll
    for (int j = 0; j < R; ++j) {  // register factors by doubling, in place
      const int q = (int)rp.u8(j);
      const T f0r = f[4 * q], f0i = f[4 * q + 1], f1r = f[4 * q + 2], f1i = f[4 * q + 3];
#pragma unroll
      for (int i = 0; i < (1 << j); ++i) {
        const int i1 = i | (1 << j);
        const cpx<T> x = t.a[i];
        t.a[i1].x = x.x * f1r - x.y * f1i;
        t.a[i1].y = x.x * f1i + x.y * f1r;
        t.a[i].x = x.x * f0r - x.y * f0i;
        t.a[i].y = x.x * f0i + x.y * f0r;
      }
    }
    if constexpr (DUAL) {
#pragma unroll
      for (int i = 0; i < NR; ++i) t.b[i] = z;
    }
  } else {
    const bool active = tid < (1 << (m - R));
    const uint32_t tl = thread_local_index<R>(S0, m, tid);
    const KWords<2> rbw(S0->rb);
    uint32_t rl[R];
#pragma unroll
    for (int j = 0; j < R; ++j) rl[j] = 1u << rbw.u8(j);
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      uint32_t o = tl;
#pragma unroll
      for (int j = 0; j < R; ++j)
        if ((i >> j) & 1) o |= rl[j];
      t.a[i] = z;
      if ((flags & PF_INIT) && active && base == 0 && o == 0u) t.a[i].x = T(1);
      if constexpr (DUAL) t.b[i] = z;
    }
  }
}

// Stages of a pass whose LDS lane parts come from a table in LDS (the rest
// compute them from the stage header).
constexpr int kLaneTabStages = 24;

// The lane parts of the LDS byte offsets of the pass's first kLaneTabStages
// stages, for reads and for the writes at the stage's exit: entry 2 (64 k + l)
// is XOR_{b : bit b of lane l} rd_lane[b] << sh of stage s0 + k, entry
// 2 (64 k + l) + 1 the same over wr_lane.  Written by the whole workgroup
// once per launch (the pass is the same for every tile).
template <class T>
__device__ __forceinline__ void fill_lane_table(kptr<PassDesc> P, kptr<StageDesc> SD, uint32_t* ltab) {
  constexpr uint32_t kSh = sizeof(cpx<T>) == 8 ? 3u : 4u;
  const int s0 = P->stage_begin;
  const int nst = min(P->stage_end - s0, kLaneTabStages);
  for (int k = threadIdx.x; k < nst * 64; k += blockDim.x) {
    const kptr<StageDesc> S = SD + s0 + (k >> 6);
    const int l = k & 63;
    uint32_t r = 0, w = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b)
      if ((l >> b) & 1) {
        r ^= S->rd_lane[b];
        w ^= S->wr_lane[b];
      }
    ltab[2 * k] = r << kSh;
    ltab[2 * k + 1] = w << kSh;
  }
  lds_sync();
}

// Byte size of the lane table of a pass with the given stage count.
__host__ __device__ constexpr size_t lane_table_bytes(int stages) {
  return (size_t)(stages < kLaneTabStages ? stages : kLaneTabStages) * 64 * 2 * sizeof(uint32_t);
}

// All stages of a tile whose first-stage registers are loaded: ops, LDS
// exchanges (with exit permutations), the store, and the block's partial sums.
// With LT, the lane parts of the LDS offsets of the first kLaneTabStages stages
// are read from ltab (fill_lane_table).
template <class T, int R, bool DUAL, bool TAIL = false, bool LT = false>
__device__ __forceinline__ double tile_run(kptr<PassDesc> P, kptr<StageDesc> SD, kptr<DevOp> OPS,
                                           cpx<T>* __restrict__ A, cpx<T>* __restrict__ B, kptr<T> coef, uint64_t base,
                                           TileRegs<T, R, DUAL>& t, cpx<T>* lds, double* red, double* gacc,
                                           double* __restrict__ grad_out, int64_t grad_stride, bool grad_add = false,
                                           const uint32_t* ltab = nullptr) {
  constexpr int NR = 1 << R;
  const int m = P->m, flags = P->flags;
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const bool active = tid < (1 << (m - R));
  const int lane = tid & 63, wave = tid >> 6, nwaves = (nthr + 63) >> 6;
  const uint32_t tsize = 1u << m;
  const uint32_t lds0 = lds_addr(lds);
  cpx<T>* a = t.a;
  cpx<T>* b = t.b;
  const int gcount = DUAL ? P->grad_count : 0;
  const int gbegin = DUAL ? P->grad_begin : 0;
  if (DUAL && (flags & PF_GRAD)) {
    for (int k = tid; k < nwaves * gcount; k += nthr) gacc[k] = 0.0;
    lds_sync();
  }
  cpx<T> z;
  z.x = 0;
  z.y = 0;
  if (!active) {
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      a[i] = z;
      if constexpr (DUAL) b[i] = z;
    }
  }
  double acc = 0.0;
  const int s0 = P->stage_begin, s1 = P->stage_end, sst = P->store_stage;
  // a pass that stores in its first stage through a permutation (see below)
  const bool cross = sst == s0 && (P->entry_perm || P->exit_perm);
  constexpr uint32_t kSh = sizeof(cpx<T>) == 8 ? 3u : 4u;  // slot -> byte offset
  const uint32_t wv = __builtin_amdgcn_readfirstlane((uint32_t)tid >> 6);
  uint32_t pend = 0;  // register i holds the amplitude of register index i ^ pend
  bool prev_wl = false;  // the tile's previous exchange kept every amplitude in its wave
  for (int s = s0; s < s1; ++s) {
    kptr<StageDesc> S = SD + s;
    pend = 0;
    // the stage header in one scalar load; the wave parts by the wave's index
    const KWords<16> hd(S);
    const uint32_t rdw = kh(&S->rd_wave[wv]), wrw = kh(&S->wr_wave[wv]);
    const int op_begin = (int)hd.w[0], op_end = (int)hd.w[1];
    const uint32_t n_aff = hd.w[2] >> 16, sflags = hd.w[3];
    // LDS addressing precomputed per stage (swizzled slots, linear over XOR):
    // lane bits per lane, wave bits by the wave's index, register bits uniform
    // (header words: rd_lane 4..6, wr_lane 7..9, rd_reg 10..12, wr_reg 13..15)
    const bool tab = LT && s - s0 < kLaneTabStages;
    const uint32_t* lt = ltab + 2 * ((s - s0) * 64 + lane);
    uint32_t rd_b;  // byte offset of the thread's slot (register index 0)
    if (tab) {
      rd_b = lt[0] ^ (rdw << kSh);
    } else {
      uint32_t rd = rdw;
#pragma unroll
      for (int k = 0; k < 6; ++k) rd ^= ((uint32_t)(tid >> k) & 1u) ? hd.u16(8 + k) : 0u;
      rd_b = rd << kSh;
    }
    uint32_t sb[R];
#pragma unroll
    for (int j = 0; j < R; ++j) sb[j] = hd.u16(20 + j) << kSh;
    auto soff = [&](int i) __attribute__((always_inline)) {
      uint32_t o = 0;
#pragma unroll
      for (int j = 0; j < R; ++j)
        if ((i >> j) & 1) o ^= sb[j];
      return o;
    };
    // full LDS address of the thread's slot (tile at address 0), opaque to the
    // optimiser so each access is one XOR with a uniform offset
    uint32_t tl_b = lds0 + rd_b;
    asm volatile("" : "+v"(tl_b));
    // the thread's local index, for ops that read index bits (controls,
    // diagonals, measurement signs); stages of a factored op alone need none
    const uint32_t tl = (sflags & SF_INDEX_OPS) ? thread_local_index<R>(S, m, tid) : 0u;

    const uint32_t bofs = tsize * (uint32_t)sizeof(cpx<T>);  // second state's tile (dual kernels)
    if (s != s0) {
      // lanes past the tile read valid slots (their local index keeps only tile bits) and are zeroed
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        const uint32_t l = tl_b ^ soff(i);
        a[i] = ld_lds<T>(l);
        if constexpr (DUAL) b[i] = ld_lds<T>(l + bofs);
      }
      if (!active) {
#pragma unroll
        for (int i = 0; i < NR; ++i) {
          a[i] = z;
          if constexpr (DUAL) b[i] = z;
        }
      }
    }

    // Rotations U_j = X^f P_j T_j E_j on every register bit (the last op of its
    // stage; the E table, when needed, is an OP_DTAB just before): each real T_j,
    // the P table; the swaps X^f stay pending as an XOR mask on the register
    // index, which the stage's exit addressing applies (block: 32 + 32 table
    // scalars, k per bit, swap mask as a raw word).
    // (two-state kernels apply the same group to both states; the swaps are common)
    auto utab1 = [&](cpx<T>* x, const kptr<T>& blk, bool real) __attribute__((always_inline)) {
      ap_tan<T, R, 0>(x, blk[64]);
      if constexpr (R > 1) {
        __builtin_amdgcn_sched_barrier(0);
        ap_tan<T, R, 1>(x, blk[65]);
      }
      if constexpr (R > 2) {
        __builtin_amdgcn_sched_barrier(0);
        ap_tan<T, R, 2>(x, blk[66]);
      }
      if constexpr (R > 3) {
        __builtin_amdgcn_sched_barrier(0);
        ap_tan<T, R, 3>(x, blk[67]);
      }
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (DUAL) {
        if (real) ap_table_real<T, R>(x, blk);
        else ap_table<T, R>(x, blk);
      } else {
        ap_table<T, R>(x, blk);
      }
    };
    auto utab = [&](int slot) __attribute__((always_inline)) {
      if constexpr (R <= 4 && std::is_same<T, float>::value) {
        const kptr<T> blk = coef + (int64_t)slot * 8;
        const bool real = (sflags & SF_REAL_TAB) != 0u;
        utab1(a, blk, real);
        if constexpr (DUAL) {
          __builtin_amdgcn_sched_barrier(0);
          utab1(b, blk, real);
        }
        pend = *(kptr<uint32_t>)(blk + 68) & (uint32_t)(NR - 1);
      }
    };
    // a factored op ends its stage: it runs after the op loop, outside the
    // op dispatch (the loop is empty for the common stage holding only it)
    int o_end = op_end;
    bool last_utab = false;
    if constexpr (R <= 4 && std::is_same<T, float>::value) {
      last_utab = (sflags & SF_LAST_UTAB) != 0u;
      if (last_utab) --o_end;
    }
    for (int o = op_begin; o < o_end; ++o) {
      kptr<DevOp> op = OPS + o;
      // type, j, ck, cb | ck2, cb2, ph, pad
      const uint32_t w0 = *(kptr<uint32_t>)op, w1 = *((kptr<uint32_t>)op + 1);
      const uint32_t type = w0 & 0xffu, opj = (w0 >> 8) & 0xffu, ck = (w0 >> 16) & 0xffu, cb = w0 >> 24;
      const uint32_t ck2 = w1 & 0xffu, cb2 = (w1 >> 8) & 0xffu, ph = (w1 >> 16) & 0xffu;
      if (type == OP_U || type == OP_RY || type == OP_X) {
        kptr<T> u = coef + (int64_t)op->slot * 8;
        const BitSel c = mkbit(ck, cb, tl, base);
        for_bit<R>(opj, [&](auto JC) __attribute__((always_inline)) {
          constexpr int J = decltype(JC)::value;
          if (type == OP_U) {
            ap_u<T, R, J>(a, u, c);
            if constexpr (DUAL) ap_u<T, R, J>(b, u, c);
          } else if (type == OP_RY) {
            ap_ry<T, R, J>(a, u, c);
            if constexpr (DUAL) ap_ry<T, R, J>(b, u, c);
          } else {
            ap_x<T, R, J>(a, c);
            if constexpr (DUAL) ap_x<T, R, J>(b, c);
          }
        });
      } else if (!DUAL && R <= 4 && (type == OP_UALL || type == OP_RYALL)) {
        // one rotation per register bit, bits 0..R-1 in order: straight-line code
        const BitSel nc{BK_NONE, 0u, 0u};
        auto slot_u = [&](int J) __attribute__((always_inline)) { return coef + (int64_t)(op + 1 + J)->slot * 8; };
        if (type == OP_UALL) {
          auto apply = [&](auto JC) __attribute__((always_inline)) {
            constexpr int J = decltype(JC)::value;
            const kptr<T> u = slot_u(J);
            ap_u<T, R, J>(a, u, nc);
            if constexpr (DUAL) ap_u<T, R, J>(b, u, nc);
          };
          apply(IC<0>{});
          // no interleaving across bits: the compiler would keep several bits' partial
          // results live at once and spill
          if constexpr (R > 1) {
            __builtin_amdgcn_sched_barrier(0);
            apply(IC<1>{});
          }
          if constexpr (R > 2) {
            __builtin_amdgcn_sched_barrier(0);
            apply(IC<2>{});
          }
          if constexpr (R > 3) {
            __builtin_amdgcn_sched_barrier(0);
            apply(IC<3>{});
          }
          if constexpr (R > 4) {
            __builtin_amdgcn_sched_barrier(0);
            apply(IC<4>{});
          }
        } else {
          auto apply = [&](auto JC) __attribute__((always_inline)) {
            constexpr int J = decltype(JC)::value;
            const kptr<T> u = slot_u(J);
            ap_ry<T, R, J>(a, u, nc);
            if constexpr (DUAL) ap_ry<T, R, J>(b, u, nc);
          };
          apply(IC<0>{});
          // no interleaving across bits: the compiler would keep several bits' partial
          // results live at once and spill
          if constexpr (R > 1) {
            __builtin_amdgcn_sched_barrier(0);
            apply(IC<1>{});
          }
          if constexpr (R > 2) {
            __builtin_amdgcn_sched_barrier(0);
            apply(IC<2>{});
          }
          if constexpr (R > 3) {
            __builtin_amdgcn_sched_barrier(0);
            apply(IC<3>{});
          }
          if constexpr (R > 4) {
            __builtin_amdgcn_sched_barrier(0);
            apply(IC<4>{});
          }
        }
        o += R;
      } else if (R <= 4 && std::is_same<T, float>::value && type == OP_DTAB) {
        ap_table<T, R>(a, coef + (int64_t)op->slot * 8 + 32);
        if constexpr (DUAL) ap_table<T, R>(b, coef + (int64_t)op->slot * 8 + 32);
      } else if (R <= 4 && type == OP_PTAB) {
        // the per-thread factor of the thread- and tile-bit phases, then one
        // complex product per amplitude with the register table times that factor
        T fr = 1, fi = 0;
        const int nrec = (int)opj;
        for (int k = 1; k <= nrec; ++k) {
          const uint32_t wr = *(kptr<uint32_t>)(OPS + o + k);
          const kptr<T> c = coef + (int64_t)(OPS + o + k)->slot * 8;
          const bool one = mkbit((wr >> 16) & 0xffu, wr >> 24, tl, base).val != 0u;
          const T dr = one ? c[2] : c[0], di = one ? c[3] : c[1];
          const T xr = fr * dr - fi * di;
          fi = fr * di + fi * dr;
          fr = xr;
        }
        const int tslot = op->slot;
        const bool lane_f = nrec > 0;
#pragma unroll
        for (int i = 0; i < NR; ++i) {
          T tr = fr, ti = fi;
          if (tslot >= 0) {
            const kptr<T> d = coef + (int64_t)tslot * 8;
            if (lane_f) {
              tr = d[2 * i] * fr - d[2 * i + 1] * fi;
              ti = d[2 * i] * fi + d[2 * i + 1] * fr;
            } else {
              tr = d[2 * i];
              ti = d[2 * i + 1];
            }
          }
          const cpx<T> x = a[i];
          a[i].x = tr * x.x - ti * x.y;
          a[i].y = tr * x.y + ti * x.x;
          if constexpr (DUAL) {
            const cpx<T> y = b[i];
            b[i].x = tr * y.x - ti * y.y;
            b[i].y = tr * y.y + ti * y.x;
          }
        }
        o += nrec;
      } else if (type == OP_PHASE) {
        kptr<T> d = coef + (int64_t)op->slot * 8;
        const BitSel c = mkbit(ck, cb, tl, base);
        ap_phase<T, R>(a, d, c);
        if constexpr (DUAL) ap_phase<T, R>(b, d, c);
      } else if (type == OP_CZ) {
        const BitSel c1 = mkbit(ck, cb, tl, base);
        const BitSel c2 = mkbit(ck2, cb2, tl, base);
        ap_cz<T, R>(a, c1, c2);
        if constexpr (DUAL) ap_cz<T, R>(b, c1, c2);
      } else if (type == OP_CZS) {
        // the sign pattern over the register index: the pairs on two register
        // bits from the planner, then per record a register bit's pattern when
        // the other bit is set, or every register when both are
        uint32_t S = op->rz;
        const int nrec = (int)opj;
        for (int k = 1; k <= nrec; ++k) {
          const uint32_t wr = *(kptr<uint32_t>)(OPS + o + k), wr1 = *((kptr<uint32_t>)(OPS + o + k) + 1);
          const BitSel c1 = mkbit((wr >> 16) & 0xffu, wr >> 24, tl, base);
          const BitSel c2 = mkbit(wr1 & 0xffu, (wr1 >> 8) & 0xffu, tl, base);
          if (c1.kind == BK_REG) S ^= c2.val ? reg_pattern<R>(c1.idx) : 0u;
          else if (c2.kind == BK_REG) S ^= c1.val ? reg_pattern<R>(c2.idx) : 0u;
          else S ^= (c1.val & c2.val) ? reg_pattern_all<R>() : 0u;
        }
        ap_signs<T, R>(a, S);
        if constexpr (DUAL) ap_signs<T, R>(b, S);
        o += nrec;
      } else if (type == OP_MEAS_Z) {
        T p[NR];  // |a_i|^2
#pragma unroll
        for (int i = 0; i < NR; ++i) p[i] = a[i].x * a[i].x + a[i].y * a[i].y;
        const uint32_t par = (__popc(tl & op->tz) + __popcll(base & op->pz) + __popc(op->rz & pend)) & 1;
        const double v = (double)meas_zp<T, R>(p, op->rz);
        acc += op->c * (par ? -v : v);
      } else if (type == OP_MEAS_ZS) {
        // W[k] = sum_i (-1)^{parity(i & k)} |a_i|^2 by an in-register Walsh-Hadamard transform;
        // each term then reads W at its register mask.
        T wt[NR];
#pragma unroll
        for (int i = 0; i < NR; ++i) wt[i] = a[i].x * a[i].x + a[i].y * a[i].y;
#pragma unroll
        for (int bb = 0; bb < R; ++bb) {
#pragma unroll
          for (int i = 0; i < NR; ++i) {
            if (i & (1 << bb)) continue;
            const T x = wt[i], y = wt[i | (1 << bb)];
            wt[i] = x + y;
            wt[i | (1 << bb)] = x - y;
          }
        }
        const int nt = op->slot;
        T part = 0;
        for (int k = 1; k <= nt; ++k) {
          kptr<DevOp> tr = OPS + o + k;
          // with pending register swaps, register i holds index i ^ pend: the term's
          // sign gains the parity of rz & pend
          const uint32_t par = (__popc(tl & tr->tz) + __popcll(base & tr->pz) + __popc(tr->rz & pend)) & 1;
          T wv = 0;
          if (tr->rz == 0u) {
            wv = wt[0];
          } else {
            for_mask<NR>(tr->rz, [&](auto KC) __attribute__((always_inline)) { wv = wt[decltype(KC)::value]; });
          }
          const T cc = (T)tr->c;
          part += par ? -cc * wv : cc * wv;
        }
        acc += (double)part;
        o += nt;
      } else if (type == OP_MEAS_F) {
        const uint32_t par = (__popc(tl & op->tz) + __popcll(base & op->pz) + __popc(op->rz & pend)) & 1;
        for_mask<NR>(op->fr, [&](auto FC) __attribute__((always_inline)) {
          constexpr int F = decltype(FC)::value;
          acc += op->c * meas_f<T, R, F>(a, op->rz, par, ph);
        });
      } else if constexpr (DUAL) {
        if (type == OP_H_Z) {
          const uint32_t par = (__popc(tl & op->tz) + __popcll(base & op->pz)) & 1;
          h_z<T, R>(a, b, (T)op->c, op->rz, par);
        } else if (type == OP_H_F) {
          const uint32_t par = (__popc(tl & op->tz) + __popcll(base & op->pz)) & 1;
          for_mask<NR>(op->fr, [&](auto FC) __attribute__((always_inline)) {
            constexpr int F = decltype(FC)::value;
            h_f<T, R, F>(a, b, (T)op->c, op->rz, par, ph);
          });
        } else if (type == OP_GRAD_X || type == OP_GRAD_Y || type == OP_GRAD_Z) {
          T v = 0;
          if (type == OP_GRAD_Z) {
            v = grad_z<T, R>(a, b, mkbit(ck, cb, tl, base));
          } else {
            for_bit<R>(opj, [&](auto JC) __attribute__((always_inline)) {
              constexpr int J = decltype(JC)::value;
              v = type == OP_GRAD_X ? grad_x<T, R, J>(a, b) : grad_y<T, R, J>(a, b);
            });
          }
          const T w = wave_sum(v);
          if (lane == 0) gacc[wave * gcount + (op->slot - gbegin)] += (double)w;
        } else if (type == OP_GZS) {
          // Z probes of up to 4 qubits on the same states: with w_i = Im(conj(b_i) a_i),
          // a register-bit probe is the Walsh coefficient W[1 << j] of w over the
          // register index, a thread- or tile-bit probe is +-W[0]
          T wt[NR];
#pragma unroll
          for (int i = 0; i < NR; ++i) wt[i] = b[i].x * a[i].y - b[i].y * a[i].x;
#pragma unroll
          for (int bb = 0; bb < R; ++bb) {
#pragma unroll
            for (int i = 0; i < NR; ++i) {
              if (i & (1 << bb)) continue;
              const T x = wt[i], y = wt[i | (1 << bb)];
              wt[i] = x + y;
              wt[i | (1 << bb)] = x - y;
            }
          }
          const int nt = op->slot;
          T v[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            v[k] = 0;
            if (k < nt) {
              const uint32_t wr = *(kptr<uint32_t>)(OPS + o + 1 + k);
              const uint32_t rk = (wr >> 16) & 0xffu, rbit = wr >> 24;
              if (rk == BK_REG) {
                for_bit<R>((int)rbit, [&](auto JC) __attribute__((always_inline)) {
                  v[k] = wt[1 << decltype(JC)::value];
                });
              } else {
                v[k] = mkbit(rk, rbit, tl, base).val ? -wt[0] : wt[0];
              }
            }
          }
          T tot[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) tot[k] = wave_sum(v[k]);
          if (lane == 0)
            for (int k = 0; k < nt; ++k)
              gacc[wave * gcount + ((OPS + o + 1 + k)->slot - gbegin)] += (double)tot[k];
          o += nt;
        } else if (type == OP_GXYS) {
          // X and Y probes on up to 4 register bits on the same states
          const int nt = op->slot;
          T v[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            v[k] = 0;
            if (k < nt) {
              const uint32_t w0 = *(kptr<uint32_t>)(OPS + o + 1 + k), w1 = *((kptr<uint32_t>)(OPS + o + 1 + k) + 1);
              const int rj = (int)((w0 >> 8) & 0xffu);
              const bool isy = ((w1 >> 16) & 0xffu) != 0u;
              for_bit<R>(rj, [&](auto JC) __attribute__((always_inline)) {
                constexpr int J = decltype(JC)::value;
                if (isy) v[k] = grad_y<T, R, J>(a, b);
                else v[k] = grad_x<T, R, J>(a, b);
              });
            }
          }
          T tot[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) tot[k] = wave_sum(v[k]);
          if (lane == 0)
            for (int k = 0; k < nt; ++k)
              gacc[wave * gcount + ((OPS + o + 1 + k)->slot - gbegin)] += (double)tot[k];
          o += nt;
        }
      }
    }
    if (last_utab) utab((int)(sflags >> 8));  // the group's first coefficient slot, from the header
    // A pass that stores in its first stage (no exchange barrier between the
    // loads and the stores) and whose loads or stores go through a permutation
    // stores to addresses that other waves load from: every wave's loads must be
    // complete before any wave stores.  Later stages (measurements) may follow.
    // The TAIL variant stores after the last stage, which is then the first.
    if (cross && s == s0) {
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      lds_sync();
    }

    if (!TAIL && s == sst) {
      const bool st_a = (flags & PF_STORE_A) != 0, st_b = DUAL && (flags & PF_STORE_B) != 0;
      uint64_t gr[R];
      uint64_t gt = store_gaddr<R>(P, S, tid, base, gr);
      // offsets combine by XOR, so index i ^ pend is gt ^ (bits of pend) ^ (bits of i)
#pragma unroll
      for (int j = 0; j < R; ++j)
        if ((pend >> j) & 1u) gt ^= gr[j];
      if (active) {
#pragma unroll
        for (int i = 0; i < NR; ++i) {
          uint64_t g = gt;
#pragma unroll
          for (int j = 0; j < R; ++j)
            if ((i >> j) & 1) g ^= gr[j];
          if (st_a) st_amp(A + g, a[i]);
          if constexpr (DUAL) {
            if (st_b) st_amp(B + g, b[i]);
          }
        }
      }
    }
    if (s + 1 < s1) {
      // An exchange that keeps every amplitude in its wave needs no barrier
      // before its writes when the tile's previous exchange kept them too (each
      // wave then only ever touches its own block), and none after them (a
      // wave's LDS operations complete in order).
      const bool wl = (sflags & SF_WAVE_LOCAL) != 0;
      if (!(wl && prev_wl)) lds_sync();
      else asm volatile("" ::: "memory");
      if (active) {
        // every amplitude to its slot in the next layout: through the stage's
        // exit permutation when it has one (the precomputed write parts are its
        // images), else the slots it was read from; register i holds index i ^ pend
        uint32_t wu = wrw;  // uniform part: wave bits and the affine part (the tile's non-local control bits)
        if (n_aff > 0) {
          uint32_t wa = 0;
          for (int j = 0; j < (int)n_aff; ++j)
            if ((base >> kb(&S->aff_pos[j])) & 1) wa ^= kh(&S->wr_aff[j]);
          wu ^= wa;
        }
        uint32_t wr_b;
        if (tab) {
          wr_b = lt[1] ^ (wu << kSh);
        } else {
          uint32_t wr = wu;
#pragma unroll
          for (int k = 0; k < 6; ++k) wr ^= ((uint32_t)(tid >> k) & 1u) ? hd.u16(14 + k) : 0u;
          wr_b = wr << kSh;
        }
        uint32_t pb[R];  // byte offsets of the images of the register bits
#pragma unroll
        for (int j = 0; j < R; ++j) pb[j] = hd.u16(26 + j) << kSh;
        uint32_t wp = 0;  // image of register index pend (linear)
#pragma unroll
        for (int j = 0; j < R; ++j)
          if ((pend >> j) & 1u) wp ^= pb[j];
        uint32_t w_b = (lds0 + wr_b) ^ wp;
        asm volatile("" : "+v"(w_b));
#pragma unroll
        for (int i = 0; i < NR; ++i) {
          uint32_t po = 0;
#pragma unroll
          for (int j = 0; j < R; ++j)
            if ((i >> j) & 1) po ^= pb[j];
          const uint32_t l = w_b ^ po;
          st_lds<T>(l, a[i]);
          if constexpr (DUAL) st_lds<T>(l + bofs, b[i]);
        }
      }
      if (wl) asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
      else lds_sync();
      prev_wl = wl;
    }
  }
  if constexpr (TAIL) {
    // The caller guarantees: psi is stored after the last stage and every lane
    // holds amplitudes of the tile.  Stores issued unconditionally let the
    // compiler count them, so waiting for a prefetched tile does not also wait
    // for these stores to complete.
    uint64_t gr[R];
    uint64_t gt = store_gaddr<R>(P, SD + (s1 - 1), tid, base, gr);
#pragma unroll
    for (int j = 0; j < R; ++j)
      if ((pend >> j) & 1u) gt ^= gr[j];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      uint64_t g = gt;
#pragma unroll
      for (int j = 0; j < R; ++j)
        if ((i >> j) & 1) g ^= gr[j];
      st_amp(A + g, a[i]);
    }
  }
  double total = 0.0;
  if (flags & PF_MEASURE) {
    const double v = wave_sum(acc);
    if (lane == 0) red[wave] = v;
    lds_sync();
    if (tid == 0)
      for (int w = 0; w < nwaves; ++w) total += red[w];
    lds_sync();
  }
  if (DUAL && (flags & PF_GRAD)) {
    lds_sync();
    for (int k = tid; k < gcount; k += nthr) {
      double sum = 0.0;
      for (int w = 0; w < nwaves; ++w) sum += gacc[w * gcount + k];
      double* dst = grad_out + (int64_t)(gbegin + k) * grad_stride;
      *dst = grad_add ? *dst + sum : sum;  // the same thread wrote the previous tile's value
    }
    lds_sync();
  }
  return total;
}

constexpr int kRedSlots = 16;

// Threads per workgroup: 2^(m-r).  Tiles hold at most 2^14 complex64
// amplitudes of one state (128 KiB of LDS), 2^13 of two states or of one
// complex128 state, 2^12 of two complex128 states.
template <class T, int R, bool DUAL>
constexpr int pass_max_threads() {
  constexpr int mmax = sizeof(T) == 4 ? (DUAL ? 13 : 14) : (DUAL ? 12 : 13);
  return (1 << (mmax - R)) < 1024 ? (1 << (mmax - R)) : 1024;
}

// Dense pass over rows x 2^(n-m) tiles.  Workgroups are persistent: each one
// walks tiles w, w + gridDim.x, ...  With PF, it issues the HBM loads of its
// next tile before working on the current one, so the loads overlap the
// register and LDS work (a 2^14-amplitude tile fills a CU's LDS, leaving no
// second workgroup to overlap with); this needs twice the data registers.
template <class T, int R, bool DUAL, bool PF, bool TAIL = false>
__global__ __launch_bounds__((pass_max_threads<T, R, DUAL>())) void k_pass(
    const PassDesc* __restrict__ Pg, const StageDesc* __restrict__ SDg, const DevOp* __restrict__ OPSg, cpx<T>* A,
    cpx<T>* B, int64_t row_stride, const T* __restrict__ coefg, int64_t coef_row_stride, double* meas, int n_meas,
    double* grad, int n_gslots, int64_t rows) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const kptr<PassDesc> P = kc(Pg);
  const kptr<StageDesc> SD = kc(SDg);
  const kptr<DevOp> OPS = kc(OPSg);
  const kptr<T> coef = kc(coefg);
  const int m = P->m, sh = P->n - m;
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem);
  double* red = reinterpret_cast<double*>(smem + ((size_t)(DUAL ? 2 : 1) * sizeof(cpx<T>) << m));
  double* gacc = red + kRedSlots;
  const int64_t tiles = 1ll << sh;
  const int64_t total = tiles * rows;
  const kptr<StageDesc> S0 = SD + P->stage_begin;
  int64_t w = blockIdx.x;
  if (w >= total) return;
  TileRegs<T, R, DUAL> cur;
  int64_t row = w >> sh;
  uint64_t tile = (uint64_t)(w & (tiles - 1));
  const uint64_t M = nonlocal_mask(P);
  const uint64_t dstep = deposit((uint64_t)gridDim.x & (uint64_t)(tiles - 1), M);
  uint64_t base = deposit(tile, M);
  tile_load<T, R, DUAL>(P, S0, A + row * row_stride, DUAL ? B + row * row_stride : nullptr, base, cur,
                        coef + row * coef_row_stride);
  // the pass's lane table after the tile, reduction and gradient slots (while the loads are in flight)
  uint32_t* ltab = reinterpret_cast<uint32_t*>(
      smem + ((size_t)(DUAL ? 2 : 1) * sizeof(cpx<T>) << m) + kRedSlots * sizeof(double) +
      (DUAL ? (size_t)kRedSlots * kMaxGradPerPass * sizeof(double) : 0));
  fill_lane_table<T>(P, SD, ltab);
  while (true) {
    const int64_t wn = w + gridDim.x;
    const bool more = wn < total;
    const int64_t rown = wn >> sh;
    const uint64_t tilen = (uint64_t)(wn & (tiles - 1));
    const uint64_t basen = next_base(base, M, dstep);
    if constexpr (PF) {
      TileRegs<T, R, DUAL> nxt;
      if (more)
        tile_load<T, R, DUAL>(P, S0, A + rown * row_stride, DUAL ? B + rown * row_stride : nullptr, basen, nxt,
                              coef + rown * coef_row_stride);
      double* gout = (DUAL && grad) ? grad + row * n_gslots * tiles + (int64_t)tile : nullptr;
      const double v = tile_run<T, R, DUAL, TAIL, true>(P, SD, OPS, A + row * row_stride,
                                                        DUAL ? B + row * row_stride : nullptr,
                                                        coef + row * coef_row_stride, base, cur, lds, red, gacc, gout,
                                                        tiles, false, ltab);
      if ((P->flags & PF_MEASURE) && threadIdx.x == 0)
        meas[(row * n_meas + P->meas_index) * tiles + (int64_t)tile] = v;
      if (!more) break;
      cur = nxt;
    } else {
      double* gout = (DUAL && grad) ? grad + row * n_gslots * tiles + (int64_t)tile : nullptr;
      const double v = tile_run<T, R, DUAL, false, true>(P, SD, OPS, A + row * row_stride,
                                                         DUAL ? B + row * row_stride : nullptr,
                                                         coef + row * coef_row_stride, base, cur, lds, red, gacc,
                                                         gout, tiles, false, ltab);
      if ((P->flags & PF_MEASURE) && threadIdx.x == 0)
        meas[(row * n_meas + P->meas_index) * tiles + (int64_t)tile] = v;
      if (!more) break;
      tile_load<T, R, DUAL>(P, S0, A + rown * row_stride, DUAL ? B + rown * row_stride : nullptr, basen, cur,
                            coef + rown * coef_row_stride);
    }
    w = wn;
    row = rown;
    tile = tilen;
    base = basen;
  }
}

template <class T, int R, bool DUAL>
__global__ __launch_bounds__((pass_max_threads<T, R, DUAL>())) void k_pass_multi(const PassItem* __restrict__ items,
                                                                             int n_items, int m_max, int64_t total) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem);
  double* red = reinterpret_cast<double*>(smem + ((size_t)(DUAL ? 2 : 1) * sizeof(cpx<T>) << m_max));
  double* gacc = red + kRedSlots;
  const kptr<PassItem> KI = kc(items);
  // Persistent workgroups walk the launch's tiles b, b + gridDim.x, ...; the
  // items' tile ranges ascend, so each search starts at the current item.
  int cur = 0;
  kptr<PassItem> it = KI;
  kptr<PassDesc> P = kc(it->pass);
  uint64_t M = nonlocal_mask(P);
  for (int64_t b = blockIdx.x; b < total; b += gridDim.x) {
    int lo = cur, hi = n_items - 1;
    while (lo < hi) {  // last item with tile_begin <= b
      const int mid = (lo + hi + 1) >> 1;
      if ((KI + mid)->tile_begin <= b) lo = mid;
      else hi = mid - 1;
    }
    if (lo != cur) {
      cur = lo;
      it = KI + lo;
      P = kc(it->pass);
      M = nonlocal_mask(P);
    }
    const kptr<StageDesc> SD = kc(it->stages);
    const int64_t tiles = 1ll << (P->n - P->m);
    const uint64_t tile = (uint64_t)(b - it->tile_begin);
    const uint64_t base = deposit(tile, M);
    double* gout = (DUAL && it->grad) ? it->grad + (int64_t)tile : nullptr;
    cpx<T>* A = reinterpret_cast<cpx<T>*>(it->A);
    cpx<T>* B = reinterpret_cast<cpx<T>*>(it->B);
    TileRegs<T, R, DUAL> t;
    tile_load<T, R, DUAL>(P, SD + P->stage_begin, A, B, base, t, kc(reinterpret_cast<const T*>(it->coef)));
    const double v = tile_run<T, R, DUAL>(P, SD, kc(it->ops), A, B, kc(reinterpret_cast<const T*>(it->coef)), base,
                                          t, lds, red, gacc, gout, tiles);
    if ((P->flags & PF_MEASURE) && threadIdx.x == 0) it->meas[(int64_t)P->meas_index * tiles + (int64_t)tile] = v;
  }
}

// One workgroup per cone: the cone's passes run in order, each over its tiles.
// A cone of at most m qubits is a single tile (LDS-resident within a pass);
// larger cones and states kept between passes live in scratch.  DUAL cones run
// forward, lambda = P psi and the adjoint sweep; their gradient probes
// accumulate over tiles into the cone's own gradient slots.
template <class T, int R, bool DUAL>
__global__ __launch_bounds__((pass_max_threads<T, R, DUAL>())) void k_cones(
    const ConeDesc* __restrict__ cones, const int32_t* __restrict__ order, const PassDesc* __restrict__ Pg,
    const StageDesc* __restrict__ SDg, const DevOp* __restrict__ OPSg, cpx<T>* scratch, const T* __restrict__ coef,
    double* out, double* grad, int m_max) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem);
  double* red = reinterpret_cast<double*>(smem + ((size_t)(DUAL ? 2 : 1) * sizeof(cpx<T>) << m_max));
  double* gacc = red + kRedSlots;
  const kptr<PassDesc> P = kc(Pg);
  const kptr<StageDesc> SD = kc(SDg);
  const kptr<DevOp> OPS = kc(OPSg);
  const kptr<ConeDesc> cd = kc(cones) + *(kc(order) + blockIdx.x);
  double total = 0.0;
  cpx<T>* st = scratch + cd->scratch_off;
  cpx<T>* st_b = DUAL ? st + (1ll << cd->n) : nullptr;
  const kptr<T> cf = kc(coef) + (int64_t)cd->coef_begin * 8;
  const int pass_end = cd->pass_end, out_index = cd->out_index;
  for (int p = cd->pass_begin; p < pass_end; ++p) {
    const kptr<PassDesc> pp = P + p;
    const int64_t tiles = 1ll << (pp->n - pp->m);
    const uint64_t M = nonlocal_mask(pp), d1 = M & (~M + 1);
    uint64_t base = 0;
    for (int64_t t = 0; t < tiles; ++t, base = next_base(base, M, d1)) {
      TileRegs<T, R, DUAL> regs;
      tile_load<T, R, DUAL>(pp, SD + pp->stage_begin, st, st_b, base, regs, cf);
      total += tile_run<T, R, DUAL>(pp, SD, OPS, st, st_b, cf, base, regs, lds, red, gacc, grad, 1, t > 0);
      lds_sync();
    }
    // the next pass reads what other waves of this workgroup stored
    __threadfence();
    __syncthreads();
  }
  if (threadIdx.x == 0) out[out_index] = total;
}

__global__ __launch_bounds__(256) void k_reduce_rows(const double* __restrict__ part, int64_t per_row, double add,
                                                     double* out) {
  __shared__ double sh[256];
  const int64_t row = blockIdx.x;
  const double* pr = part + row * per_row;
  double s = 0.0;
  int64_t k = threadIdx.x;
  // each thread adds its values in index order; loads are issued 16 at a time
  // so their latencies overlap (the sum order is unchanged)
  for (; k + 15 * 256 < per_row; k += 16 * 256) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = pr[k + u * 256];
#pragma unroll
    for (int u = 0; u < 16; ++u) s += v[u];
  }
  for (; k < per_row; k += 256) s += pr[k];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[row] = sh[0] + add;
}

__global__ __launch_bounds__(256) void k_grad_scatter(const double* __restrict__ slot_total, int rows, int n_slots,
                                                      const int32_t* __restrict__ p_off,
                                                      const int32_t* __restrict__ p_slots, int n_params,
                                                      double* grad) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)rows * n_params) return;
  const int64_t row = idx / n_params;
  const int p = (int)(idx % n_params);
  double s = 0.0;
  for (int k = p_off[p]; k < p_off[p + 1]; ++k) s += slot_total[row * n_slots + p_slots[k]];
  grad[idx] = s;
}

__global__ __launch_bounds__(256) void k_term_products(const double* __restrict__ fval, const int32_t* __restrict__ off,
                                                       const int32_t* __restrict__ fac,
                                                       const double* __restrict__ coef, int T, double* tval) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= T) return;
  double v = coef[t];
  for (int k = off[t]; k < off[t + 1]; ++k) v *= fval[fac[k]];
  tval[t] = v;
}

__global__ __launch_bounds__(256) void k_factor_weights(const double* __restrict__ fval,
                                                        const int32_t* __restrict__ f_off,
                                                        const int32_t* __restrict__ f_terms,
                                                        const int32_t* __restrict__ t_off,
                                                        const int32_t* __restrict__ t_fac,
                                                        const double* __restrict__ t_coef, int F, double* w) {
  const int f = blockIdx.x * 256 + threadIdx.x;
  if (f >= F) return;
  double s = 0.0;
  for (int i = f_off[f]; i < f_off[f + 1]; ++i) {
    const int t = f_terms[i];
    double v = t_coef[t];
    for (int k = t_off[t]; k < t_off[t + 1]; ++k)
      if (t_fac[k] != f) v *= fval[t_fac[k]];
    s += v;
  }
  w[f] = s;
}

__global__ __launch_bounds__(256) void k_weighted_scatter(const double* __restrict__ g,
                                                          const int32_t* __restrict__ g_cone,
                                                          const double* __restrict__ w,
                                                          const int32_t* __restrict__ p_off,
                                                          const int32_t* __restrict__ p_slots, int n_params,
                                                          double* grad) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= n_params) return;
  double s = 0.0;
  for (int k = p_off[p]; k < p_off[p + 1]; ++k) {
    const int slot = p_slots[k];
    s += w[g_cone[slot]] * g[slot];
  }
  grad[p] = s;
}

// The reference stream: one 16-byte element per thread, one workgroup per 256
// elements (faster on this chip than a persistent grid-stride copy: 6.2 against
// 4.8 TB/s for 8 GiB each way).
__global__ __launch_bounds__(256) void k_copy(const float4* __restrict__ src, float4* __restrict__ dst, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// Kernels running tiles: the dynamic LDS size allowance, and a check that the
// kernel has no static LDS, so the tile buffer (the start of dynamic LDS) sits
// at LDS address 0 as the XOR slot addressing assumes.
template <class K>
hipError_t allow_lds(K kernel, size_t bytes) {
  static std::mutex mu;
  static std::map<const void*, hipError_t> checked;
  const void* f = reinterpret_cast<const void*>(kernel);
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = checked.find(f);
    if (it == checked.end()) {
      hipFuncAttributes fa;
      hipError_t e = hipFuncGetAttributes(&fa, f);
      if (e == hipSuccess && fa.sharedSizeBytes != 0) e = hipErrorInvalidDeviceFunction;
      it = checked.emplace(f, e).first;
    }
    if (it->second != hipSuccess) return it->second;
  }
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

int device_cus() {
  static int cus = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess || v <= 0)
      v = 256;
    return v;
  }();
  return cus;
}

// Workgroups of a kernel resident on one CU at once (occupancy query; at least 1).
template <class K>
int resident_per_cu(K kernel, int threads, size_t lds) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(kernel), threads, lds) !=
          hipSuccess ||
      nb < 1) {
    (void)hipGetLastError();
    nb = std::max(1, std::min((int)((size_t)max_lds_bytes() / lds), 2048 / threads));
  }
  return nb;
}

template <class T, int R, bool DUAL, bool PF, bool TAIL = false>
hipError_t launch_pass_t(const PassLaunch& L, hipStream_t stream) {
  const int m = L.h_pass->m, n = L.h_pass->n;
  const size_t lds = pass_lds_bytes(m, sizeof(T) == 8, DUAL) +
                     lane_table_bytes(L.h_pass->stage_end - L.h_pass->stage_begin);
  auto kern = k_pass<T, R, DUAL, PF, TAIL>;
  hipError_t e = allow_lds(kern, lds);
  if (e != hipSuccess) return e;
  const int threads = std::max(64, 1 << (m - R));
  // persistent workgroups: as many as fit on the device at once (registers, LDS, threads)
  const int per_cu = resident_per_cu(kern, threads, lds);
  const int64_t total = (int64_t)L.rows << (n - m);
  const int64_t grid = std::min<int64_t>(total, (int64_t)device_cus() * per_cu);
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(threads), lds, stream, L.d_pass, L.d_stages, L.d_ops,
                     reinterpret_cast<cpx<T>*>(L.A), reinterpret_cast<cpx<T>*>(L.B), L.row_stride,
                     reinterpret_cast<const T*>(L.coef), L.coef_row_stride, L.meas, L.n_meas, L.grad, L.n_gslots,
                     (int64_t)L.rows);
  return hipGetLastError();
}

// Register bits per thread by precision and kind; the 32-register complex64
// single-state variant prefetches (its 512 threads leave 256 VGPRs each).
template <class T, bool DUAL>
hipError_t launch_pass_r(const PassLaunch& L, hipStream_t stream) {
  switch (L.h_pass->r) {
    case 1: return launch_pass_t<T, 1, DUAL, false>(L, stream);
    case 2: return launch_pass_t<T, 2, DUAL, false>(L, stream);
    case 3:
      if constexpr (!DUAL && sizeof(T) == 4) {
        // 8 amplitudes per thread leave room for a register prefetch of the next tile
        const PassDesc& p = *L.h_pass;
        if (L.prefetch && p.m - 3 >= 6 && (p.flags & PF_STORE_A) && p.store_stage == p.stage_end - 1)
          return launch_pass_t<T, 3, false, true, true>(L, stream);
      }
      return launch_pass_t<T, 3, DUAL, false>(L, stream);
    case 4:
      if constexpr (DUAL && sizeof(T) == 8) return hipErrorInvalidValue;
      else if (DUAL && !L.prefetch) return launch_pass_t<T, 4, DUAL, false>(L, stream);
      else return launch_pass_t<T, 4, DUAL, DUAL && sizeof(T) == 4>(L, stream);
    case 5:
      if constexpr (DUAL || sizeof(T) == 8) return hipErrorInvalidValue;
      else {
        if (!L.prefetch) return launch_pass_t<T, 5, false, false>(L, stream);
        // psi stored after the last stage by every lane: the store-at-the-end variant
        const PassDesc& p = *L.h_pass;
        const bool tail = (p.flags & PF_STORE_A) && p.store_stage == p.stage_end - 1 && p.m - 5 >= 6;
        return tail ? launch_pass_t<T, 5, false, true, true>(L, stream) : launch_pass_t<T, 5, false, true>(L, stream);
      }
    default: return hipErrorInvalidValue;
  }
}

template <class T, int R, bool DUAL>
hipError_t launch_cones_t(const ConeLaunch& L, hipStream_t stream) {
  const size_t lds = pass_lds_bytes(L.m_max, sizeof(T) == 8, DUAL);
  auto kern = k_cones<T, R, DUAL>;
  hipError_t e = allow_lds(kern, lds);
  if (e != hipSuccess) return e;
  const int threads = std::max(64, 1 << (L.m_max - R));
  hipLaunchKernelGGL(kern, dim3((unsigned)L.n_cones), dim3(threads), lds, stream, L.d_cones, L.d_order,
                     L.d_passes, L.d_stages, L.d_ops, reinterpret_cast<cpx<T>*>(L.scratch),
                     reinterpret_cast<const T*>(L.coef), L.out, L.grad, L.m_max);
  return hipGetLastError();
}

template <class T, int R, bool DUAL>
hipError_t launch_multi_t(const PassItem* items, int n_items, int64_t total, int m_max, hipStream_t stream) {
  const size_t lds = pass_lds_bytes(m_max, sizeof(T) == 8, DUAL);
  auto kern = k_pass_multi<T, R, DUAL>;
  hipError_t e = allow_lds(kern, lds);
  if (e != hipSuccess) return e;
  const int threads = std::max(64, 1 << (m_max - R));
  const int per_cu = resident_per_cu(kern, threads, lds);
  const int64_t grid = std::min<int64_t>(total, (int64_t)device_cus() * per_cu);
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(threads), lds, stream, items, n_items, m_max, total);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_pass_multi(const PassItem* d_items, int n_items, int64_t total_tiles, int m_max, int r, int c128,
                             int dual, hipStream_t stream) {
  if (n_items == 0) return hipSuccess;
  if (c128) return hipErrorInvalidValue;  // serving runs complex64
  if (dual && r == 4) return launch_multi_t<float, 4, true>(d_items, n_items, total_tiles, m_max, stream);
  if (!dual && r == 4) return launch_multi_t<float, 4, false>(d_items, n_items, total_tiles, m_max, stream);
  if (!dual && r == 5) return launch_multi_t<float, 5, false>(d_items, n_items, total_tiles, m_max, stream);
  return hipErrorInvalidValue;
}

hipError_t launch_term_products(const double* fval, const int32_t* off, const int32_t* fac, const double* coef, int T,
                                double* tval, hipStream_t stream) {
  if (T <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_term_products, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, stream, fval, off, fac, coef, T,
                     tval);
  return hipGetLastError();
}

hipError_t launch_factor_weights(const double* fval, const int32_t* f_off, const int32_t* f_terms,
                                 const int32_t* t_off, const int32_t* t_fac, const double* t_coef, int F, double* w,
                                 hipStream_t stream) {
  if (F <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_factor_weights, dim3((unsigned)((F + 255) / 256)), dim3(256), 0, stream, fval, f_off, f_terms,
                     t_off, t_fac, t_coef, F, w);
  return hipGetLastError();
}

hipError_t launch_weighted_scatter(const double* g, const int32_t* g_cone, const double* w, const int32_t* p_off,
                                   const int32_t* p_slots, int n_params, double* grad, hipStream_t stream) {
  if (n_params <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_weighted_scatter, dim3((unsigned)((n_params + 255) / 256)), dim3(256), 0, stream, g, g_cone, w,
                     p_off, p_slots, n_params, grad);
  return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, uint64_t n16, hipStream_t stream) {
  const uint64_t blocks = (n16 + 255) / 256;
  if (blocks > 0x7fffffffull) return hipErrorInvalidValue;  // above 32 TiB
  hipLaunchKernelGGL(k_copy, dim3((unsigned)std::max<uint64_t>(1, blocks)), dim3(256), 0, stream,
                     reinterpret_cast<const float4*>(src), reinterpret_cast<float4*>(dst), n16);
  return hipGetLastError();
}

size_t pass_lds_bytes(int m, int c128, int dual) {
  const size_t amp = c128 ? 16 : 8;
  return (size_t)(dual ? 2 : 1) * (amp << m) + kRedSlots * sizeof(double) +
         (dual ? (size_t)kRedSlots * kMaxGradPerPass * sizeof(double) : 0);
}

int max_lds_bytes() { return 160 * 1024; }

hipError_t launch_pass(const PassLaunch& L, hipStream_t stream) {
  if (L.c128) return L.dual ? launch_pass_r<double, true>(L, stream) : launch_pass_r<double, false>(L, stream);
  return L.dual ? launch_pass_r<float, true>(L, stream) : launch_pass_r<float, false>(L, stream);
}

hipError_t launch_cones(const ConeLaunch& L, hipStream_t stream) {
  if (L.n_cones == 0) return hipSuccess;
  if (L.r != 4) return hipErrorInvalidValue;
  const int mmax = (L.c128 ? 13 : 14) - (L.dual ? 1 : 0);
  if (L.m_max > mmax || L.m_max < 4 || (L.dual && !L.grad)) return hipErrorInvalidValue;
  if (L.dual) return L.c128 ? launch_cones_t<double, 4, true>(L, stream) : launch_cones_t<float, 4, true>(L, stream);
  return L.c128 ? launch_cones_t<double, 4, false>(L, stream) : launch_cones_t<float, 4, false>(L, stream);
}

hipError_t launch_reduce_rows(const double* part, int rows, int64_t per_row, double add, double* out,
                              hipStream_t stream) {
  if (rows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_rows, dim3((unsigned)rows), dim3(256), 0, stream, part, per_row, add, out);
  return hipGetLastError();
}

hipError_t launch_grad_scatter(const double* slot_total, int rows, int n_slots, const int32_t* p_off,
                               const int32_t* p_slots, int n_params, double* grad, hipStream_t stream) {
  const int64_t total = (int64_t)rows * n_params;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_grad_scatter, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, slot_total, rows,
                     n_slots, p_off, p_slots, n_params, grad);
  return hipGetLastError();
}

}  // namespace qsim
