// Gate matrices and coefficient blocks in fp64, for the host (rows built on
// CPU threads) and for the device (rows built from a parameter buffer that
// stays in device memory).  One definition serves both, so a coefficient row
// means the same whichever side builds it.
//
// Conventions: RX/RY/RZ(t) = exp(-i t P / 2); a slot's matrix is the product of
// its source gates in application order (later gates on the left), adjoint
// when the slot is flagged inverse.
//
// Every value here is computed from correctly rounded IEEE operations only (+,
// -, *, /, sqrt, rint, comparisons), with multiply-add contraction switched off
// and no math-library call (the sine and cosine are the series below), so the
// host and the device produce the same bits.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "qsim_types.h"

#pragma float_control(push)
#pragma clang fp contract(off)

namespace qsim {
namespace cm {

// pi/2 split in three parts of at most 33 significant bits (the first two), so
// k * part is exact for |k| < 2^20; and 2/pi.
constexpr double kPio2a = 0x1.921fb544p+0;
constexpr double kPio2b = 0x1.0b4611a6p-34;
constexpr double kPio2c = 0x1.3198a2e037073p-69;
constexpr double kTwoOverPi = 0x1.45f306dc9c883p-1;

// sin x and cos x: x = k pi/2 + r with |r| <= pi/4 (three-part reduction,
// accurate for |x| < 1.6e6), then the Taylor series of sin r and cos r to
// degree 21 and 20 (truncation below 1e-24 on |r| <= pi/4) in Horner form, and
// the quadrant from k mod 4.
__host__ __device__ inline void sincos_ieee(double x, double* s_out, double* c_out) {
  const double k = ::rint(x * kTwoOverPi);
  double r = x - k * kPio2a;
  r = r - k * kPio2b;
  r = r - k * kPio2c;
  const double u = r * r;
  // sin r = r (1 - u/3! + u^2/5! - ...), cos r = 1 - u/2! + u^2/4! - ...
  double ps = -1.0 / 51090942171709440000.0;  // -1/21!
  ps = ps * u + 1.0 / 121645100408832000.0;    // 1/19!
  ps = ps * u - 1.0 / 355687428096000.0;       // 1/17!
  ps = ps * u + 1.0 / 1307674368000.0;         // 1/15!
  ps = ps * u - 1.0 / 6227020800.0;            // 1/13!
  ps = ps * u + 1.0 / 39916800.0;              // 1/11!
  ps = ps * u - 1.0 / 362880.0;                // 1/9!
  ps = ps * u + 1.0 / 5040.0;                  // 1/7!
  ps = ps * u - 1.0 / 120.0;                   // 1/5!
  ps = ps * u + 1.0 / 6.0;                     // 1/3!
  const double sr = r - (r * u) * ps;
  double pc = 1.0 / 2432902008176640000.0;     // 1/20!
  pc = pc * u - 1.0 / 6402373705728000.0;      // 1/18!
  pc = pc * u + 1.0 / 20922789888000.0;        // 1/16!
  pc = pc * u - 1.0 / 87178291200.0;           // 1/14!
  pc = pc * u + 1.0 / 479001600.0;             // 1/12!
  pc = pc * u - 1.0 / 3628800.0;               // 1/10!
  pc = pc * u + 1.0 / 40320.0;                 // 1/8!
  pc = pc * u - 1.0 / 720.0;                   // 1/6!
  pc = pc * u + 1.0 / 24.0;                    // 1/4!
  pc = pc * u - 1.0 / 2.0;                     // 1/2!
  const double cr = 1.0 + u * pc;
  const int q = (int)((int64_t)k & 3);
  *s_out = q == 0 ? sr : q == 1 ? cr : q == 2 ? -sr : -cr;
  *c_out = q == 0 ? cr : q == 1 ? -sr : q == 2 ? -cr : sr;
}

struct C {
  double re, im;
};

__host__ __device__ inline C mk(double r, double i = 0.0) { return C{r, i}; }
__host__ __device__ inline C add(C a, C b) { return C{a.re + b.re, a.im + b.im}; }
__host__ __device__ inline C mul(C a, C b) { return C{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__host__ __device__ inline C neg(C a) { return C{-a.re, -a.im}; }
__host__ __device__ inline C conj(C a) { return C{a.re, -a.im}; }
__host__ __device__ inline double norm2(C a) { return a.re * a.re + a.im * a.im; }
__host__ __device__ inline double cabs(C a) { return ::sqrt(norm2(a)); }
__host__ __device__ inline C scale(C a, double s) { return C{a.re * s, a.im * s}; }
// a / b (Smith's method: no overflow for entries of a unitary)
__host__ __device__ inline C cdiv(C a, C b) {
  if (::fabs(b.re) >= ::fabs(b.im)) {
    const double r = b.im / b.re, d = b.re + b.im * r;
    return C{(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  }
  const double r = b.re / b.im, d = b.re * r + b.im;
  return C{(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}

struct M2 {
  C a[2][2];
};

__host__ __device__ inline M2 eye() {
  M2 m;
  m.a[0][0] = mk(1);
  m.a[0][1] = mk(0);
  m.a[1][0] = mk(0);
  m.a[1][1] = mk(1);
  return m;
}

__host__ __device__ inline M2 mul(const M2& x, const M2& y) {
  M2 z;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) z.a[i][j] = add(mul(x.a[i][0], y.a[0][j]), mul(x.a[i][1], y.a[1][j]));
  return z;
}

__host__ __device__ inline M2 adjoint(const M2& m) {
  M2 h;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) h.a[i][j] = conj(m.a[j][i]);
  return h;
}

// Gate kinds as in the C-ABI: RX = 0, RY = 1, RZ = 2, U1 = 5 (mat: row-major re, im).
__host__ __device__ inline M2 gate_m2(int kind, double t, const double* mat) {
  M2 u;
  if (kind == 5) {
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) u.a[i][j] = mk(mat[(i * 2 + j) * 2], mat[(i * 2 + j) * 2 + 1]);
    return u;
  }
  double s, c;
  sincos_ieee(0.5 * t, &s, &c);
  if (kind == 0) {  // cos(t/2) I - i sin(t/2) X
    u.a[0][0] = mk(c); u.a[0][1] = mk(0, -s); u.a[1][0] = mk(0, -s); u.a[1][1] = mk(c);
  } else if (kind == 1) {  // cos(t/2) I - i sin(t/2) Y
    u.a[0][0] = mk(c); u.a[0][1] = mk(-s); u.a[1][0] = mk(s); u.a[1][1] = mk(c);
  } else {  // RZ: cos(t/2) I - i sin(t/2) Z
    u.a[0][0] = mk(c, -s); u.a[0][1] = mk(0); u.a[1][0] = mk(0); u.a[1][1] = mk(c, s);
  }
  return u;
}

// Factored form of a unitary 2x2: U = diag(p0, p1) K diag(1, e) with
// K = [[1, -k], [k, 1]] when |u00| >= |u01| (cot = false), else [[k, -1], [1, k]];
// |k| <= 1 either way.  Unitarity (orthogonal rows) makes the remaining entries
// agree: tan form k e = -u01/u00, p0 = u00, p1 = u11/e; cot form k e = u11/u10,
// p1 = u10, p0 = -u01/e.  The sign of k is chosen so that Re e >= 0, which makes
// e = 1 (snapped) whenever k e is real, as for any RZ-after-RY product.
struct KForm {
  bool cot;
  double k;
  C p0, p1, e;
};

__host__ __device__ inline KForm kform(const M2& M) {
  KForm f;
  f.k = 0;
  f.p0 = mk(1);
  f.p1 = mk(1);
  f.e = mk(1);
  const C m00 = M.a[0][0], m01 = M.a[0][1], m10 = M.a[1][0], m11 = M.a[1][1];
  f.cot = norm2(m01) > norm2(m00);
  const C z = f.cot ? cdiv(m11, m10) : neg(cdiv(m01, m00));
  const double az = cabs(z);
  if (az > 0) {
    f.k = z.re >= 0 ? az : -az;
    f.e = scale(z, 1.0 / f.k);
    if (cabs(C{f.e.re - 1.0, f.e.im}) <= 1e-13) f.e = mk(1);
  }
  if (f.cot) {
    f.p1 = m10;
    f.p0 = neg(cdiv(m01, f.e));
  } else {
    f.p0 = m00;
    f.p1 = cdiv(m11, f.e);
  }
  return f;
}

// The coefficient block of one factored group over up to four register bits
// (layout: kTabScalars doubles; see the PG_TAB description in planner.h).  The
// cot form diag(p0, p1) [[k, -1], [1, k]] is rewritten X diag(p1, -p0) T(-k).
// has[j] = 0: no rotation on register bit j (identity).
constexpr int kTabScalars = 72;

__host__ __device__ inline void tab_block(const M2* ms, const int* has, int r, double* blk) {
  for (int k = 0; k < kTabScalars; ++k) blk[k] = 0;
  KForm f[4];
  uint32_t form = 0, pre = 0;
  for (int j = 0; j < r && j < 4; ++j) {
    if (!has[j]) continue;
    f[j] = kform(ms[j]);
    if (f[j].cot) {
      form |= 1u << j;
      const C p0 = f[j].p0;
      f[j].p0 = f[j].p1;
      f[j].p1 = neg(p0);
      f[j].k = -f[j].k;
    }
    if (f[j].e.re != 1.0 || f[j].e.im != 0.0) pre = 1;
    blk[64 + j] = f[j].k;
  }
  for (int i = 0; i < 16; ++i) {
    C post = mk(1), pe = mk(1);
    for (int j = 0; j < r && j < 4; ++j) {
      if (!has[j]) continue;
      const bool one = (i >> j) & 1;
      post = mul(post, one ? f[j].p1 : f[j].p0);
      if (one) pe = mul(pe, f[j].e);
    }
    blk[2 * i] = post.re;
    blk[2 * i + 1] = post.im;
    blk[32 + 2 * i] = pe.re;
    blk[32 + 2 * i + 1] = pe.im;
  }
  blk[68] = form;
  blk[69] = pre;
}

// Stores a scalar of a coefficient row; entries 68 and 69 of a factored block
// are raw 32-bit words in the scalar's low bytes.
template <class T>
__host__ __device__ inline void put_raw(T* o, uint32_t w) {
  uint32_t* p = reinterpret_cast<uint32_t*>(o);
  p[0] = w;
  if (sizeof(T) == 8) p[1] = 0;
}

}  // namespace cm
}  // namespace qsim

#pragma float_control(pop)
