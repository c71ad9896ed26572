// Exact perturbed predicates for the kinetic hull, device side.
//
// Points are int4 (x, y, z, i): lattice coordinates (|c| <= 2^29) and the
// 0-based input index i (< 2^26) that drives the symbolic perturbation
//   p~ = (x + e1*i, y + e2*i^2, z + e3*i^3),   1 >> e1 >> e2 >> e3 > 0.
// The paper uses floating-point coordinates and does not treat ties (Sec. 3,
// Fig. "point_datatypes"); this perturbation is the project's reading.
//
// For a rank-ordered triple (a, b, c):
//   D = D0 + e1 D1 + e2 D2 + e1e2 D12    (xy orientation, z of (b-a)x(c-a))
//   N = N0 + e1 N1 + e3 N3 + e1e3 N13    (xz orientation; negated for the
//                                         upper run, z -> -z)
// and the kinetic event time (the paper's time() of Fig.
// "time_calculations") is tau = N / D: the time at which the three points,
// placed at (x, z - t*y), become collinear.  Two times compare through
// sign(tau_A - tau_B) = sign(N_A D_B - N_B D_A) sign(D_A) sign(D_B), whose
// 12 epsilon coefficients are taken in decreasing order of size.
//
// Fast path: the "standard part" of tau (its real limit as e -> 0), computed
// in double and stored with every event rounded to float.  Two standard parts
// that differ by more than a proven rounding bound decide the order; anything
// closer, equal, infinite on both sides or not covered goes to the exact
// cascade (int128, then 256-bit).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace hull {

typedef __int128 i128;
typedef unsigned __int128 u128;

struct Tri {
  int a, w, b;  // ranks, a < w < b
};

// A point of the wide coordinate range, |x|, |y| <= 2^30 and |z| <= 2^42 (the
// lifted points of a Delaunay triangulation, float input on a 30-bit
// lattice); w is the index within the hull, as in the int4 (x, y, z, w) of
// the standard range.
struct __align__(16) WPt {
  int x, y, w, pad;
  long long z;
  long long pad2;
};

// Range of each coordinate: int32 rows, |c| <= 2^29; int64 rows (the wide
// range), |x|, |y| <= 2^30 and |z| <= 2^42.
__device__ __forceinline__ bool pt_out_of_range(int32_t x, int32_t y, int32_t z) {
  return (x > kMaxCoord) | (x < -kMaxCoord) | (y > kMaxCoord) | (y < -kMaxCoord) |
         (z > kMaxCoord) | (z < -kMaxCoord);
}
__device__ __forceinline__ bool pt_out_of_range(int64_t x, int64_t y, int64_t z) {
  return (x > kMaxWideXY) | (x < -kMaxWideXY) | (y > kMaxWideXY) | (y < -kMaxWideXY) |
         (z > kMaxWideZ) | (z < -kMaxWideZ);
}

// A point by rank: int4 (x, y, z, index within the hull) from int32 rows, WPt
// from int64 rows (x and y of a row in range fit int32).
__device__ __forceinline__ int4 make_pt(const int32_t* xyz, int64_t i, int local) {
  return make_int4(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], local);
}
__device__ __forceinline__ WPt make_pt(const int64_t* xyz, int64_t i, int local) {
  WPt q;
  q.x = (int)xyz[3 * i];
  q.y = (int)xyz[3 * i + 1];
  q.w = local;
  q.pad = 0;
  q.z = xyz[3 * i + 2];
  q.pad2 = 0;
  return q;
}

// ---------------------------------------------------------------------------
// 256-bit signed accumulator: value = hi * 2^128 + lo (lo unsigned).
// ---------------------------------------------------------------------------
struct W256 {
  i128 hi;
  u128 lo;
};

__device__ __forceinline__ W256 w_zero() { return W256{0, 0}; }

// Full 128 x 128 -> 256 signed product.
__device__ __noinline__ W256 w_mul(i128 x, i128 y) {
  bool neg = (x < 0) != (y < 0);
  u128 ux = x < 0 ? (u128)(-x) : (u128)x;
  u128 uy = y < 0 ? (u128)(-y) : (u128)y;
  uint64_t x0 = (uint64_t)ux, x1 = (uint64_t)(ux >> 64);
  uint64_t y0 = (uint64_t)uy, y1 = (uint64_t)(uy >> 64);
  u128 p00 = (u128)x0 * y0, p01 = (u128)x0 * y1, p10 = (u128)x1 * y0, p11 = (u128)x1 * y1;
  u128 mid = (p00 >> 64) + (uint64_t)p01 + (uint64_t)p10;
  u128 lo = ((u128)(uint64_t)mid << 64) | (uint64_t)p00;
  u128 hi = p11 + (p01 >> 64) + (p10 >> 64) + (mid >> 64);
  W256 r;
  if (!neg) {
    r.hi = (i128)hi;
    r.lo = lo;
  } else {  // two's complement negation of (hi, lo)
    u128 nlo = ~lo + 1;
    u128 nhi = ~hi + (nlo == 0 ? 1 : 0);
    r.hi = (i128)nhi;
    r.lo = nlo;
  }
  return r;
}

__device__ __forceinline__ W256 w_add(W256 x, W256 y) {
  W256 r;
  r.lo = x.lo + y.lo;
  r.hi = x.hi + y.hi + (r.lo < x.lo ? 1 : 0);
  return r;
}

__device__ __forceinline__ W256 w_sub(W256 x, W256 y) {
  W256 r;
  r.lo = x.lo - y.lo;
  r.hi = x.hi - y.hi - (x.lo < y.lo ? 1 : 0);
  return r;
}

__device__ __forceinline__ int w_sign(W256 x) {
  if (x.hi < 0) return -1;
  if (x.hi > 0 || x.lo != 0) return 1;
  return 0;
}

template <typename T>
__device__ __forceinline__ int sgn(T v) {
  return (v > 0) - (v < 0);
}

// ---------------------------------------------------------------------------
// Coefficients of D and N for one triple (exact, cold path).
// ---------------------------------------------------------------------------
struct Coef {
  i128 d[4];  // D0, D1, D2, D12
  i128 n[4];  // N0, N1, N3, N13
  int dsign;  // sign of the perturbed D (never 0 for distinct indices)
};

// Both point types: every difference fits int64 (|dx|, |dy| <= 2^31, |dz| <=
// 2^43) and every coefficient int128 (at most 2^110 on the wide range).
template <class PT>
__device__ __noinline__ void coef_of(PT P, PT Q, PT R, int zs, Coef& c) {
  int64_t dx1 = (int64_t)Q.x - P.x, dx2 = (int64_t)R.x - P.x;
  int64_t dy1 = (int64_t)Q.y - P.y, dy2 = (int64_t)R.y - P.y;
  int64_t dz1 = (int64_t)Q.z - P.z, dz2 = (int64_t)R.z - P.z;
  int64_t ia = P.w, ib = Q.w, ic = R.w;
  int64_t di1 = ib - ia, di2 = ic - ia;
  // squares / cubes of the index differences for the e2 and e3 columns
  i128 sq1 = (i128)ib * ib - (i128)ia * ia, sq2 = (i128)ic * ic - (i128)ia * ia;
  i128 cu1 = (i128)ib * ib * ib - (i128)ia * ia * ia;
  i128 cu2 = (i128)ic * ic * ic - (i128)ia * ia * ia;
  c.d[0] = (i128)dx1 * dy2 - (i128)dx2 * dy1;
  c.d[1] = (i128)di1 * dy2 - (i128)di2 * dy1;
  c.d[2] = (i128)dx1 * sq2 - (i128)dx2 * sq1;
  c.d[3] = (i128)di1 * sq2 - (i128)di2 * sq1;  // = (b-a)(c-a)(c-b)
  c.n[0] = (i128)dx1 * dz2 - (i128)dx2 * dz1;
  c.n[1] = (i128)di1 * dz2 - (i128)di2 * dz1;
  c.n[2] = (i128)dx1 * cu2 - (i128)dx2 * cu1;
  c.n[3] = (i128)di1 * cu2 - (i128)di2 * cu1;  // = (b-a)(c-a)(c-b)(a+b+c)
  if (zs < 0)
    for (int k = 0; k < 4; ++k) c.n[k] = -c.n[k];
  int s = 0;
  for (int k = 0; k < 4 && s == 0; ++k) s = sgn(c.d[k]);
  c.dsign = s;
}

// sign(tau_A - tau_B), exactly.  The product N_A D_B has monomials
// e1^p e2^q e3^r, p <= 2, q <= 1, r <= 1; listed by decreasing size:
//   1       : N0 D0
//   e1      : N0 D1 + N1 D0
//   e1^2    : N1 D1
//   e2      : N0 D2
//   e1e2    : N0 D12 + N1 D2
//   e1^2e2  : N1 D12
//   e3      : N3 D0
//   e1e3    : N3 D1 + N13 D0
//   e1^2e3  : N13 D1
//   e2e3    : N3 D2
//   e1e2e3  : N3 D12 + N13 D2
//   e1^2e2e3: N13 D12
__device__ __noinline__ int tau_cmp_exact(const Coef& A, const Coef& B) {
  // index pairs (N term, D term) per monomial; -1 = unused second pair
  const signed char tab[12][4] = {
      {0, 0, -1, -1}, {0, 1, 1, 0}, {1, 1, -1, -1}, {0, 2, -1, -1},
      {0, 3, 1, 2},   {1, 3, -1, -1}, {2, 0, -1, -1}, {2, 1, 3, 0},
      {3, 1, -1, -1}, {2, 2, -1, -1}, {2, 3, 3, 2},   {3, 3, -1, -1}};
  for (int m = 0; m < 12; ++m) {
    W256 acc = w_zero();
    for (int t = 0; t < 2; ++t) {
      int ni = tab[m][2 * t], di = tab[m][2 * t + 1];
      if (ni < 0) continue;
      acc = w_add(acc, w_mul(A.n[ni], B.d[di]));
      acc = w_sub(acc, w_mul(B.n[ni], A.d[di]));
    }
    int s = w_sign(acc);
    if (s) return s * A.dsign * B.dsign;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Fast path: standard part of tau in double.
// ---------------------------------------------------------------------------
// Coordinate differences fit int32 (|coord| <= 2^29; indices < 2^26), so the
// orientation products are 32 x 32 -> 64-bit multiplies.  The subtraction is
// done in unsigned arithmetic (defined wrap-around for inputs the range check
// rejects: no merge runs on them).
__device__ __forceinline__ int dif32(int a, int b) { return (int)((unsigned)a - (unsigned)b); }
__device__ __forceinline__ int64_t mul32(int a, int b) { return (int64_t)a * (int64_t)b; }
// Returns the real limit of tau as the epsilons vanish when it is finite and
// one of the two leading cases holds (D0 != 0, or D0 = N0 = 0 and D1 != 0);
// NaN otherwise (the exact path then decides every comparison).
__device__ __forceinline__ double tau_std(int4 P, int4 Q, int4 R, int zs) {
  const int dx1 = dif32(Q.x, P.x), dx2 = dif32(R.x, P.x);
  const int dy1 = dif32(Q.y, P.y), dy2 = dif32(R.y, P.y);
  const int dz1 = dif32(Q.z, P.z), dz2 = dif32(R.z, P.z);
  const int64_t D0 = mul32(dx1, dy2) - mul32(dx2, dy1);
  const int64_t N0 = mul32(dx1, dz2) - mul32(dx2, dz1);
  if (D0 != 0) return (double)(zs * N0) / (double)D0;
  if (N0 != 0) return __builtin_nan("");
  const int di1 = Q.w - P.w, di2 = R.w - P.w;
  const int64_t D1 = mul32(di1, dy2) - mul32(di2, dy1);
  if (D1 == 0) return __builtin_nan("");
  const int64_t N1 = mul32(di1, dz2) - mul32(di2, dz1);
  return (double)(zs * N1) / (double)D1;
}

// Correctly rounded conversion of an int128 below 2^127 in magnitude: the
// top 64 bits with a sticky bit for the rest, converted once (the bits below
// the double's rounding position only decide "above half" versus "exactly
// half", and the sticky bit keeps that), then scaled exactly.
__device__ __forceinline__ double to_double(i128 v) {
  const bool neg = v < 0;
  const u128 u = neg ? (u128)(-v) : (u128)v;
  const uint64_t hi = (uint64_t)(u >> 64);
  double r;
  if (hi == 0) {
    r = (double)(uint64_t)u;
  } else {
    const int sh = 64 - __builtin_clzll(hi);
    uint64_t t = (uint64_t)(u >> sh);
    if ((u << (128 - sh)) != 0) t |= 1;
    r = ldexp((double)t, sh);
  }
  return neg ? -r : r;
}

// Standard part of tau on the wide range: D0 fits int128 (up to 2^63), N0 up
// to 2^75, D1 int64 (up to 2^58), N1 up to 2^70; each converted once
// (correctly rounded) and divided once, so the filter bound below holds as
// on the standard range.
__device__ __forceinline__ double tau_std(const WPt& P, const WPt& Q, const WPt& R, int zs) {
  const int64_t dx1 = (int64_t)Q.x - P.x, dx2 = (int64_t)R.x - P.x;
  const int64_t dy1 = (int64_t)Q.y - P.y, dy2 = (int64_t)R.y - P.y;
  const int64_t dz1 = Q.z - P.z, dz2 = R.z - P.z;
  const i128 D0 = (i128)dx1 * dy2 - (i128)dx2 * dy1;
  const i128 N0 = (i128)dx1 * dz2 - (i128)dx2 * dz1;
  if (D0 != 0) return to_double(zs * N0) / to_double(D0);
  if (N0 != 0) return __builtin_nan("");
  const int64_t di1 = Q.w - P.w, di2 = R.w - P.w;
  const int64_t D1 = di1 * dy2 - di2 * dy1;
  if (D1 == 0) return __builtin_nan("");
  const i128 N1 = (i128)di1 * dz2 - (i128)di2 * dz1;
  return to_double(zs * N1) / to_double(D1);
}

// Does the standard-part filter decide sign(tau_A - tau_B)?  Each standard
// part is a quotient of two integers below 2^76, each rounded once to double
// and divided once (relative error at most 3 * 2^-53 (1 + 2^-52)), and the
// value stored with an event is that double rounded once more to float
// (2^-24 more): the error of either kind is below 2^-24 + 2^-51 relative,
// and the quotients stay inside float's normal range (between 2^-76 and
// 2^76 in magnitude).  A gap larger than 2^-23 (|sa| + |sb|) therefore fixes
// the sign; the subtraction of two such values is exact or rounds by at most
// 2^-53 relative, which the margin covers.
__device__ __forceinline__ int std_cmp(double sa, double sb) {
  if (!(sa == sa) || !(sb == sb)) return 0;  // NaN: not covered
  double d = sa - sb;
  double tol = 0x1p-23 * (fabs(sa) + fabs(sb));
  if (d > tol) return 1;
  if (-d > tol) return -1;
  return 0;
}

}  // namespace hull
