// Table-driven FP64 complex exponential for bounded arguments:
//   cexp_neg(g, phi) = exp(-g) (cos phi + i sin phi),  0 <= g <~ 700 (larger g: exactly 0 up to g ~ 2800),
//   |phi| < 2^20 pi/128.
//
// exp: Tang's table-driven method.  x = -g = (256 m + j) ln2/256 + r with
//   |r| <= ln2/512, so exp(x) = 2^m 2^{j/256} (1 + r + r^2/2 + r^3/6 + r^4/24);
//   the omitted r^5/120 term is below 4e-17 relative.
// sin/cos: reduction by multiples of pi/128 (three-part Cody-Waite constant),
//   |r| <= pi/256, Taylor polynomials of r (through r^5 for sin, r^6 for cos,
//   truncation below 1e-17 absolute), then the angle-addition formulas with
//   sin(j pi/128), cos(j pi/128) from a 256-entry table.
// The tables are filled per workgroup from the device library's exp2/sincos,
// so every entry is correctly rounded or within an ulp.
//
// cexp_neg_units takes the phase in units of pi/128 (v = phi 128/pi, so the
// reduction is v - rint(v) with no constant to split) and a mask; both
// roundings to an integer add 1.5 2^52, which leaves round-to-nearest(x) in
// the low mantissa bits for |x| < 2^51.
#pragma once

#include <hip/hip_runtime.h>

namespace fga {

constexpr int TRIG_N = 256;
struct TrigTables {
  double e2[TRIG_N];    // 2^(j/256)
  double2 sc[TRIG_N];   // (sin(j pi/128), cos(j pi/128)): one 16-byte read per lookup
};

// Fill the tables; call from every thread of the block, then __syncthreads().
__device__ __forceinline__ void fill_tables(TrigTables &t)
{
  for (int j = threadIdx.x; j < TRIG_N; j += blockDim.x) {
    t.e2[j] = exp2((double)j / 256.0);
    double s, c;
    sincospi((double)j / 128.0, &s, &c);
    t.sc[j] = make_double2(s, c);
  }
}

// 256/ln2, ln2/256 split so that k*LN2_256_HI is exact for |k| < 2^20
// (hi has 32 significant bits; hi + lo = ln2/256 to ~5e-30).
constexpr double INV_LN2_256 = 369.3299304675746;
constexpr double LN2_256_HI = 0.0027076061742263846;
constexpr double LN2_256_LO = -1.6409824502660487e-13;
// 128/pi and pi/128 in three parts (hi and mid with 32 significant bits).
constexpr double INV_PI_128 = 40.74366543152521;
constexpr double PI_128_HI = 0.024543692605220713;
constexpr double PI_128_MID = 9.495469541099947e-13;
constexpr double PI_128_LO = 3.159791013743673e-23;

__device__ __forceinline__ void cexp_neg(const TrigTables &t, double g, double phi, double &re, double &im)
{
  // exp(-g)
  const double x = -g;
  const double kd = rint(x * INV_LN2_256);
  const int k = (int)kd;
  const int j = k & (TRIG_N - 1);
  const int m = (k - j) >> 8;
  double r = fma(-kd, LN2_256_HI, x);
  r = fma(-kd, LN2_256_LO, r);
  double q = fma(r, 1.0 / 24.0, 1.0 / 6.0);
  q = fma(r, q, 0.5);
  q = fma(r, q, 1.0);
  q = q * r;  // p(r) - 1
  const double tj = t.e2[j];
  const double ex = ldexp(fma(tj, q, tj), m);
  // sin / cos
  const double nd = rint(phi * INV_PI_128);
  const int n = (int)nd & (TRIG_N - 1);
  double u = fma(-nd, PI_128_HI, phi);
  u = fma(-nd, PI_128_MID, u);
  u = fma(-nd, PI_128_LO, u);
  const double u2 = u * u;
  const double sp = fma(u2, 1.0 / 120.0, -1.0 / 6.0);
  const double su = fma(u * u2, sp, u);
  double cp = fma(u2, -1.0 / 720.0, 1.0 / 24.0);
  cp = fma(u2, cp, -0.5);
  const double cu = fma(u2, cp, 1.0);
  const double2 scn = t.sc[n];
  const double sj = scn.x, cj = scn.y;
  const double sphi = fma(su, cj, cu * sj);
  const double cphi = fma(cu, cj, -(su * sj));
  re = ex * cphi;
  im = ex * sphi;
}

constexpr double RND_MAGIC = 6755399441055744.0;  // 1.5 * 2^52
constexpr double PI_128 = 0.02454369260617026;      // pi/128

// in ? exp(-g) (cos(v pi/128) + i sin(v pi/128)) : 0, for 0 <= g <~ 700 and
// |v| < 2^51 where in is true; where it is false g >= 0 and v may be any
// finite values (the magnitude is replaced by 0 before it meets the phase).
__device__ __forceinline__ void cexp_neg_units(const TrigTables &t, double g, double v, bool in, double &re,
                                               double &im)
{
  // exp(-g)
  const double tk = fma(g, -INV_LN2_256, RND_MAGIC);
  const double kd = tk - RND_MAGIC;
  const int k = __double2loint(tk);
  const int j = k & (TRIG_N - 1);
  const int m = k >> 8;  // floor(k / 256)
  double r = fma(-kd, LN2_256_HI, -g);
  r = fma(-kd, LN2_256_LO, r);
  double q = fma(r, 1.0 / 24.0, 1.0 / 6.0);
  q = fma(r, q, 0.5);
  q = fma(r, q, 1.0);
  q = q * r;  // p(r) - 1
  const double tj = t.e2[j];
  double ex = ldexp(fma(tj, q, tj), m);
  ex = in ? ex : 0.0;
  // sin / cos: v - rint(v) is exact, |u| <= pi/256
  const double tn = v + RND_MAGIC;
  const double nd = tn - RND_MAGIC;
  const int n = __double2loint(tn) & (TRIG_N - 1);
  const double u = (v - nd) * PI_128;
  const double u2 = u * u;
  const double sp = fma(u2, 1.0 / 120.0, -1.0 / 6.0);
  const double su = fma(u * u2, sp, u);
  double cp = fma(u2, -1.0 / 720.0, 1.0 / 24.0);
  cp = fma(u2, cp, -0.5);
  const double cu = fma(u2, cp, 1.0);
  const double2 scn = t.sc[n];
  const double sj = scn.x, cj = scn.y;
  const double sphi = fma(su, cj, cu * sj);
  const double cphi = fma(cu, cj, -(su * sj));
  re = ex * cphi;
  im = ex * sphi;
}

}  // namespace fga
