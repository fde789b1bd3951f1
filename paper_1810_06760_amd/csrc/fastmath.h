// Table-driven FP64 complex exponential for bounded arguments:
//   cexp_neg(g, phi) = exp(-g) (cos phi + i sin phi),  0 <= g <~ 700, |phi| < 2^20 pi/32.
//
// exp: Tang's table-driven method.  x = -g = (64 m + j) ln2/64 + r with
//   |r| <= ln2/128, so exp(x) = 2^m 2^{j/64} (1 + r + r^2/2 + ... + r^5/120);
//   the omitted r^6/720 term is below 4e-17 relative.
// sin/cos: reduction by multiples of pi/32 (three-part Cody-Waite constant),
//   |r| <= pi/64, Taylor polynomials of r (through r^9 for sin, r^8 for cos,
//   truncation below 1e-17), then the angle-addition formulas with
//   sin(j pi/32), cos(j pi/32) from a 64-entry table.
// The tables are filled per workgroup from the device library's exp2/sincos,
// so every entry is correctly rounded or within an ulp.
#pragma once

#include <hip/hip_runtime.h>

namespace fga {

struct TrigTables {
  double e2[64];    // 2^(j/64)
  double sn[64];    // sin(j pi/32)
  double cs[64];    // cos(j pi/32)
};

// Fill the tables; call from every thread of the block, then __syncthreads().
__device__ __forceinline__ void fill_tables(TrigTables &t)
{
  for (int j = threadIdx.x; j < 64; j += blockDim.x) {
    t.e2[j] = exp2((double)j / 64.0);
    double s, c;
    sincospi((double)j / 32.0, &s, &c);
    t.sn[j] = s;
    t.cs[j] = c;
  }
}

// 64/ln2, ln2/64 split so that k*LN2_64_HI is exact for |k| < 2^20
// (hi has 32 significant bits; hi + lo = ln2/64 to ~1e-29).
constexpr double INV_LN2_64 = 92.33248261689366;
constexpr double LN2_64_HI = 0.010830424696905538;
constexpr double LN2_64_LO = -6.563929801064195e-13;
// 32/pi and pi/32 in three parts (hi and mid with 32 significant bits).
constexpr double INV_PI_32 = 10.185916357881302;
constexpr double PI_32_HI = 0.09817477042088285;
constexpr double PI_32_MID = 3.798187816439979e-12;
constexpr double PI_32_LO = 1.2639164054974691e-22;

__device__ __forceinline__ void cexp_neg(const TrigTables &t, double g, double phi, double &re, double &im)
{
  // exp(-g)
  const double x = -g;
  const double kd = rint(x * INV_LN2_64);
  const int k = (int)kd;
  const int j = k & 63;
  const int m = (k - j) >> 6;
  double r = fma(-kd, LN2_64_HI, x);
  r = fma(-kd, LN2_64_LO, r);
  double q = fma(r, 1.0 / 120.0, 1.0 / 24.0);
  q = fma(r, q, 1.0 / 6.0);
  q = fma(r, q, 0.5);
  q = fma(r, q, 1.0);
  q = q * r;  // p(r) - 1
  const double tj = t.e2[j];
  const double ex = ldexp(fma(tj, q, tj), m);
  // sin / cos
  const double nd = rint(phi * INV_PI_32);
  const int n = (int)nd & 63;
  double u = fma(-nd, PI_32_HI, phi);
  u = fma(-nd, PI_32_MID, u);
  u = fma(-nd, PI_32_LO, u);
  const double u2 = u * u;
  double sp = fma(u2, 1.0 / 362880.0, -1.0 / 5040.0);
  sp = fma(u2, sp, 1.0 / 120.0);
  sp = fma(u2, sp, -1.0 / 6.0);
  const double su = fma(u * u2, sp, u);
  double cp = fma(u2, 1.0 / 40320.0, -1.0 / 720.0);
  cp = fma(u2, cp, 1.0 / 24.0);
  cp = fma(u2, cp, -0.5);
  const double cu = fma(u2, cp, 1.0);
  const double sj = t.sn[n], cj = t.cs[n];
  const double sphi = fma(su, cj, cu * sj);
  const double cphi = fma(cu, cj, -(su * sj));
  re = ex * cphi;
  im = ex * sphi;
}

}  // namespace fga
