// The FP64 right-hand side of the FGA ODE system and the classic RK4 step,
// shared by the integrator and the interface step.  The right-hand side is,
// for sigma = +1 / -1 (Sec. 2.2):
//   dQ/dt = sigma c P/|P|,  dP/dt = -sigma |P| grad c         (eq:char_plus, eq:char_minus)
//   d(dzQ)/dt = sigma [dzQ (grad c (x) P)/|P| + c dzP (I - P (x) P/|P|^2)/|P|]
//   d(dzP)/dt = sigma [-|P| dzQ Hess c - dzP (P (x) grad c)/|P|]   (eq:DzDt)
//   da_P/dt = a_P (sigma grad c . P/|P| + tr(Z^{-1} dZ/dt)/2)       (eq:amp_P)
//   d(a_SV, a_SH)/dt = s (a_SV, a_SH) + omega (-a_SH, a_SV),
//     omega = dN_SH/dt . N_SV = sigma (P.e) e.(grad c x P)/|e x P|^2  (eq:amp_SV, eq:amp_SH)
//   dS/dt = P . dQ/dt - sigma c |P|
// tr(Z^{-1} dZ/dt) is formed as (sum_ij cof(Z)_ij dZ_ij) / det Z, so no
// matrix inverse is built.  Frame-free S amplitudes (SV = 1): the physical
// polarisation A = a_SV N_SV + a_SH N_SH is advanced instead, by
//   dA/dt = s A - (A . dPhat/dt) Phat,  dPhat/dt = (dP/dt - Phat (Phat . dP/dt))/|P|,
// which is the framed system with the frame's rotation differentiated out.
#pragma once

#include "device_common.h"

namespace fga {
namespace rk {

constexpr int NS = 47;
enum { IQ = 0, IP = 3, IZQR = 6, IZQI = 15, IZPR = 24, IZPI = 33, IA = 42, IS = 46 };
// frame-free S state: A_x at IA, IA+1, A_y at IA+2, IA+3, A_z at IAZ, IAZ+1
constexpr int IAZ = 47;
template <int SV> constexpr int nstate() { return SV ? 49 : NS; }
constexpr double COS10 = 0.98480775301220805936;  // cos(10 degrees)

// One RK4 stage: k = f(yt); acc += wacc*k; yt <- y + cnext*k in place.  The
// derivative is folded in as soon as each group of components is complete,
// row by row for dzQ/dzP, so the live state stays at y, acc and yt.
template <int MK, int SV = 0>
__device__ __forceinline__ void stage(const DevMedium &med, int sp, int layer, double sg, bool isS,
                                      const double e[3], const double *__restrict__ y, double *__restrict__ yt,
                                      double *__restrict__ acc, double wacc, double cnext,
                                      const MedBlock *blk = nullptr)
{
  double c, g[3], H6[6];
  medium_eval<MK>(med, sp, layer, yt + IQ, c, g, H6, blk);
  const double H[3][3] = {{H6[0], H6[3], H6[4]}, {H6[3], H6[1], H6[5]}, {H6[4], H6[5], H6[2]}};
  const double P0 = yt[IP], P1 = yt[IP + 1], P2 = yt[IP + 2];
  const double np = sqrt(P0 * P0 + P1 * P1 + P2 * P2);
  const double inp = 1.0 / np;
  const double ph[3] = {P0 * inp, P1 * inp, P2 * inp};
  const double sc = sg * c;
  const double ci = sc * inp;

  // cofactors of Z = dzQ + i dzP and det Z (cyclic index form carries the sign)
  double Cr[9], Ci[9];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
      const int a = 3 * i1 + j1, b = 3 * i2 + j2, cc = 3 * i1 + j2, d = 3 * i2 + j1;
      const double ar = yt[IZQR + a] - yt[IZPI + a], ai = yt[IZQI + a] + yt[IZPR + a];
      const double br = yt[IZQR + b] - yt[IZPI + b], bi = yt[IZQI + b] + yt[IZPR + b];
      const double cr = yt[IZQR + cc] - yt[IZPI + cc], cim = yt[IZQI + cc] + yt[IZPR + cc];
      const double dr = yt[IZQR + d] - yt[IZPI + d], di = yt[IZQI + d] + yt[IZPR + d];
      Cr[3 * i + j] = (ar * br - ai * bi) - (cr * dr - cim * di);
      Ci[3 * i + j] = (ar * bi + ai * br) - (cr * di + cim * dr);
    }
  }
  double detr = 0.0, deti = 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const double zr = yt[IZQR + j] - yt[IZPI + j], zi = yt[IZQI + j] + yt[IZPR + j];
    detr += zr * Cr[j] - zi * Ci[j];
    deti += zr * Ci[j] + zi * Cr[j];
  }

  double Tr = 0.0, Ti = 0.0;
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const double ur = yt[IZQR + 3 * m] * g[0] + yt[IZQR + 3 * m + 1] * g[1] + yt[IZQR + 3 * m + 2] * g[2];
    const double ui = yt[IZQI + 3 * m] * g[0] + yt[IZQI + 3 * m + 1] * g[1] + yt[IZQI + 3 * m + 2] * g[2];
    const double vr = yt[IZPR + 3 * m] * ph[0] + yt[IZPR + 3 * m + 1] * ph[1] + yt[IZPR + 3 * m + 2] * ph[2];
    const double vi = yt[IZPI + 3 * m] * ph[0] + yt[IZPI + 3 * m + 1] * ph[1] + yt[IZPI + 3 * m + 2] * ph[2];
    double kq_r[3], kq_i[3], kp_r[3], kp_i[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int o = 3 * m + j;
      kq_r[j] = sg * ur * ph[j] + ci * (yt[IZPR + o] - vr * ph[j]);
      kq_i[j] = sg * ui * ph[j] + ci * (yt[IZPI + o] - vi * ph[j]);
      const double hr = yt[IZQR + 3 * m] * H[0][j] + yt[IZQR + 3 * m + 1] * H[1][j] + yt[IZQR + 3 * m + 2] * H[2][j];
      const double hi = yt[IZQI + 3 * m] * H[0][j] + yt[IZQI + 3 * m + 1] * H[1][j] + yt[IZQI + 3 * m + 2] * H[2][j];
      kp_r[j] = -sg * (np * hr + vr * g[j]);
      kp_i[j] = -sg * (np * hi + vi * g[j]);
      // dZ = d(dzQ) + i d(dzP); T += cof(Z) : dZ
      const double dr = kq_r[j] - kp_i[j], di = kq_i[j] + kp_r[j];
      Tr += Cr[o] * dr - Ci[o] * di;
      Ti += Cr[o] * di + Ci[o] * dr;
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int o = 3 * m + j;
      const double kk[4] = {kq_r[j], kq_i[j], kp_r[j], kp_i[j]};
      const int base[4] = {IZQR, IZQI, IZPR, IZPI};
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int f = base[t] + o;
        acc[f] += wacc * kk[t];
        yt[f] = y[f] + cnext * kk[t];
      }
    }
  }
  const double idd = 1.0 / (detr * detr + deti * deti);
  const double trr = (Tr * detr + Ti * deti) * idd;
  const double tri = (Ti * detr - Tr * deti) * idd;
  const double sr = sg * (g[0] * ph[0] + g[1] * ph[1] + g[2] * ph[2]) + 0.5 * trr;
  const double si = 0.5 * tri;
  double ka[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (SV && isS) {
    // parallel transport of A: dPhat/dt from dP/dt = -sigma |P| grad c
    const double dq0 = -sg * g[0], dq1 = -sg * g[1], dq2 = -sg * g[2];   // (dP/dt)/|P|
    const double pd = ph[0] * dq0 + ph[1] * dq1 + ph[2] * dq2;
    const double dph[3] = {dq0 - ph[0] * pd, dq1 - ph[1] * pd, dq2 - ph[2] * pd};
    const double Ar[3] = {yt[IA], yt[IA + 2], yt[IAZ]}, Ai[3] = {yt[IA + 1], yt[IA + 3], yt[IAZ + 1]};
    const double adr = Ar[0] * dph[0] + Ar[1] * dph[1] + Ar[2] * dph[2];
    const double adi = Ai[0] * dph[0] + Ai[1] * dph[1] + Ai[2] * dph[2];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      ka[2 * c] = sr * Ar[c] - si * Ai[c] - adr * ph[c];
      ka[2 * c + 1] = sr * Ai[c] + si * Ar[c] - adi * ph[c];
    }
  } else {
    const double a0r = yt[IA], a0i = yt[IA + 1], a1r = yt[IA + 2], a1i = yt[IA + 3];
    if (!isS) {
      ka[0] = sr * a0r - si * a0i;
      ka[1] = sr * a0i + si * a0r;
      ka[2] = 0.0;
      ka[3] = 0.0;
    } else {
      const double gx0 = g[1] * P2 - g[2] * P1, gx1 = g[2] * P0 - g[0] * P2, gx2 = g[0] * P1 - g[1] * P0;
      const double egp = e[0] * gx0 + e[1] * gx1 + e[2] * gx2;
      const double pe = P0 * e[0] + P1 * e[1] + P2 * e[2];
      const double x0 = e[1] * P2 - e[2] * P1, x1 = e[2] * P0 - e[0] * P2, x2 = e[0] * P1 - e[1] * P0;
      const double om = sg * pe * egp / (x0 * x0 + x1 * x1 + x2 * x2);
      ka[0] = sr * a0r - si * a0i - om * a1r;
      ka[1] = sr * a0i + si * a0r - om * a1i;
      ka[2] = sr * a1r - si * a1i + om * a0r;
      ka[3] = sr * a1i + si * a1r + om * a0i;
    }
  }
  double kr[7];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    kr[j] = sc * ph[j];
    kr[3 + j] = -sg * np * g[j];
  }
  kr[6] = P0 * kr[0] + P1 * kr[1] + P2 * kr[2] - sc * np;
  const int fr[7] = {IQ, IQ + 1, IQ + 2, IP, IP + 1, IP + 2, IS};
#pragma unroll
  for (int t = 0; t < (SV ? 6 : 4); ++t) {
    const int f = t < 4 ? IA + t : IAZ + t - 4;
    acc[f] += wacc * ka[t];
    yt[f] = y[f] + cnext * ka[t];
  }
#pragma unroll
  for (int t = 0; t < 7; ++t) {
    const int f = fr[t];
    acc[f] += wacc * kr[t];
    yt[f] = y[f] + cnext * kr[t];
  }
}

// After a step: an S beam whose P has come within 10 degrees of its frame
// axis switches axis (e_z <-> e_x) and re-expresses (a_SV, a_SH) so that the
// physical polarisation a_SV N_SV + a_SH N_SH is unchanged.
__device__ __forceinline__ void reframe_s(const double P[3], double A[4], double e[3])
{
  const double np = sqrt(P[0] * P[0] + P[1] * P[1] + P[2] * P[2]);
  const double pe = P[0] * e[0] + P[1] * e[1] + P[2] * e[2];
  if (fabs(pe) / np > COS10) {
    double nsh[3], nsv[3];
    s_frame(P, e, nsh, nsv);
    double Ar[3], Ai[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Ar[c] = A[0] * nsv[c] + A[2] * nsh[c];
      Ai[c] = A[1] * nsv[c] + A[3] * nsh[c];
    }
    const bool was_z = e[2] != 0.0 && e[0] == 0.0 && e[1] == 0.0;
    e[0] = was_z ? 1.0 : 0.0;
    e[1] = 0.0;
    e[2] = was_z ? 0.0 : 1.0;
    s_frame(P, e, nsh, nsv);
    A[0] = Ar[0] * nsv[0] + Ar[1] * nsv[1] + Ar[2] * nsv[2];
    A[1] = Ai[0] * nsv[0] + Ai[1] * nsv[1] + Ai[2] * nsv[2];
    A[2] = Ar[0] * nsh[0] + Ar[1] * nsh[1] + Ar[2] * nsh[2];
    A[3] = Ai[0] * nsh[0] + Ai[1] * nsh[1] + Ai[2] * nsh[2];
  }
}

__device__ __forceinline__ void reframe_s(double *y, double e[3]) { reframe_s(y + IP, y + IA, e); }

// One classic RK4 step of size dt in place, y' = y + dt/6 (k1 + 2 k2 + 2 k3 + k4);
// the four stages run as a loop so that only y, acc and the stage input stay live.
// SV = 1: frame-free S amplitudes (y holds nstate<1>() values); after the
// step A is projected on the plane orthogonal to the new P, which the exact
// solution never leaves (the projection removes the step's truncation drift).
template <int MK, int SV = 0>
__device__ __forceinline__ void rk4_step(const DevMedium &med, int sp, int layer, double sg, bool isS,
                                         const double e[3], double *y, double dt, const MedBlock *blk = nullptr)
{
  constexpr int N = nstate<SV>();
  double acc[N], yt[N];
#pragma unroll
  for (int f = 0; f < N; ++f) { yt[f] = y[f]; acc[f] = 0.0; }
  const double h2 = 0.5 * dt, h6 = dt / 6.0;
#pragma nounroll
  for (int st = 0; st < 4; ++st) {
    const double wacc = (st == 0 || st == 3) ? 1.0 : 2.0;
    const double cnext = st == 2 ? dt : (st == 3 ? 0.0 : h2);
    stage<MK, SV>(med, sp, layer, sg, isS, e, y, yt, acc, wacc, cnext, blk);
  }
#pragma unroll
  for (int f = 0; f < N; ++f) y[f] += h6 * acc[f];
  if (SV && isS) {
    const double inp = 1.0 / sqrt(y[IP] * y[IP] + y[IP + 1] * y[IP + 1] + y[IP + 2] * y[IP + 2]);
    const double ph[3] = {y[IP] * inp, y[IP + 1] * inp, y[IP + 2] * inp};
    const double apr = y[IA] * ph[0] + y[IA + 2] * ph[1] + y[IAZ] * ph[2];
    const double api = y[IA + 1] * ph[0] + y[IA + 3] * ph[1] + y[IAZ + 1] * ph[2];
    y[IA] -= apr * ph[0];
    y[IA + 2] -= apr * ph[1];
    y[IAZ] -= apr * ph[2];
    y[IA + 1] -= api * ph[0];
    y[IA + 3] -= api * ph[1];
    y[IAZ + 1] -= api * ph[2];
  }
}

// The pieces of the classic RK4 step where grad c = 0 (a homogeneous medium,
// or inside one layer of a layered medium).  There P and dzP have zero
// derivative and Q, dzQ and S constant ones, so every stage's derivative of
// those equals the first; only the amplitudes' derivative depends on the
// stage, through Z = dzQ + i dzP at the stage input in tr(Z^{-1} dZ/dt).
// Since dzP is fixed, Z at a stage input is Z0 + c K with Z0 = Z at the step's
// start and K = d(dzQ)/dt.  The stage formulas, weights and summation order
// are those of rk4_step with the medium's gradient and Hessian at zero
// (omega = 0 for S beams), so the two agree to rounding.

// y0 + dt/6 (k + 2k + 2k + k) for a derivative equal in all four stages,
// summed in rk4_step's order.
__device__ __forceinline__ double rk4_const(double y0, double k, double h6)
{
  return y0 + h6 * (((k + 2.0 * k) + 2.0 * k) + k);
}

// dQ/dt and dS/dt for speed c (eq:char_plus, eq:char_minus); also P/|P| and
// sigma c / |P| for the Jacobian rates.
__device__ __forceinline__ void pc_ray_rates(double c, double sg, const double P[3], double kQ[3], double &kS,
                                             double ph[3], double &ci)
{
  const double np = sqrt(P[0] * P[0] + P[1] * P[1] + P[2] * P[2]);
  const double inp = 1.0 / np;
  ph[0] = P[0] * inp;
  ph[1] = P[1] * inp;
  ph[2] = P[2] * inp;
  const double sc = sg * c;
  ci = sc * inp;
#pragma unroll
  for (int j = 0; j < 3; ++j) kQ[j] = sc * ph[j];
  kS = P[0] * kQ[0] + P[1] * kQ[1] + P[2] * kQ[2] - sc * np;
}

// d(dzQ)/dt = sigma c dzP (I - P (x) P/|P|^2)/|P| (eq:DzDt with grad c = 0),
// rows m, real and imaginary parts; dzr/dzi are dzP's.
__device__ __forceinline__ void pc_jac_rates(const double ph[3], double ci, const double dzr[9],
                                             const double dzi[9], double kr[9], double ki[9])
{
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const double vr = dzr[3 * m] * ph[0] + dzr[3 * m + 1] * ph[1] + dzr[3 * m + 2] * ph[2];
    const double vi = dzi[3 * m] * ph[0] + dzi[3 * m + 1] * ph[1] + dzi[3 * m + 2] * ph[2];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      kr[3 * m + j] = ci * (dzr[3 * m + j] - vr * ph[j]);
      ki[3 * m + j] = ci * (dzi[3 * m + j] - vi * ph[j]);
    }
  }
}

// The four stages of the amplitudes (eq:amp_P, eq:amp_SV, eq:amp_SH with
// grad c = 0: da/dt = a tr(Z^{-1} dZ/dt)/2), a[4] = (re, im) of a_P or of
// (a_SV, a_SH), advanced in place.
__device__ __forceinline__ void pc_amplitude(const double z0r[9], const double z0i[9], const double kr[9],
                                             const double ki[9], bool isS, double a0[4], double dt)
{
  const double h2 = 0.5 * dt, h6 = dt / 6.0;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  double a[4] = {a0[0], a0[1], a0[2], a0[3]};  // stage input
#pragma nounroll
  for (int st = 0; st < 4; ++st) {
    const double cs = st == 0 ? 0.0 : (st == 3 ? dt : h2);  // this stage's input: Z0 + cs K
    const double wacc = (st == 0 || st == 3) ? 1.0 : 2.0;
    const double cnext = st == 2 ? dt : (st == 3 ? 0.0 : h2);
    double zr[9], zi[9];
#pragma unroll
    for (int o = 0; o < 9; ++o) {
      zr[o] = z0r[o] + cs * kr[o];
      zi[o] = z0i[o] + cs * ki[o];
    }
    // cofactors (cyclic index form), det Z and T = cof(Z) : dZ/dt, dZ/dt = K
    double detr = 0.0, deti = 0.0, Tr = 0.0, Ti = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
        const int ia = 3 * i1 + j1, ib = 3 * i2 + j2, ic = 3 * i1 + j2, id = 3 * i2 + j1;
        const double Cr = (zr[ia] * zr[ib] - zi[ia] * zi[ib]) - (zr[ic] * zr[id] - zi[ic] * zi[id]);
        const double Ci = (zr[ia] * zi[ib] + zi[ia] * zr[ib]) - (zr[ic] * zi[id] + zi[ic] * zr[id]);
        if (i == 0) {
          detr += zr[j] * Cr - zi[j] * Ci;
          deti += zr[j] * Ci + zi[j] * Cr;
        }
        Tr += Cr * kr[3 * i + j] - Ci * ki[3 * i + j];
        Ti += Cr * ki[3 * i + j] + Ci * kr[3 * i + j];
      }
    }
    const double idd = 1.0 / (detr * detr + deti * deti);
    const double sr = 0.5 * ((Tr * detr + Ti * deti) * idd);
    const double si = 0.5 * ((Ti * detr - Tr * deti) * idd);
    double ka[4];
    ka[0] = sr * a[0] - si * a[1];
    ka[1] = sr * a[1] + si * a[0];
    ka[2] = isS ? sr * a[2] - si * a[3] : 0.0;
    ka[3] = isS ? sr * a[3] + si * a[2] : 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      acc[t] += wacc * ka[t];
      a[t] = a0[t] + cnext * ka[t];
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) a0[t] += h6 * acc[t];
}

// One classic RK4 step of the whole state y where grad c = 0, in place.
template <int MK>
__device__ __forceinline__ void rk4_step_pc(const DevMedium &med, int sp, int layer, double sg, bool isS, double *y,
                                            double dt)
{
  double c, g[3], H6[6];
  medium_eval<MK>(med, sp, layer, y + IQ, c, g, H6);
  double kQ[3], kS, ph[3], ci, kr[9], ki[9], z0r[9], z0i[9];
  pc_ray_rates(c, sg, y + IP, kQ, kS, ph, ci);
  pc_jac_rates(ph, ci, y + IZPR, y + IZPI, kr, ki);
#pragma unroll
  for (int o = 0; o < 9; ++o) {
    z0r[o] = y[IZQR + o] - y[IZPI + o];
    z0i[o] = y[IZQI + o] + y[IZPR + o];
  }
  pc_amplitude(z0r, z0i, kr, ki, isS, y + IA, dt);
  const double h6 = dt / 6.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) y[IQ + j] = rk4_const(y[IQ + j], kQ[j], h6);
#pragma unroll
  for (int o = 0; o < 9; ++o) {
    y[IZQR + o] = rk4_const(y[IZQR + o], kr[o], h6);
    y[IZQI + o] = rk4_const(y[IZQI + o], ki[o], h6);
  }
  y[IS] = rk4_const(y[IS], kS, h6);
}

}  // namespace rk
}  // namespace fga
