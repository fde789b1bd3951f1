// Interface step of layered media (Sec. 3.1: eq:p:int, eq:Yilmaz,
// eq:Inter_DzQDzP), run after every integrator step.
//
// The integrator leaves a beam that left its layer during the step at the
// start of the step, flagged FGA_FLAG_CROSS.  Here each such beam redoes the
// step to find where it left (speeds are constant inside a layer, so the ray
// is the straight segment Q0 -> Q1 and the crossing fraction theta is found
// exactly on it), advances theta dt, is put exactly on the interface, and
// is split into the outgoing plane-wave modes:
//   - Snell: every mode keeps the tangential momentum and the frequency
//     H = c_in |P|; transmitted modes keep the sign of the normal momentum,
//     reflected ones flip it; a mode with imaginary normal momentum is
//     evanescent and is not made (it stays in the boundary problem).
//   - Amplitudes: continuity of displacement and of traction sigma.n across
//     the interface for u = A d exp(i P.x/eps), with sigma_ij = lambda div u
//     delta_ij + mu (d_i u_j + d_j u_i).  In the local frame (e3 = normal
//     into the far layer, e1 = tangential momentum direction, e2 = e3 x e1)
//     the in-plane (P, SV) part is a 4x4 complex system for (R_P, R_S, T_P,
//     T_S) and the SH part a 2x2 one; P modes are polarised along k/|k|,
//     in-plane S modes along e2 x k/|k|, SH modes along e2.
//   - Jacobians (map_jacobians): from the crossing-time constraint, the
//     Snell update P' = P + mu n(x*) with H = c|P| fixed, and the child
//     started at the crossing.  Where grad c = 0 on a plane this is
//     dzQ' = dzQ F, dzP' = dzP F^{-T}, F = I + n (x) v in any frame with third
//     axis n, v = (kappa - 1) p_t / p_n + (kappa p_n' / p_n - 1) n,
//     kappa = (c_out / c_in)^2; the turning normal of a sphere (shape
//     operator kcurv (I - n n^T), kcurv = s/R) and speed gradients add terms.
// In layers with a speed gradient rays bend: the step is the general RK4
// step, and theta is refined by four secant iterations on RK4 sub-steps.
// Children with |A_child| >= child_cut |A_in| are made (generation + 1,
// lineage FGA_LINEAGE_CHILD) and take the remaining (1 - theta) dt in their
// own layer.  The first child reuses the parent's slot; the others go after
// the current count, at offsets from a two-pass count / exclusive scan over
// workgroups, so slot assignment is deterministic.
#include <hipcub/hipcub.hpp>

#include "rk4.h"

namespace fga {
namespace {

using namespace rk;

struct cx {
  double r, i;
};
__device__ __forceinline__ cx mk(double r, double i = 0.0) { return cx{r, i}; }
__device__ __forceinline__ cx operator+(cx a, cx b) { return cx{a.r + b.r, a.i + b.i}; }
__device__ __forceinline__ cx operator-(cx a, cx b) { return cx{a.r - b.r, a.i - b.i}; }
__device__ __forceinline__ cx operator-(cx a) { return cx{-a.r, -a.i}; }
__device__ __forceinline__ cx operator*(cx a, cx b) { return cx{a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ cx operator*(double s, cx a) { return cx{s * a.r, s * a.i}; }
__device__ __forceinline__ cx operator/(cx a, cx b)
{
  const double d = b.r * b.r + b.i * b.i;
  return cx{(a.r * b.r + a.i * b.i) / d, (a.i * b.r - a.r * b.i) / d};
}
__device__ __forceinline__ double cabs2(cx a) { return a.r * a.r + a.i * a.i; }

__device__ __forceinline__ double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// A x = b for n <= 4 by Gaussian elimination with partial pivoting (by modulus).
__device__ void solve_small(int n, cx A[4][4], cx b[4], cx x[4])
{
  for (int c = 0; c < n; ++c) {
    int pv = c;
    for (int r = c + 1; r < n; ++r)
      if (cabs2(A[r][c]) > cabs2(A[pv][c])) pv = r;
    if (pv != c) {
      for (int j = 0; j < n; ++j) {
        const cx t = A[c][j];
        A[c][j] = A[pv][j];
        A[pv][j] = t;
      }
      const cx t = b[c];
      b[c] = b[pv];
      b[pv] = t;
    }
    for (int r = c + 1; r < n; ++r) {
      const cx f = A[r][c] / A[c][c];
      for (int j = c; j < n; ++j) A[r][j] = A[r][j] - f * A[c][j];
      b[r] = b[r] - f * b[c];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    cx s = b[r];
    for (int j = r + 1; j < n; ++j) s = s - A[r][j] * x[j];
    x[r] = s / A[r][r];
  }
}

// Crossing fraction of the straight segment Q0 -> Q1 with interface `iface`.
__device__ double crossing(const DevMedium &m, int iface, const double *Q0, const double *Q1)
{
  const double r = iface_level(m, iface);
  double th;
  if (m.geometry == 1) {
    const double D[3] = {Q1[0] - Q0[0], Q1[1] - Q0[1], Q1[2] - Q0[2]};
    const double a = dot3(D, D), b = dot3(Q0, D), c = dot3(Q0, Q0) - r * r;
    const double disc = fmax(b * b - a * c, 0.0);
    th = c > 0.0 ? (-b - sqrt(disc)) / a : (-b + sqrt(disc)) / a;  // first contact with the sphere
  } else {
    th = (r - Q0[2]) / (Q1[2] - Q0[2]);
  }
  return fmin(fmax(th, 0.0), 1.0);
}

struct Modes {
  bool exists[4];
  int sp[4], side[4];
  double P[4][3];
  cx A[4][3];
};

// Outgoing modes (0 P reflected, 1 S reflected, 2 P transmitted,
// 3 S transmitted) for the plane wave (Pin, Ain) of type sp_in hitting the
// interface from layer L into layer L2 across unit normal n at the point xc
// (where the speeds of both layers are taken).  free: a traction-free surface
// (nothing beyond it): only the reflected modes, from sigma.n = 0 (rows t1,
// t3 in plane; mu (k3_in A_SH + k3_r R_SH) = 0 for SH).
__device__ void outgoing_modes(const DevMedium &m, int L, int L2, const double xc[3], const double n[3], int sp_in,
                               const double Pin[3], const cx Ain[3], Modes &o, bool free = false)
{
  const int lay[2] = {L, L2};
  double cP[2], cS[2];
  for (int s = 0; s < 2; ++s) {
    double g[3], H6[6];
    medium_eval<MK_LAYERED>(m, 0, lay[s], xc, cP[s], g, H6);
    medium_eval<MK_LAYERED>(m, 1, lay[s], xc, cS[s], g, H6);
  }
  const double pabs = sqrt(dot3(Pin, Pin));
  const double c_in = sp_in == 0 ? cP[0] : cS[0];
  const double H = c_in * pabs;
  const double pn = dot3(Pin, n);
  double e1[3], e2[3], t[3];
  for (int d = 0; d < 3; ++d) t[d] = Pin[d] - pn * n[d];
  double p1 = sqrt(dot3(t, t));
  if (p1 > 1e-12 * pabs) {
    for (int d = 0; d < 3; ++d) e1[d] = t[d] / p1;
  } else {
    // normal incidence: any tangent (the problem is then symmetric about n)
    p1 = 0.0;
    double u[3] = {1.0, 0.0, 0.0};
    if (fabs(n[0]) > 0.9) { u[0] = 0.0; u[1] = 1.0; }
    const double un = dot3(u, n);
    for (int d = 0; d < 3; ++d) u[d] -= un * n[d];
    const double nu = sqrt(dot3(u, u));
    for (int d = 0; d < 3; ++d) e1[d] = u[d] / nu;
  }
  e2[0] = n[1] * e1[2] - n[2] * e1[1];
  e2[1] = n[2] * e1[0] - n[0] * e1[2];
  e2[2] = n[0] * e1[1] - n[1] * e1[0];
  const double dirn = pn >= 0.0 ? 1.0 : -1.0;
  double lam[2], mu[2];
  for (int s = 0; s < 2; ++s) {
    const double rho = m.rhol[lay[s]], a = cP[s], b = cS[s];
    mu[s] = rho * b * b;
    lam[s] = rho * (a * a - 2.0 * b * b);
  }
  // normal momentum k3 and in-plane polarisation (d1, d3) per wave:
  // 0..3 the outgoing modes, 4 the incident wave
  cx k3[5], d1[5], d3[5];
  int sd[5];
  for (int w = 0; w < 5; ++w) {
    int spw, s;
    double kabs;
    if (w < 4) {
      spw = w & 1;
      s = w >> 1;
      kabs = H / (spw == 0 ? cP[s] : cS[s]);
      const double rad = kabs * kabs - p1 * p1;
      if (rad >= 0.0) {
        k3[w] = mk((s == 1 ? dirn : -dirn) * sqrt(rad));
        o.exists[w] = true;
      } else {
        k3[w] = mk(0.0, (s == 1 ? 1.0 : -1.0) * sqrt(-rad));  // decays away from the interface
        o.exists[w] = false;
      }
      o.sp[w] = spw;
      o.side[w] = s;
    } else {
      spw = sp_in;
      s = 0;
      kabs = H / c_in;
      k3[w] = mk(pn);
    }
    sd[w] = s;
    const cx h1 = mk(p1 / kabs), h3 = (1.0 / kabs) * k3[w];
    if (spw == 0) {
      d1[w] = h1;
      d3[w] = h3;
    } else {
      d1[w] = h3;
      d3[w] = -h1;
    }
  }
  // incident amplitude: in-plane part along (d1, d3) of the incident wave, SH part along e2
  cx A1 = mk(0.0), A2 = mk(0.0), A3 = mk(0.0);
  for (int d = 0; d < 3; ++d) {
    A1 = A1 + e1[d] * Ain[d];
    A2 = A2 + e2[d] * Ain[d];
    A3 = A3 + n[d] * Ain[d];
  }
  const cx ain = A1 * d1[4] + A3 * d3[4];
  // P-SV: rows u1, u3, t1, t3; incident and reflected on side 0 = transmitted on side 1
  cx M[4][4], rhs[4], x[4];
  for (int w = 0; w < 5; ++w) {
    const int s = sd[w];
    const cx k1 = mk(p1);
    const cx col[4] = {d1[w], d3[w], mu[s] * (k1 * d3[w] + k3[w] * d1[w]),
                       lam[s] * (k1 * d1[w] + k3[w] * d3[w]) + (2.0 * mu[s]) * (k3[w] * d3[w])};
    for (int r = 0; r < 4; ++r) {
      if (w == 4) rhs[r] = -(ain * col[r]);
      else M[r][w] = s == 0 ? col[r] : -col[r];
    }
  }
  if (free) {
    // rows t1, t3 and the reflected columns only
    cx F[4][4], bf[4];
    for (int r = 0; r < 2; ++r) {
      bf[r] = rhs[2 + r];
      for (int w = 0; w < 2; ++w) F[r][w] = M[2 + r][w];
    }
    solve_small(2, F, bf, x);
    x[2] = x[3] = mk(0.0);
    o.exists[2] = o.exists[3] = false;
  } else {
    solve_small(4, M, rhs, x);
  }
  // SH: rows u2, t2 (polarisation e2 for every SH wave)
  cx y[2] = {mk(0.0), mk(0.0)};
  if (sp_in == 1 && free) {
    y[0] = -((k3[4] * A2) / k3[1]);
  } else if (sp_in == 1) {
    cx S[4][4], bs[4], xs[4];
    S[0][0] = mk(1.0);
    S[0][1] = mk(-1.0);
    S[1][0] = mu[0] * k3[1];
    S[1][1] = -(mu[1] * k3[3]);
    bs[0] = -A2;
    bs[1] = -(mu[0] * (k3[4] * A2));
    solve_small(2, S, bs, xs);
    y[0] = xs[0];
    y[1] = xs[1];
  }
  for (int w = 0; w < 4; ++w) {
    for (int d = 0; d < 3; ++d) o.P[w][d] = p1 * e1[d] + k3[w].r * n[d];
    const cx sh = o.sp[w] == 1 ? y[w >> 1] : mk(0.0);
    for (int d = 0; d < 3; ++d) o.A[w][d] = x[w] * (e1[d] * d1[w] + n[d] * d3[w]) + e2[d] * sh;
  }
}

// dzQ, dzP (planes of y) mapped to an outgoing mode with momentum Pout at
// the crossing point, for each row (the derivative by one z_m), with
// V = c P/|P|, s = V_in.n, q_n = row(dzQ).n, mu = p_n' - p_n:
//   dzQ* = dzQ - V_in q_n / s (the crossing point), dzP* = dzP + |Pin| gin q_n / s,
//   dmu = [(V_in - V_out).dzP* + (|Pin| gin - |Pout| gout).dzQ* - mu V_out.K dzQ*] / V_out.n,
//   dzQ' = dzQ* + V_out q_n / s,  dzP' = dzP* + n dmu + mu K dzQ* - |Pout| gout q_n / s,
// K dzQ* = kcurv dzQ* (dzQ* is tangent); gin, gout: gradients of the incident
// and outgoing speeds at the crossing point; kcurv: s/R on a sphere, 0 flat.
__device__ void map_jacobians(double *y, const double n[3], const double Pin[3], const double Pout[3], double c_in,
                              double c_out, const double gin[3], const double gout[3], double kcurv)
{
  const double Pi = sqrt(dot3(Pin, Pin)), Po = sqrt(dot3(Pout, Pout));
  double vin[3], vout[3];
  for (int d = 0; d < 3; ++d) {
    vin[d] = c_in * Pin[d] / Pi;
    vout[d] = c_out * Pout[d] / Po;
  }
  const double s_in = dot3(vin, n), s_out = dot3(vout, n), mu = dot3(Pout, n) - dot3(Pin, n);
  const int base[2][2] = {{IZQR, IZPR}, {IZQI, IZPI}};
  for (int r = 0; r < 3; ++r)
    for (int ri = 0; ri < 2; ++ri) {  // real and imaginary parts map alike
      double *zq = y + base[ri][0] + 3 * r, *zp = y + base[ri][1] + 3 * r;
      const double qn = (zq[0] * n[0] + zq[1] * n[1] + zq[2] * n[2]) / s_in;
      double qs[3], ps[3];
      for (int d = 0; d < 3; ++d) {
        qs[d] = zq[d] - vin[d] * qn;
        ps[d] = zp[d] + Pi * gin[d] * qn;
      }
      double num = 0.0;
      for (int d = 0; d < 3; ++d)
        num += (vin[d] - vout[d]) * ps[d] + (Pi * gin[d] - Po * gout[d]) * qs[d] - mu * kcurv * vout[d] * qs[d];
      const double dmu = num / s_out;
      for (int d = 0; d < 3; ++d) {
        zq[d] = qs[d] + vout[d] * qn;
        zp[d] = ps[d] + n[d] * dmu + mu * kcurv * qs[d] - Po * gout[d] * qn;
      }
    }
}

__device__ __forceinline__ void initial_axis(const double P[3], double e[3])
{
  const double np = sqrt(dot3(P, P));
  const bool nearz = fabs(P[2]) / np > 0.93969262078590838405;  // cos(20 degrees)
  e[0] = nearz ? 1.0 : 0.0;
  e[1] = 0.0;
  e[2] = nearz ? 0.0 : 1.0;
}

// One RK4 step of a layered-medium beam: the specialised step where the
// medium has no gradient, else the general one.
__device__ __forceinline__ void layered_step(const DevMedium &m, int sp, int L, double sg, const double e[3],
                                             double *y, double h)
{
  if (m.any_grad) rk4_step<MK_LAYERED>(m, sp, L, sg, sp == 1, e, y, h);
  else rk4_step_pc<MK_LAYERED>(m, sp, L, sg, sp == 1, y, h);
}

__device__ __forceinline__ double level_of(const DevMedium &m, const double *Q)
{
  return m.geometry == 1 ? sqrt(dot3(Q, Q)) : Q[2];
}

// Crossing fraction of the step from y0 in a layer whose speed varies (a
// curved ray): four secant iterations on the level of the RK4 sub-step of
// theta dt from y0, started from theta = 0 and the straight-ray estimate.
__device__ double crossing_secant(const DevMedium &m, int sp, int L, double sg, const double e[3],
                                  const double *y0, int iface, double dt, double th0)
{
  const double b = iface_level(m, iface);
  double ta = 0.0, fa = level_of(m, y0 + IQ) - b, tb = th0;
  double x[NS];
  for (int f = 0; f < NS; ++f) x[f] = y0[f];
  layered_step(m, sp, L, sg, e, x, tb * dt);
  double fb = level_of(m, x + IQ) - b;
  for (int it = 0; it < 4; ++it) {
    if (fb == fa) break;
    const double tn = fmin(fmax(tb - fb * (tb - ta) / (fb - fa), 0.0), 1.0);
    ta = tb;
    fa = fb;
    tb = tn;
    for (int f = 0; f < NS; ++f) x[f] = y0[f];
    layered_step(m, sp, L, sg, e, x, tb * dt);
    fb = level_of(m, x + IQ) - b;
  }
  return tb;
}

// Per crossing beam: the crossing point state (in y), the modes, and which
// of them become children.
struct Crossing {
  double th;
  int newL;
  double n[3];
  double kcurv;  // signed curvature of the interface at the crossing (0: flat)
  Modes md;
  bool keep[4];
  int nkeep;
  bool capped;
};

__device__ void analyse(const DevMedium &m, const InterfaceArgs &a, int64_t i, double *y, double e[3], Crossing &c)
{
  const int64_t cap = a.cap;
  const int br = a.i32[FGA_BRANCH * cap + i];
  const int sp = br == 0 ? 0 : 1;
  const double sg = (double)a.i32[FGA_SIGMA * cap + i];
  const int L = a.i32[FGA_LAYER * cap + i];
  const int gen = a.i32[FGA_GEN * cap + i];
  for (int f = 0; f < NS; ++f) y[f] = a.f64[f * cap + i];
  for (int d = 0; d < 3; ++d) e[d] = a.f64[(FGA_E + d) * cap + i];
  double y1[NS];
  for (int f = 0; f < NS; ++f) y1[f] = y[f];
  layered_step(m, sp, L, sg, e, y1, a.dt);
  int iface = 0, newL = L;
  c.nkeep = 0;
  c.capped = false;
  for (int k = 0; k < 4; ++k) c.keep[k] = false;
  if (!layer_exit(m, L, y1 + IQ, iface, newL)) {
    // not reached when the integrator flagged the beam: treat as an ordinary step
    c.th = -1.0;
    for (int f = 0; f < NS; ++f) y[f] = y1[f];
    return;
  }
  c.newL = newL;
  c.th = crossing(m, iface, y + IQ, y1 + IQ);
  if (m.gradl[L] != 0.0 || m.anom_amp[L] != 0.0) c.th = crossing_secant(m, sp, L, sg, e, y, iface, a.dt, c.th);
  layered_step(m, sp, L, sg, e, y, c.th * a.dt);
  const double rb = iface_level(m, iface);
  const bool surf = iface == IFACE_SURFACE;
  if (m.geometry == 1) {
    const double r = sqrt(dot3(y + IQ, y + IQ));
    for (int d = 0; d < 3; ++d) y[IQ + d] *= rb / r;
    c.kcurv = (surf ? 1.0 : (newL > L ? -1.0 : 1.0)) / rb;
    for (int d = 0; d < 3; ++d) c.n[d] = c.kcurv * y[IQ + d];
  } else {
    y[IQ + 2] = rb;
    c.kcurv = 0.0;
    c.n[0] = c.n[1] = 0.0;
    c.n[2] = surf ? 1.0 : (newL > L ? 1.0 : -1.0);
  }
  if (gen >= a.gen_max) {
    c.capped = true;
    return;
  }
  // incident displacement amplitude vector
  cx Ain[3];
  if (sp == 0) {
    const double ip = 1.0 / sqrt(dot3(y + IP, y + IP));
    for (int d = 0; d < 3; ++d) Ain[d] = mk(y[IA] * y[IP + d] * ip, y[IA + 1] * y[IP + d] * ip);
  } else {
    double nsh[3], nsv[3];
    s_frame(y + IP, e, nsh, nsv);
    for (int d = 0; d < 3; ++d)
      Ain[d] = mk(y[IA] * nsv[d] + y[IA + 2] * nsh[d], y[IA + 1] * nsv[d] + y[IA + 3] * nsh[d]);
  }
  const double ain = sqrt(cabs2(Ain[0]) + cabs2(Ain[1]) + cabs2(Ain[2]));
  outgoing_modes(m, L, newL, y + IQ, c.n, sp, y + IP, Ain, c.md, surf);
  for (int k = 0; k < 4; ++k) {
    const double am = sqrt(cabs2(c.md.A[k][0]) + cabs2(c.md.A[k][1]) + cabs2(c.md.A[k][2]));
    c.keep[k] = c.md.exists[k] && am >= a.child_cut * ain;
    c.nkeep += c.keep[k] ? 1 : 0;
  }
}

// exclusive prefix sum over the workgroup of v (small non-negative ints); total in *tot
__device__ int block_exscan(int v, int *tot)
{
  __shared__ int ws[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int incl = v;
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(incl, off);
    if (lane >= off) incl += t;
  }
  if (lane == 63) ws[w] = incl;
  __syncthreads();
  int base = 0, all = 0;
  for (int k = 0; k < 4; ++k) {
    if (k < w) base += ws[k];
    all += ws[k];
  }
  __syncthreads();
  *tot = all;
  return base + incl - v;
}

template <bool WRITE>
__global__ __launch_bounds__(256) void k_interface(DevMedium m, InterfaceArgs a)
{
  const int64_t li = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t i = li < a.nlist ? a.list[li] : 0;
  const bool mine = li < a.nlist && (a.i32[FGA_FLAGS * a.cap + i] & FGA_FLAG_CROSS);
  if (!__syncthreads_or(mine)) {
    if (!WRITE && threadIdx.x == 0) a.blk_extra[blockIdx.x] = 0;
    return;
  }
  double y[NS], e[3];
  Crossing c;
  c.nkeep = 0;
  c.th = -1.0;
  c.capped = false;
  if (mine) analyse(m, a, i, y, e, c);
  const int extra = (mine && c.th >= 0.0 && c.nkeep > 1) ? c.nkeep - 1 : 0;
  int tot;
  const int off = block_exscan(extra, &tot);
  if (!WRITE) {
    if (threadIdx.x == 0) a.blk_extra[blockIdx.x] = tot;
    return;
  }
  if (!mine) return;
  const int64_t cap = a.cap;
  const int L = a.i32[FGA_LAYER * cap + i];
  const int br = a.i32[FGA_BRANCH * cap + i];
  const int sp_in = br == 0 ? 0 : 1;
  const int sigma = a.i32[FGA_SIGMA * cap + i];
  const int gen = a.i32[FGA_GEN * cap + i];
  const int flags = a.i32[FGA_FLAGS * cap + i] & ~FGA_FLAG_CROSS;
  const int64_t lin = a.lineage[i];
  const double wr = a.f64[FGA_W_RE * cap + i], wi = a.f64[FGA_W_IM * cap + i];
  if (c.th < 0.0) {
    // no crossing found after all: the ordinary step result
    if (sp_in == 1) reframe_s(y, e);
    for (int f = 0; f < NS; ++f) a.f64[f * cap + i] = y[f];
    for (int d = 0; d < 3; ++d) a.f64[(FGA_E + d) * cap + i] = e[d];
    a.i32[FGA_FLAGS * cap + i] = flags;
    return;
  }
  unsigned long long nchild = 0;
  if (c.nkeep == 0) a.i32[FGA_FLAGS * cap + i] = 0;  // retired (generation cap or no child)
  double c_in, g_in[3], H6[6];
  medium_eval<MK_LAYERED>(m, sp_in, L, y + IQ, c_in, g_in, H6);  // at the crossing point
  int j = 0;
  for (int k = 0; k < 4; ++k) {
    if (!c.keep[k]) continue;
    const int64_t slot = j == 0 ? i : a.n + a.blk_off[blockIdx.x] + off + (j - 1);
    ++j;
    const int layc = c.md.side[k] == 1 ? c.newL : L;
    const int spc = c.md.sp[k];
    double c_out, g_out[3];
    medium_eval<MK_LAYERED>(m, spc, layc, y + IQ, c_out, g_out, H6);
    double z[NS], ec[3];
    for (int f = 0; f < NS; ++f) z[f] = y[f];
    for (int d = 0; d < 3; ++d) z[IP + d] = c.md.P[k][d];
    map_jacobians(z, c.n, y + IP, z + IP, c_in, c_out, g_in, g_out, c.kcurv);
    initial_axis(z + IP, ec);
    if (spc == 0) {
      const double ip = 1.0 / sqrt(dot3(z + IP, z + IP));
      cx ap = mk(0.0);
      for (int d = 0; d < 3; ++d) ap = ap + (z[IP + d] * ip) * c.md.A[k][d];
      z[IA] = ap.r;
      z[IA + 1] = ap.i;
      z[IA + 2] = 0.0;
      z[IA + 3] = 0.0;
    } else {
      double nsh[3], nsv[3];
      s_frame(z + IP, ec, nsh, nsv);
      cx asv = mk(0.0), ash = mk(0.0);
      for (int d = 0; d < 3; ++d) {
        asv = asv + nsv[d] * c.md.A[k][d];
        ash = ash + nsh[d] * c.md.A[k][d];
      }
      z[IA] = asv.r;
      z[IA + 1] = asv.i;
      z[IA + 2] = ash.r;
      z[IA + 3] = ash.i;
    }
    layered_step(m, spc, layc, (double)sigma, ec, z, (1.0 - c.th) * a.dt);
    if (spc == 1) reframe_s(z, ec);
    for (int f = 0; f < NS; ++f) a.f64[f * cap + slot] = z[f];
    for (int d = 0; d < 3; ++d) a.f64[(FGA_E + d) * cap + slot] = ec[d];
    a.f64[FGA_W_RE * cap + slot] = wr;
    a.f64[FGA_W_IM * cap + slot] = wi;
    a.i32[FGA_BRANCH * cap + slot] = spc == 0 ? 0 : 2;
    a.i32[FGA_SIGMA * cap + slot] = sigma;
    a.i32[FGA_LAYER * cap + slot] = layc;
    a.i32[FGA_GEN * cap + slot] = gen + 1;
    a.i32[FGA_FLAGS * cap + slot] = FGA_FLAG_ALIVE;
    a.lineage[slot] = FGA_LINEAGE_CHILD(lin, gen, k);
    ++nchild;
  }
  if (a.counters) {
    atomicAdd(a.counters + 0, 1ull);
    if (nchild) atomicAdd(a.counters + 1, nchild);
    if (c.capped) atomicAdd(a.counters + 2, 1ull);
  }
}


// Crossing beams of [0, n): one atomic per wavefront reserves its run of the
// (unordered) list; the list is then sorted, so the children's slots do not
// depend on the order in which wavefronts ran.
__global__ __launch_bounds__(256) void k_collect_cross(const int32_t *__restrict__ flags, int64_t n,
                                                       int32_t *__restrict__ list, unsigned long long *__restrict__ count)
{
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool c = i < n && (flags[i] & FGA_FLAG_CROSS);
  const unsigned long long b = __ballot(c);
  if (b == 0) return;
  const int lane = threadIdx.x & 63;
  unsigned long long base = 0;
  if (lane == 0) base = atomicAdd(count, (unsigned long long)__popcll(b));
  base = __shfl(base, 0);
  if (c) list[base + __popcll(b & ((1ull << lane) - 1))] = (int32_t)i;
}

}  // namespace

size_t cross_sort_bytes(int64_t cap)
{
  size_t bytes = 0;
  hipcub::DeviceRadixSort::SortKeys(nullptr, bytes, (const int32_t *)nullptr, (int32_t *)nullptr,
                                    (int)(cap > 0 ? cap : 1), 0, 32);
  return bytes;
}

hipError_t collect_crossers(const int32_t *flags, int64_t n, int32_t *list, int32_t *sorted,
                            unsigned long long *count, void *tmp, size_t tmp_bytes, hipStream_t st,
                            int64_t *ncross)
{
  *ncross = 0;
  if (n <= 0) return hipSuccess;
  hipError_t e = hipMemsetAsync(count, 0, sizeof(unsigned long long), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_collect_cross, (unsigned)((n + 255) / 256), 256, 0, st, flags, n, list, count);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  unsigned long long h = 0;
  if ((e = hipMemcpyAsync(&h, count, sizeof h, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  if (h == 0) return hipSuccess;
  if ((e = hipcub::DeviceRadixSort::SortKeys(tmp, tmp_bytes, list, sorted, (int)h, 0, 32, st)) != hipSuccess)
    return e;
  *ncross = (int64_t)h;
  return hipSuccess;
}


hipError_t launch_interface(const DevMedium &m, const InterfaceArgs &a, int write, hipStream_t st)
{
  if (a.nlist <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((a.nlist + 255) / 256);
  if (write) hipLaunchKernelGGL(k_interface<true>, blocks, 256, 0, st, m, a);
  else hipLaunchKernelGGL(k_interface<false>, blocks, 256, 0, st, m, a);
  return hipGetLastError();
}

}  // namespace fga
