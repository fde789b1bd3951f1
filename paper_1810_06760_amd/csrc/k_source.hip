// Step 1 for a point moment-tensor source (closed form, no quadrature).
//
// An impulsive moment-tensor source is the initial velocity
// g = -(1/rho0) M grad delta(x - x0) with u(0) = 0; integrating by parts,
//   FBI[g/c_b](q, p) = (1/rho0) M . grad_y [K(y)/c_b(y)] at y = x0,
//   K(y) = exp(-i p.(y - q)/eps - |y - q|^2/(2 eps)),
// and with f = 0, eq:psi / eq:alpha^k give psi_{b,+-} = +-(i eps/(2|p|))
// FBI[g/c_b].n_b.  A Ricker wavelet multiplies each beam, whose frequency is
// c_b|p|/eps, by R(w) = (w/w0)^2 exp(1 - (w/w0)^2), w0 = c_P(x0)/eps.  The
// q mesh is nq^3 cell-centred points of the cube x0 +- qhalf; the p mesh is
// Fibonacci directions x Gauss-Legendre |p| shells on
// [shell_lo, shell_hi] c_P(x0)/c_b(x0) with measure |p|^2 w 4 pi / ndir.
// One thread per candidate (lineage order ((b*2 + dir) Np + ip) Nq + iq),
// count / scan / write so the kept beams stay in lineage order.
#include <cmath>
#include <cstring>

#include "device_common.h"

namespace fga {
namespace {

constexpr int MAXSH = 64;

struct SourceArgs {
  int kind;                 // 0: moment tensor (Ricker optional); 1: point force with its time function
  double eps, x0[3], M[3][3], rho0;
  double d[3], omega, t0, width, t_ref;  // point force
  int nq;
  double qhalf, hq;
  int ndir, nshell;
  double shell_lo, shell_hi;
  double gl_t[MAXSH], gl_w[MAXSH];  // Gauss-Legendre nodes and weights on [-1, 1]
  int ricker, mask;
  int merge;                // one S beam per (q, p, direction): SH candidates carry the SV term too
  double cull, norm;
  int64_t Nq, Np, ncand;
  int layer0;
};

// psi (pr, pi) of candidate L and its p-cell measure dp; false for a masked
// branch.  With a.merge the SV candidates are not candidates, and an SH
// candidate also returns the psi of its SV partner (s2r, s2i).
template <int MK>
__device__ bool candidate(const DevMedium &m, const SourceArgs &a, int64_t L, double q[3], double p[3], double e[3],
                          double &pr, double &pi, double &s2r, double &s2i, double &dp, int &br, int &sg)
{
  const int64_t iq = L % a.Nq;
  const int64_t ip = (L / a.Nq) % a.Np;
  const int bd = (int)(L / (a.Nq * a.Np));
  br = bd >> 1;
  sg = (bd & 1) ? -1 : 1;
  if (!(a.mask & (1 << br)) || (a.merge && br == 2)) return false;
  s2r = s2i = 0.0;
  const bool two = a.merge && br == 1;
  const int sp = br == 0 ? 0 : 1;
  double cP, gP[3], H6[6], cb, gb[3];
  medium_eval<MK>(m, 0, a.layer0, a.x0, cP, gP, H6);
  medium_eval<MK>(m, sp, a.layer0, a.x0, cb, gb, H6);
  // p: shell sh, Fibonacci direction dj
  const int sh = (int)(ip / a.ndir), dj = (int)(ip % a.ndir);
  const double lo = a.shell_lo * cP / cb, hi = a.shell_hi * cP / cb;
  const double np = 0.5 * (lo + hi) + 0.5 * (hi - lo) * a.gl_t[sh];
  const double wsh = 0.5 * (hi - lo) * a.gl_w[sh];
  const double ga = 3.14159265358979323846 * (3.0 - sqrt(5.0));
  const double z = 1.0 - (2.0 * dj + 1.0) / a.ndir;
  const double r = sqrt(fmax(0.0, 1.0 - z * z));
  double sn, cs;
  sincos(ga * dj, &sn, &cs);
  p[0] = np * r * cs;
  p[1] = np * r * sn;
  p[2] = np * z;
  dp = np * np * wsh * 4.0 * 3.14159265358979323846 / a.ndir;
  // q
  const int ix = (int)(iq % a.nq), iy = (int)((iq / a.nq) % a.nq), iz = (int)(iq / ((int64_t)a.nq * a.nq));
  q[0] = a.x0[0] - a.qhalf + (ix + 0.5) * a.hq;
  q[1] = a.x0[1] - a.qhalf + (iy + 0.5) * a.hq;
  q[2] = a.x0[2] - a.qhalf + (iz + 0.5) * a.hq;
  // frame axis and polarisation
  const bool nearz = fabs(z) > 0.93969262078590838405;  // |p_z|/|p| > cos 20 deg
  e[0] = nearz ? 1.0 : 0.0;
  e[1] = 0.0;
  e[2] = nearz ? 0.0 : 1.0;
  double nh[3], nh2[3] = {0.0, 0.0, 0.0};
  if (br == 0) {
    nh[0] = p[0] / np;
    nh[1] = p[1] / np;
    nh[2] = p[2] / np;
  } else {
    double nsh[3], nsv[3];
    s_frame(p, e, nsh, nsv);
    for (int d = 0; d < 3; ++d) {
      nh[d] = br == 1 ? nsh[d] : nsv[d];
      nh2[d] = nsv[d];
    }
  }
  // K and grad(K / c_b) at x0
  const double d0 = a.x0[0] - q[0], d1 = a.x0[1] - q[1], d2 = a.x0[2] - q[2];
  const double ie = 1.0 / a.eps;
  if (a.kind == 1) {
    // point force: FBI[g/c_b] = F(s) (d.n_b)/(rho0 c_b) K(x0) of the impulse at time s,
    // launched from q' = q - sigma c (s - t_ref) p/|p| and integrated over s in
    // closed form: K(x0) I with the Gaussian integral I (v = s + t0,
    // v0 = t0 + t_ref, D = x0 - q', D_par = D.p/|p|):
    //   I = 1/2 sum_{+-} sqrt(pi/A) exp(B^2/(4A) + C), A = 1/width^2 + c^2/(2 eps),
    //   B = c^2 v0/eps + sigma c D_par/eps + i (sigma c |p|/eps +- omega),
    //   C = -c^2 v0^2/(2 eps) - sigma c D_par v0/eps - i sigma c |p| v0/eps
    const double dpar = (p[0] * d0 + p[1] * d1 + p[2] * d2) / np;
    const double v0 = a.t0 + a.t_ref;
    const double A = 1.0 / (a.width * a.width) + cb * cb * 0.5 * ie;
    const double Cr = -cb * cb * v0 * v0 * 0.5 * ie - sg * cb * dpar * v0 * ie;
    const double Ci = -sg * cb * np * v0 * ie;
    const double Br = cb * cb * v0 * ie + sg * cb * dpar * ie;
    // K(x0) = exp(-i p.D/eps - |D|^2/(2 eps)) folded into the same exponent
    const double Kre = -(d0 * d0 + d1 * d1 + d2 * d2) * 0.5 * ie;
    const double Kim = -(p[0] * d0 + p[1] * d1 + p[2] * d2) * ie;
    const double sq = sqrt(3.14159265358979323846 / A);
    double Ir = 0.0, Ii = 0.0;
    for (int k = 0; k < 2; ++k) {
      const double Bi = sg * cb * np * ie + (k == 0 ? a.omega : -a.omega);
      const double er = (Br * Br - Bi * Bi) / (4.0 * A) + Cr + Kre;
      const double ei = (2.0 * Br * Bi) / (4.0 * A) + Ci + Kim;
      double sn, cs;
      sincos(ei, &sn, &cs);
      const double mg = 0.5 * sq * exp(er);
      Ir += mg * cs;
      Ii += mg * sn;
    }
    // psi = sg (i eps / (2|p|)) (d.n/(rho0 c)) K I
    auto force_psi = [&](const double nn[3], double &r, double &im) {
      const double dn = (a.d[0] * nn[0] + a.d[1] * nn[1] + a.d[2] * nn[2]) / (a.rho0 * cb);
      const double f = sg * a.eps / (2.0 * np) * dn;
      r = -f * Ii;
      im = f * Ir;
    };
    force_psi(nh, pr, pi);
    if (two) force_psi(nh2, s2r, s2i);
    return true;
  }
  double ks, kc;
  sincos(-(p[0] * d0 + p[1] * d1 + p[2] * d2) * ie, &ks, &kc);
  const double kmag = exp(-(d0 * d0 + d1 * d1 + d2 * d2) * 0.5 * ie);
  const double Kr = kmag * kc, Ki = kmag * ks;
  const double dd[3] = {d0, d1, d2};
  double gr[3], gi[3];
  for (int j = 0; j < 3; ++j) {
    // K (-i p_j/eps - d_j/eps) / c_b - K g_j / c_b^2
    const double ar = -dd[j] * ie, ai = -p[j] * ie;
    gr[j] = (Kr * ar - Ki * ai) / cb - Kr * gb[j] / (cb * cb);
    gi[j] = (Kr * ai + Ki * ar) / cb - Ki * gb[j] / (cb * cb);
  }
  double mr[3], mi[3];  // M grad(K/c)
  for (int i = 0; i < 3; ++i) {
    mr[i] = mi[i] = 0.0;
    for (int j = 0; j < 3; ++j) {
      mr[i] += a.M[i][j] * gr[j];
      mi[i] += a.M[i][j] * gi[j];
    }
  }
  double rk = 1.0;
  if (a.ricker) {
    const double w = cb * np / a.eps, w0 = cP / a.eps;
    const double x = (w / w0) * (w / w0);
    rk = x * exp(1.0 - x);
  }
  // psi = sg (i eps / (2|p|)) G rk, G = (M grad(K/c)).n / rho0
  auto mt_psi = [&](const double nn[3], double &r, double &im) {
    double Gr = 0.0, Gi = 0.0;
    for (int i = 0; i < 3; ++i) {
      Gr += mr[i] * nn[i];
      Gi += mi[i] * nn[i];
    }
    Gr /= a.rho0;
    Gi /= a.rho0;
    const double f = sg * a.eps / (2.0 * np) * rk;
    r = -f * Gi;
    im = f * Gr;
  };
  mt_psi(nh, pr, pi);
  if (two) mt_psi(nh2, s2r, s2i);
  return true;
}

// Whether a candidate is kept: |psi| >= cull; a merged S candidate when
// either member's is (each member's term is then kept only if its own is).
__device__ __forceinline__ bool source_kept(const SourceArgs &a, int br, double pr, double pi, double s2r,
                                            double s2i)
{
  const bool k1 = !(sqrt(pr * pr + pi * pi) < a.cull);
  if (!(a.merge && br == 1)) return k1;
  return k1 || !(sqrt(s2r * s2r + s2i * s2i) < a.cull);
}

template <int MK>
__global__ __launch_bounds__(256) void k_source_count(DevMedium m, SourceArgs a, int64_t *__restrict__ counts)
{
  const int64_t L = (int64_t)blockIdx.x * 256 + threadIdx.x;
  bool keep = false;
  if (L < a.ncand) {
    double q[3], p[3], e[3], pr = 0.0, pi = 0.0, s2r = 0.0, s2i = 0.0, dp = 0.0;
    int br, sg;
    if (candidate<MK>(m, a, L, q, p, e, pr, pi, s2r, s2i, dp, br, sg)) keep = source_kept(a, br, pr, pi, s2r, s2i);
  }
  int total;
  block_rank(keep, &total);
  if (threadIdx.x == 0) counts[blockIdx.x] = total;
}

template <int MK>
__global__ __launch_bounds__(256) void k_source_write(DevMedium m, SourceArgs a, const int64_t *__restrict__ offs,
                                                      double *__restrict__ F, int32_t *__restrict__ I,
                                                      int64_t *__restrict__ lineage, int64_t cap)
{
  const int64_t L = (int64_t)blockIdx.x * 256 + threadIdx.x;
  bool keep = false;
  double q[3], p[3], e[3], pr = 0.0, pi = 0.0, s2r = 0.0, s2i = 0.0, dp = 0.0;
  int br = 0, sg = 1;
  if (L < a.ncand) {
    if (candidate<MK>(m, a, L, q, p, e, pr, pi, s2r, s2i, dp, br, sg)) keep = source_kept(a, br, pr, pi, s2r, s2i);
  }
  int total;
  const int r = block_rank(keep, &total);
  if (!keep) return;
  const int64_t i = offs[blockIdx.x] + r;
  for (int d = 0; d < 3; ++d) {
    F[(FGA_Q + d) * cap + i] = q[d];
    F[(FGA_P + d) * cap + i] = p[d];
    F[(FGA_E + d) * cap + i] = e[d];
  }
  for (int o = 0; o < 9; ++o) {
    const bool diag = o % 4 == 0;
    F[(FGA_ZQ_RE + o) * cap + i] = diag ? 1.0 : 0.0;
    F[(FGA_ZQ_IM + o) * cap + i] = 0.0;
    F[(FGA_ZP_RE + o) * cap + i] = 0.0;
    F[(FGA_ZP_IM + o) * cap + i] = diag ? -1.0 : 0.0;
  }
  const double a0 = 2.8284271247461900976;  // 2^{3/2}
  if (a.merge && br == 1) {
    // merged S beam: weight 1, (a_SV, a_SH) = 2^{3/2} (w_SV, w_SH) of the kept members
    const bool ksh = !(sqrt(pr * pr + pi * pi) < a.cull), ksv = !(sqrt(s2r * s2r + s2i * s2i) < a.cull);
    F[FGA_A0_RE * cap + i] = ksv ? a0 * (s2r * dp * a.norm) : 0.0;
    F[FGA_A0_IM * cap + i] = ksv ? a0 * (s2i * dp * a.norm) : 0.0;
    F[FGA_A1_RE * cap + i] = ksh ? a0 * (pr * dp * a.norm) : 0.0;
    F[FGA_A1_IM * cap + i] = ksh ? a0 * (pi * dp * a.norm) : 0.0;
    F[FGA_W_RE * cap + i] = 1.0;
    F[FGA_W_IM * cap + i] = 0.0;
  } else {
    F[FGA_A0_RE * cap + i] = br == 1 ? 0.0 : a0;
    F[FGA_A0_IM * cap + i] = 0.0;
    F[FGA_A1_RE * cap + i] = br == 1 ? a0 : 0.0;
    F[FGA_A1_IM * cap + i] = 0.0;
    F[FGA_W_RE * cap + i] = pr * dp * a.norm;  // w = psi dq dp (2 pi eps)^{-9/2}
    F[FGA_W_IM * cap + i] = pi * dp * a.norm;
  }
  F[FGA_S * cap + i] = 0.0;
  int layer = 0;
  if (MK == MK_LAYERED) {
    int iface, nl;
    while (layer_exit(m, layer, q, iface, nl) && nl > layer) layer = nl;
  }
  I[FGA_BRANCH * cap + i] = br;
  I[FGA_SIGMA * cap + i] = sg;
  I[FGA_LAYER * cap + i] = layer;
  I[FGA_GEN * cap + i] = 0;
  I[FGA_FLAGS * cap + i] = FGA_FLAG_ALIVE;
  lineage[i] = L;
}

// Gauss-Legendre nodes and weights on [-1, 1] by Newton iteration on P_n.
void gauss_legendre(int n, double *t, double *w)
{
  for (int i = 0; i < n; ++i) {
    double x = std::cos(3.14159265358979323846 * (i + 0.75) / (n + 0.5));
    double dpn = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) p0 = 1.0;
      dpn = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dpn;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    if (n == 1) p0 = 1.0;
    dpn = n * (x * p1 - p0) / (x * x - 1.0);
    t[i] = x;
    w[i] = 2.0 / ((1.0 - x * x) * dpn * dpn);
  }
}

fga_status source_args(const fga_point_source *s, SourceArgs *a);

// The point force in the candidate layout of the moment-tensor source.
fga_status force_args(const fga_point_force *s, SourceArgs *a)
{
  if (!s) return fail(FGA_EINVAL, "point force is NULL");
  if (!(s->width > 0) || !(s->omega >= 0))
    return fail(FGA_EINVAL, "point force: need width > 0 and omega >= 0");
  fga_point_source ps{};
  ps.eps = s->eps;
  for (int d = 0; d < 3; ++d) ps.x0[d] = s->x0[d];
  ps.rho0 = s->rho0;
  ps.nq = s->nq;
  ps.qhalf = s->qhalf;
  ps.ndir = s->ndir;
  ps.nshell = s->nshell;
  ps.shell_lo = s->shell_lo;
  ps.shell_hi = s->shell_hi;
  ps.ricker = 0;
  ps.branch_mask = s->branch_mask;
  ps.cull_abs = s->cull_abs;
  ps.merge_s = s->merge_s;
  fga_status st = source_args(&ps, a);
  if (st != FGA_OK) return st;
  a->kind = 1;
  for (int d = 0; d < 3; ++d) a->d[d] = s->d[d];
  a->omega = s->omega;
  a->t0 = s->t0;
  a->width = s->width;
  a->t_ref = s->t_ref;
  return FGA_OK;
}

fga_status source_args(const fga_point_source *s, SourceArgs *a)
{
  if (!s) return fail(FGA_EINVAL, "point source is NULL");
  if (!(s->eps > 0) || s->nq < 1 || !(s->qhalf > 0) || s->ndir < 1 || s->nshell < 1 || s->nshell > MAXSH ||
      !(s->shell_lo > 0) || !(s->shell_hi > s->shell_lo))
    return fail(FGA_EINVAL, "point source: need eps > 0, nq >= 1, qhalf > 0, ndir >= 1, 1 <= nshell <= %d, "
                            "0 < shell_lo < shell_hi", MAXSH);
  std::memset(a, 0, sizeof(*a));
  a->eps = s->eps;
  a->rho0 = s->rho0;  // <= 0: the medium's density at x0, set by the caller
  for (int d = 0; d < 3; ++d) a->x0[d] = s->x0[d];
  const double M[3][3] = {{s->M[0], s->M[3], s->M[4]}, {s->M[3], s->M[1], s->M[5]}, {s->M[4], s->M[5], s->M[2]}};
  std::memcpy(a->M, M, sizeof(M));
  a->nq = s->nq;
  a->qhalf = s->qhalf;
  a->hq = 2.0 * s->qhalf / s->nq;
  a->ndir = s->ndir;
  a->nshell = s->nshell;
  a->shell_lo = s->shell_lo;
  a->shell_hi = s->shell_hi;
  gauss_legendre(s->nshell, a->gl_t, a->gl_w);
  a->ricker = s->ricker ? 1 : 0;
  a->mask = s->branch_mask & 7;
  a->merge = s->merge_s && (a->mask & 6) == 6;
  a->cull = s->cull_abs;
  a->Nq = (int64_t)s->nq * s->nq * s->nq;
  a->Np = (int64_t)s->ndir * s->nshell;
  a->ncand = 6 * a->Nq * a->Np;
  a->norm = a->hq * a->hq * a->hq * std::pow(2.0 * 3.14159265358979323846 * s->eps, -4.5);
  return FGA_OK;
}

template <int MK>
fga_status run_source(const DevMedium &dm, const SourceArgs &a, fga_beams *beams, int64_t *counts, int64_t *offs,
                      int64_t *total, hipStream_t st)
{
  const int64_t nblk = (a.ncand + 255) / 256;
  hipLaunchKernelGGL(k_source_count<MK>, (unsigned)nblk, 256, 0, st, dm, a, counts);
  FGA_LAUNCH_CHECK();
  FGA_HIP(launch_scan(counts, offs, nblk, total, st));
  int64_t n = 0;
  FGA_HIP(hipMemcpyAsync(&n, total, sizeof(n), hipMemcpyDeviceToHost, st));
  FGA_HIP(hipStreamSynchronize(st));
  if (n > beams->capacity)
    return fail(FGA_ECAPACITY, "point source makes %lld beams, capacity %lld", (long long)n,
                (long long)beams->capacity);
  hipLaunchKernelGGL(k_source_write<MK>, (unsigned)nblk, 256, 0, st, dm, a, offs, beams->f64, beams->i32,
                     beams->lineage, beams->capacity);
  FGA_LAUNCH_CHECK();
  beams->count = n;
  return FGA_OK;
}

}  // namespace
}  // namespace fga

using namespace fga;

extern "C" {

int64_t fga_point_source_candidates(const fga_point_source *s)
{
  if (!s || s->nq < 1 || s->ndir < 1 || s->nshell < 1) return 0;
  return 6 * (int64_t)s->nq * s->nq * s->nq * s->ndir * s->nshell;
}

size_t fga_decompose_point_source_workspace_bytes(const fga_point_source *s)
{
  const int64_t nc = fga_point_source_candidates(s);
  const int64_t nblk = (nc + 255) / 256 + 1;
  return Arena::need(nblk * sizeof(int64_t)) * 2 + Arena::need(sizeof(int64_t));
}

static fga_status decompose_source(const fga_medium *med, SourceArgs &a, fga_beams *beams, void *workspace,
                                   size_t workspace_bytes, void *stream);

fga_status fga_decompose_point_source(const fga_medium *med, const fga_point_source *src, fga_beams *beams,
                                      void *workspace, size_t workspace_bytes, void *stream)
{
  SourceArgs a;
  fga_status s;
  if ((s = source_args(src, &a)) != FGA_OK) return s;
  return decompose_source(med, a, beams, workspace, workspace_bytes, stream);
}

int64_t fga_point_force_candidates(const fga_point_force *s)
{
  if (!s || s->nq < 1 || s->ndir < 1 || s->nshell < 1) return 0;
  return 6 * (int64_t)s->nq * s->nq * s->nq * s->ndir * s->nshell;
}

size_t fga_decompose_point_force_workspace_bytes(const fga_point_force *s)
{
  const int64_t nc = fga_point_force_candidates(s);
  const int64_t nblk = (nc + 255) / 256 + 1;
  return Arena::need(nblk * sizeof(int64_t)) * 2 + Arena::need(sizeof(int64_t));
}

fga_status fga_decompose_point_force(const fga_medium *med, const fga_point_force *src, fga_beams *beams,
                                     void *workspace, size_t workspace_bytes, void *stream)
{
  SourceArgs a;
  fga_status s;
  if ((s = force_args(src, &a)) != FGA_OK) return s;
  return decompose_source(med, a, beams, workspace, workspace_bytes, stream);
}

}  // extern "C"

static fga_status decompose_source(const fga_medium *med, SourceArgs &a, fga_beams *beams, void *workspace,
                                   size_t workspace_bytes, void *stream)
{
  fga_status s;
  DevMedium dm;
  if ((s = make_dev_medium(med, &dm)) != FGA_OK) return s;
  if (!beams || beams->capacity < 0 || (beams->capacity > 0 && (!beams->f64 || !beams->i32 || !beams->lineage)))
    return fail(FGA_EINVAL, "beams invalid");
  const double *x0 = a.x0;
  // layer and density at x0
  if (dm.kind == FGA_MEDIUM_LAYERED) {
    int L = 0;
    if (dm.geometry == 1) {
      const double r = std::sqrt(x0[0] * x0[0] + x0[1] * x0[1] + x0[2] * x0[2]);
      while (L < dm.nlayer - 1 && r < dm.bound[L]) ++L;
    } else {
      while (L < dm.nlayer - 1 && x0[2] > dm.bound[L]) ++L;
    }
    a.layer0 = L;
  }
  a.rho0 = a.rho0 > 0.0 ? a.rho0
           : (dm.kind == FGA_MEDIUM_LAYERED ? dm.rhol[a.layer0] : (med->rho > 0.0 ? med->rho : 1.0));
  const int64_t nblk = (a.ncand + 255) / 256 + 1;
  Arena ar(workspace, workspace_bytes);
  int64_t *counts = ar.take<int64_t>(nblk), *offs = ar.take<int64_t>(nblk), *total = ar.take<int64_t>(1);
  if (!counts || !offs || !total)
    return fail(FGA_ENOMEM, "point-source workspace too small (%zu bytes given, %zu needed)", workspace_bytes,
                ar.used);
  hipStream_t st = (hipStream_t)stream;
  switch (dm.kind) {
  case FGA_MEDIUM_HOMOGENEOUS: return run_source<MK_HOMOG>(dm, a, beams, counts, offs, total, st);
  case FGA_MEDIUM_GRID:
    if (dm.smooth) return run_source<MK_GRID3>(dm, a, beams, counts, offs, total, st);
    return run_source<MK_GRID>(dm, a, beams, counts, offs, total, st);
  default: return run_source<MK_LAYERED>(dm, a, beams, counts, offs, total, st);
  }
}


