/*
 * fga_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of the frozen Gaussian approximation
 * (FGA) for the 3-D isotropic elastic wave equation (Hateley, Chai, Tong, Yang,
 * "Frozen Gaussian Approximation for 3-D Elastic Wave Equation and Seismic
 * Tomography").  It exists so that tests can check the GPU library against an
 * independent, obviously-correct computation.  Only the tests, the smoke check
 * and the CPU-baseline leg of the benchmark may load it; the product path never
 * does.  It shares no source with the GPU library.
 *
 * What it computes (paper section / equation for each step):
 *   - wave speeds c_P, c_S and their first/second derivatives   (Sec. 2, eq:ps_speed)
 *   - FBI weights psi of the initial data                        (Sec. 2.1, eq:psi, eq:alpha^k)
 *   - ray ODEs for "+" and "-" propagation                       (Sec. 2.2, eq:char_plus, eq:char_minus)
 *   - variational ODEs for dzQ, dzP                              (App. A, eq:DzDt)
 *   - P amplitude and coupled SV/SH amplitudes                   (Sec. 2.2, eq:amp_P, eq:amp_SV, eq:amp_SH)
 *   - classic fixed-step RK4                                     (Sec. 2.3)
 *   - Gaussian summation of the beams                            (Sec. 2.1, eq:FGA)
 *   - flat / spherical interface map: Snell, Zoeppritz, F and W  (Sec. 3.1, eq:p:int, eq:Yilmaz, eq:Inter_DzQDzP)
 *   - point moment-tensor source weights (closed-form FBI)      (Sec. 2.1 eq:psi with f = 0)
 *   - point force with a time function, Duhamel superposition   (Sec. 2.3 eq:ex_homo; eq:psi with f = 0)
 *
 * Readings where the paper is silent or garbled are noted at each use.
 * Parity status: every function here is pinned by a CPU test against closed
 * forms, invariants, brute force, finite differences or quadrature.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* Media                                                                     */
/* ------------------------------------------------------------------------ */

enum {
  OM_HOMOGENEOUS = 0,  /* constant c_P, c_S                                        */
  OM_GRID = 1,         /* periodic node grid of c_P (and c_S or a fixed ratio)      */
  OM_BUMP = 2,         /* c_b(x) = c0_b (1 + amp exp(-|x-x0|^2/(2 s^2)))            */
  OM_LINEAR = 3,       /* c_b(x) = c0_b (1 + g.x)                                   */
  OM_LAYERED = 4       /* flat layers in z or spherical shells, each with a speed that is
                          constant or linear in the level (z or |x|)                  */
};

#define OM_MAXL 8

typedef struct {
  int kind;
  int geometry;          /* layered media: 0 = flat interfaces z = zi, 1 = spheres |x| = ri */
  double cp, cs, rho;    /* homogeneous values, and c0 of the analytic media             */
  /* grid media: nodes lo + i*h, i = 0..n-1, periodic with period n*h                  */
  int n[3];
  double lo[3], h[3];
  const double *tab;     /* derived fields, [speed 0/1][node][10], built by om_grid_fields */
  double cs_ratio;       /* c_S = cs_ratio * c_P when only one node field is given          */
  int two_fields;        /* 1: tab holds independent c_P and c_S fields                     */
  int smooth;            /* 1: c is the periodic cubic B-spline through the node values    */
  const double *coef;    /* its coefficients, [speed 0/1][node], from om_grid_spline_coefficients */
  /* analytic media                                                                         */
  double x0[3], amp, s, g[3];
  /* layered media: layer i occupies level in (bound[i], bound[i-1]) for geometry 1        */
  /* (radii, descending; layer 0 outermost) or z in (bound[i-1], bound[i]) for geometry 0  */
  int nlayer;
  double bound[OM_MAXL];
  double cpl[OM_MAXL], csl[OM_MAXL], rhol[OM_MAXL];
  /* relative gradient of each layer: c_b(x) = c_b,i (1 + gradl[i] v(x)) with the level
     v = z (flat) or |x| (spherical); 0 for a constant layer                               */
  double gradl[OM_MAXL];
  /* Gaussian anomaly of each layer (the low-velocity region of the crosswell model,
     Sec. 4 eq:true_c): c_b(x) is multiplied by 1 - anom_amp[i] exp(-anom_beta[i] q),
     q = sum_d anom_w[i][d] (x_d - anom_x[i][d])^2 (weights 0 drop an axis: the
     model is invariant along it); anom_amp[i] = 0: none                               */
  double anom_amp[OM_MAXL], anom_beta[OM_MAXL], anom_x[OM_MAXL][3], anom_w[OM_MAXL][3];
  /* > 0: a traction-free surface closing the outermost region (spherical: |x| = surface
     around layer 0; flat: z = surface above the last layer); 0: none                      */
  double surface;
} om_medium;

#define OM_SURFACE (-1) /* interface index of the free surface */

/* Derived fields of one scalar node field: c, dc/dx, dc/dy, dc/dz,
 * d2c/dx2, d2c/dy2, d2c/dz2, d2c/dxdy, d2c/dxdz, d2c/dydz, from second-order
 * central differences on the periodic grid (the paper gives no discretisation
 * of a gridded medium; this is the reading used throughout).  Node arrays are
 * stored [z][y][x]. */
void om_grid_fields(const double *c, const int n[3], const double h[3], double *out)
{
  const int nx = n[0], ny = n[1], nz = n[2];
#define C(i, j, k) c[((size_t)(((k) + nz) % nz) * ny + (((j) + ny) % ny)) * nx + (((i) + nx) % nx)]
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        double *o = out + 10 * ((size_t)(k * ny + j) * nx + i);
        double c0 = C(i, j, k);
        o[0] = c0;
        o[1] = (C(i + 1, j, k) - C(i - 1, j, k)) / (2.0 * h[0]);
        o[2] = (C(i, j + 1, k) - C(i, j - 1, k)) / (2.0 * h[1]);
        o[3] = (C(i, j, k + 1) - C(i, j, k - 1)) / (2.0 * h[2]);
        o[4] = (C(i + 1, j, k) - 2.0 * c0 + C(i - 1, j, k)) / (h[0] * h[0]);
        o[5] = (C(i, j + 1, k) - 2.0 * c0 + C(i, j - 1, k)) / (h[1] * h[1]);
        o[6] = (C(i, j, k + 1) - 2.0 * c0 + C(i, j, k - 1)) / (h[2] * h[2]);
        o[7] = (C(i + 1, j + 1, k) - C(i + 1, j - 1, k) - C(i - 1, j + 1, k) + C(i - 1, j - 1, k)) /
               (4.0 * h[0] * h[1]);
        o[8] = (C(i + 1, j, k + 1) - C(i + 1, j, k - 1) - C(i - 1, j, k + 1) + C(i - 1, j, k - 1)) /
               (4.0 * h[0] * h[2]);
        o[9] = (C(i, j + 1, k + 1) - C(i, j + 1, k - 1) - C(i, j - 1, k + 1) + C(i, j - 1, k - 1)) /
               (4.0 * h[1] * h[2]);
      }
#undef C
}

/* Coefficients of the periodic cubic B-spline that takes the node values c
 * at the nodes (the C^2 reading of a gridded medium): along each axis in
 * turn, the periodic system (a_{i-1} + 4 a_i + a_{i+1}) / 6 = f_i, solved by
 * elimination of the cyclic tridiagonal system (the Sherman-Morrison form of
 * the Thomas algorithm).  Arrays [z][y][x]. */
static void om_cyclic_solve(int n, const double *f, double *a, double *wk)
{
  /* A = tridiag(1, 4, 1)/6 with corners 1/6; A = T + u v^T, T tridiagonal */
  if (n == 1) { a[0] = f[0]; return; }
  const double lo = 1.0 / 6.0, di = 4.0 / 6.0, gam = -di;
  double *cp = wk, *y = wk + n, *z = wk + 2 * n, *rhs = wk + 3 * n;
  /* T has diagonal di - gam at 0, di - lo*lo/gam at n-1, di elsewhere */
  for (int pass = 0; pass < 2; ++pass) {
    for (int i = 0; i < n; ++i) rhs[i] = pass == 0 ? f[i] : (i == 0 ? gam : (i == n - 1 ? lo : 0.0));
    double *out = pass == 0 ? y : z;
    double b0 = di - gam;
    cp[0] = lo / b0;
    out[0] = rhs[0] / b0;
    for (int i = 1; i < n; ++i) {
      const double bi = (i == n - 1 ? di - lo * lo / gam : di) - lo * cp[i - 1];
      cp[i] = lo / bi;
      out[i] = (rhs[i] - lo * out[i - 1]) / bi;
    }
    for (int i = n - 2; i >= 0; --i) out[i] -= cp[i] * out[i + 1];
  }
  /* v = (1, 0, ..., 0, lo/gam) */
  const double vy = y[0] + lo / gam * y[n - 1], vz = z[0] + lo / gam * z[n - 1];
  const double fac = vy / (1.0 + vz);
  for (int i = 0; i < n; ++i) a[i] = y[i] - fac * z[i];
}

void om_grid_spline_coefficients(const double *c, const int n[3], double *out)
{
  const int nx = n[0], ny = n[1], nz = n[2];
  const size_t N = (size_t)nx * ny * nz;
  memcpy(out, c, N * sizeof(double));
  const int nm = nx > ny ? (nx > nz ? nx : nz) : (ny > nz ? ny : nz);
  double *f = (double *)malloc(sizeof(double) * nm), *a = (double *)malloc(sizeof(double) * nm);
  double *wk = (double *)malloc(sizeof(double) * 4 * nm);
  for (int axis = 0; axis < 3; ++axis) {
    const int len = n[axis];
    const size_t stride = axis == 0 ? 1 : (axis == 1 ? (size_t)nx : (size_t)nx * ny);
    for (size_t base = 0; base < N; ++base) {
      /* one line per base index whose coordinate along the axis is 0 */
      const size_t coord = (base / stride) % len;
      if (coord != 0) continue;
      for (int i = 0; i < len; ++i) f[i] = out[base + i * stride];
      om_cyclic_solve(len, f, a, wk);
      for (int i = 0; i < len; ++i) out[base + i * stride] = a[i];
    }
  }
  free(f);
  free(a);
  free(wk);
}

/* Cubic B-spline weights of the four nodes i-1 .. i+2 at fraction t, and
 * their first and second derivatives in t. */
static void om_bspline(double t, double w[4], double d1[4], double d2[4])
{
  const double s = 1.0 - t;
  w[0] = s * s * s / 6.0;
  w[1] = (3.0 * t * t * t - 6.0 * t * t + 4.0) / 6.0;
  w[2] = (-3.0 * t * t * t + 3.0 * t * t + 3.0 * t + 1.0) / 6.0;
  w[3] = t * t * t / 6.0;
  d1[0] = -s * s / 2.0;
  d1[1] = (9.0 * t * t - 12.0 * t) / 6.0;
  d1[2] = (-9.0 * t * t + 6.0 * t + 3.0) / 6.0;
  d1[3] = t * t / 2.0;
  d2[0] = s;
  d2[1] = 3.0 * t - 2.0;
  d2[2] = -3.0 * t + 1.0;
  d2[3] = t;
}

/* Layer index of point x in a layered medium. */
int om_layer_of(const om_medium *m, const double x[3])
{
  if (m->kind != OM_LAYERED) return 0;
  if (m->geometry == 1) {
    double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    int L = 0;
    while (L < m->nlayer - 1 && r < m->bound[L]) ++L;
    return L;
  }
  int L = 0;
  while (L < m->nlayer - 1 && x[2] > m->bound[L]) ++L;
  return L;
}

/* Speed of wave type sp (0 = P, 1 = S) at x in layer `layer`, with gradient
 * and Hessian (H[i][j] = d2c/dx_i dx_j). */
void om_speed(const om_medium *m, int sp, int layer, const double x[3],
              double *c, double gc[3], double H[3][3])
{
  memset(gc, 0, 3 * sizeof(double));
  memset(H, 0, 9 * sizeof(double));
  switch (m->kind) {
  case OM_HOMOGENEOUS:
    *c = sp == 0 ? m->cp : m->cs;
    return;
  case OM_LAYERED: {
    const double c0 = sp == 0 ? m->cpl[layer] : m->csl[layer];
    const double gm = m->gradl[layer];
    *c = c0;
    if (gm != 0.0) {
      if (m->geometry == 1) {
        /* c = c0 (1 + gm r): grad c = c0 gm x/r, Hess c = c0 gm (I - x x^T/r^2)/r */
        const double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        *c = c0 * (1.0 + gm * r);
        for (int i = 0; i < 3; ++i) gc[i] = c0 * gm * x[i] / r;
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) H[i][j] = c0 * gm * ((i == j ? 1.0 : 0.0) - x[i] * x[j] / (r * r)) / r;
      } else {
        *c = c0 * (1.0 + gm * x[2]);
        gc[2] = c0 * gm;
      }
    }
    const double al = m->anom_amp[layer];
    if (al != 0.0) {
      /* c = g f with f = 1 - al E, E = exp(-beta q): the product rule for the
       * gradient, f H_g + grad g (x) grad f + grad f (x) grad g + g H_f for the Hessian;
       * grad f = al E beta 2 w d, H_f = al E (2 beta diag(w) - 4 beta^2 (w d)(w d)^T) */
      const double be = m->anom_beta[layer];
      double wd[3], q = 0.0;
      for (int d = 0; d < 3; ++d) {
        const double dd = x[d] - m->anom_x[layer][d];
        wd[d] = m->anom_w[layer][d] * dd;
        q += wd[d] * dd;
      }
      const double E = exp(-be * q);
      const double f = 1.0 - al * E;
      double gf[3], Hf[3][3];
      for (int i = 0; i < 3; ++i) gf[i] = al * E * be * 2.0 * wd[i];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          Hf[i][j] = al * E * ((i == j ? 2.0 * be * m->anom_w[layer][i] : 0.0) - 4.0 * be * be * wd[i] * wd[j]);
      const double g = *c;
      double gg[3], Hg[3][3];
      for (int i = 0; i < 3; ++i) gg[i] = gc[i];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Hg[i][j] = H[i][j];
      *c = g * f;
      for (int i = 0; i < 3; ++i) gc[i] = f * gg[i] + g * gf[i];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) H[i][j] = f * Hg[i][j] + gg[i] * gf[j] + gf[i] * gg[j] + g * Hf[i][j];
    }
    return;
  }
  case OM_BUMP: {
    double c0 = sp == 0 ? m->cp : m->cs;
    double d[3] = {x[0] - m->x0[0], x[1] - m->x0[1], x[2] - m->x0[2]};
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double s2 = m->s * m->s;
    double E = m->amp * exp(-r2 / (2.0 * s2));
    *c = c0 * (1.0 + E);
    for (int i = 0; i < 3; ++i) gc[i] = -c0 * E * d[i] / s2;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        H[i][j] = c0 * E * (d[i] * d[j] / (s2 * s2) - (i == j ? 1.0 / s2 : 0.0));
    return;
  }
  case OM_LINEAR: {
    double c0 = sp == 0 ? m->cp : m->cs;
    *c = c0 * (1.0 + m->g[0] * x[0] + m->g[1] * x[1] + m->g[2] * x[2]);
    for (int i = 0; i < 3; ++i) gc[i] = c0 * m->g[i];
    return;
  }
  case OM_GRID: {
    const int nx = m->n[0], ny = m->n[1], nz = m->n[2];
    if (m->smooth) {
      /* the periodic cubic B-spline through the node values and its derivatives */
      int i0[3];
      double w[3][4], d1[3][4], d2[3][4];
      for (int d = 0; d < 3; ++d) {
        double u = (x[d] - m->lo[d]) / m->h[d];
        double fl = floor(u);
        long long ii = (long long)fl % m->n[d];
        if (ii < 0) ii += m->n[d];
        i0[d] = (int)ii;
        om_bspline(u - fl, w[d], d1[d], d2[d]);
        for (int a = 0; a < 4; ++a) {
          d1[d][a] /= m->h[d];
          d2[d][a] /= m->h[d] * m->h[d];
        }
      }
      const double *cf = m->coef;
      double scale = 1.0;
      if (sp == 1) {
        if (m->two_fields) cf += (size_t)nx * ny * nz;
        else scale = m->cs_ratio;
      }
      double v = 0.0, g[3] = {0, 0, 0}, hh[3][3] = {{0}};
      for (int c3 = 0; c3 < 4; ++c3)
        for (int b = 0; b < 4; ++b)
          for (int a = 0; a < 4; ++a) {
            const int ix = (i0[0] - 1 + a + nx) % nx, iy = (i0[1] - 1 + b + ny) % ny, iz = (i0[2] - 1 + c3 + nz) % nz;
            const double co = cf[((size_t)iz * ny + iy) * nx + ix];
            const double wx = w[0][a], wy = w[1][b], wz = w[2][c3];
            v += co * wx * wy * wz;
            g[0] += co * d1[0][a] * wy * wz;
            g[1] += co * wx * d1[1][b] * wz;
            g[2] += co * wx * wy * d1[2][c3];
            hh[0][0] += co * d2[0][a] * wy * wz;
            hh[1][1] += co * wx * d2[1][b] * wz;
            hh[2][2] += co * wx * wy * d2[2][c3];
            hh[0][1] += co * d1[0][a] * d1[1][b] * wz;
            hh[0][2] += co * d1[0][a] * wy * d1[2][c3];
            hh[1][2] += co * wx * d1[1][b] * d1[2][c3];
          }
      *c = scale * v;
      for (int i = 0; i < 3; ++i) gc[i] = scale * g[i];
      H[0][0] = scale * hh[0][0]; H[1][1] = scale * hh[1][1]; H[2][2] = scale * hh[2][2];
      H[0][1] = H[1][0] = scale * hh[0][1];
      H[0][2] = H[2][0] = scale * hh[0][2];
      H[1][2] = H[2][1] = scale * hh[1][2];
      return;
    }
    /* trilinear interpolation of the ten derived node fields */
    int i0[3];
    double t[3];
    for (int d = 0; d < 3; ++d) {
      double u = (x[d] - m->lo[d]) / m->h[d];
      double fl = floor(u);
      t[d] = u - fl;
      long long ii = (long long)fl % m->n[d];
      if (ii < 0) ii += m->n[d];
      i0[d] = (int)ii;
    }
    const double *tab = m->tab;
    double scale = 1.0;
    if (sp == 1) {
      if (m->two_fields) tab += (size_t)10 * nx * ny * nz;
      else scale = m->cs_ratio;
    }
    double v[10] = {0};
    for (int corner = 0; corner < 8; ++corner) {
      int dx = corner & 1, dy = (corner >> 1) & 1, dz = (corner >> 2) & 1;
      int ix = (i0[0] + dx) % nx, iy = (i0[1] + dy) % ny, iz = (i0[2] + dz) % nz;
      double wgt = (dx ? t[0] : 1.0 - t[0]) * (dy ? t[1] : 1.0 - t[1]) * (dz ? t[2] : 1.0 - t[2]);
      const double *o = tab + 10 * ((size_t)(iz * ny + iy) * nx + ix);
      for (int f = 0; f < 10; ++f) v[f] += wgt * o[f];
    }
    for (int f = 0; f < 10; ++f) v[f] *= scale;
    *c = v[0];
    gc[0] = v[1]; gc[1] = v[2]; gc[2] = v[3];
    H[0][0] = v[4]; H[1][1] = v[5]; H[2][2] = v[6];
    H[0][1] = H[1][0] = v[7];
    H[0][2] = H[2][0] = v[8];
    H[1][2] = H[2][1] = v[9];
    return;
  }
  }
}

/* ------------------------------------------------------------------------ */
/* Beams                                                                     */
/* ------------------------------------------------------------------------ */

/* One frozen Gaussian packet.  ZQ[m][j] = d Q_j / d z_m, ZP likewise, with
 * d/dz = d/dq - i d/dp (eq:op_zZ_app).  P beams carry a[0] = a_P; S beams
 * carry (a[0], a[1]) = (a_SV, a_SH) in the frame
 *   N_SH = (e x P)/|e x P|,  N_SV = (P/|P|) x N_SH
 * built from the reference axis e (the paper only requires two unit vectors
 * orthogonal to P; this frame is the reading used here).  w folds the weight
 * psi, the cell volumes and the (k/2 pi)^{9/2} normalisation of eq:FGA. */
typedef struct {
  double Q[3], P[3];
  cplx ZQ[3][3], ZP[3][3];
  cplx a[2];
  double S;
  cplx w;
  double e[3];
  int32_t branch;   /* 0 = P, 1 = SH, 2 = SV */
  int32_t sigma;    /* +1 or -1: the "+" or "-" propagation direction */
  int32_t layer;
  int32_t gen;
  int32_t alive;
  int64_t lineage;
} om_beam;

size_t om_beam_size(void) { return sizeof(om_beam); }

typedef struct {
  double Q[3], P[3];
  cplx ZQ[3][3], ZP[3][3];
  cplx a[2];
  double S;
} om_state;

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double a[3], const double b[3], double o[3])
{
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

/* SH / SV polarisation directions for momentum P and reference axis e. */
void om_s_frame(const double P[3], const double e[3], double nsh[3], double nsv[3])
{
  double ex[3], ph[3];
  cross3(e, P, ex);
  double n = sqrt(dot3(ex, ex));
  for (int i = 0; i < 3; ++i) nsh[i] = ex[i] / n;
  double np = sqrt(dot3(P, P));
  for (int i = 0; i < 3; ++i) ph[i] = P[i] / np;
  cross3(ph, nsh, nsv);
}

/* Reference axis for a new S beam: e_z, unless P is within 20 degrees of it,
 * then e_x. */
void om_initial_axis(const double P[3], double e[3])
{
  double np = sqrt(dot3(P, P));
  e[0] = e[1] = e[2] = 0.0;
  if (fabs(P[2]) / np > cos(20.0 * M_PI / 180.0)) e[0] = 1.0;
  else e[2] = 1.0;
}

/* Solve Z X = B for complex 3x3 matrices by Gaussian elimination with
 * partial pivoting. */
static void csolve3(cplx Z[3][3], cplx B[3][3], cplx X[3][3])
{
  cplx A[3][3], R[3][3];
  memcpy(A, Z, sizeof(A));
  memcpy(R, B, sizeof(R));
  for (int col = 0; col < 3; ++col) {
    int piv = col;
    for (int r = col + 1; r < 3; ++r)
      if (cabs(A[r][col]) > cabs(A[piv][col])) piv = r;
    if (piv != col) {
      for (int j = 0; j < 3; ++j) {
        cplx t = A[col][j]; A[col][j] = A[piv][j]; A[piv][j] = t;
        t = R[col][j]; R[col][j] = R[piv][j]; R[piv][j] = t;
      }
    }
    for (int r = col + 1; r < 3; ++r) {
      cplx f = A[r][col] / A[col][col];
      for (int j = 0; j < 3; ++j) { A[r][j] -= f * A[col][j]; R[r][j] -= f * R[col][j]; }
    }
  }
  for (int col = 2; col >= 0; --col)
    for (int j = 0; j < 3; ++j) {
      cplx s = R[col][j];
      for (int k = col + 1; k < 3; ++k) s -= A[col][k] * X[k][j];
      X[col][j] = s / A[col][col];
    }
}

/* Right-hand side of the FGA ODE system for one beam (Sec. 2.2):
 *   dQ/dt = sigma c P/|P|,  dP/dt = -sigma |P| grad c            (eq:char_plus / eq:char_minus)
 *   d(dzQ)/dt, d(dzP)/dt from eq:DzDt, times sigma for the "-" flow
 *   da_P/dt = a_P (sigma grad c . P/|P| + tr(Z^{-1} dZ/dt)/2)      (eq:amp_P)
 *   da_SV/dt = s a_SV - a_SH (dN_SH/dt . N_SV)                     (eq:amp_SV)
 *   da_SH/dt = s a_SH + a_SV (dN_SH/dt . N_SV)                     (eq:amp_SH)
 *   dS/dt = P . dQ/dt - H, H = sigma c |P|
 * The action S is not in the paper's ansatz; since H is homogeneous of degree
 * one in P it stays zero up to rounding, and is carried so that the phase
 * factor exp(i k S) is explicit. */
static cplx om_rhs_core(const om_medium *m, const om_beam *b, const om_state *y, om_state *dy, double gc_out[3]);

void om_rhs(const om_medium *m, const om_beam *b, const om_state *y, om_state *dy)
{
  double gc[3];
  const cplx s = om_rhs_core(m, b, y, dy, gc);
  const double *P = y->P;
  if (b->branch == 0) {
    dy->a[0] = s * y->a[0];
    dy->a[1] = 0;
  } else {
    /* omega = dN_SH/dt . N_SV, with N_SH = (e x P)/|e x P| differentiated
     * along dP/dt (e is fixed during a step). */
    double ex[3], exd[3], nsh[3], nsv[3];
    cross3(b->e, P, ex);
    cross3(b->e, dy->P, exd);
    double n2 = dot3(ex, ex), n = sqrt(n2);
    double proj = dot3(ex, exd);
    double dnsh[3];
    for (int i = 0; i < 3; ++i) dnsh[i] = exd[i] / n - ex[i] * proj / (n2 * n);
    om_s_frame(P, b->e, nsh, nsv);
    double om = dot3(dnsh, nsv);
    dy->a[0] = s * y->a[0] - om * y->a[1];
    dy->a[1] = s * y->a[1] + om * y->a[0];
  }
}

/* Everything but the amplitudes: dQ, dP, d(dzQ), d(dzP), dS; returns the
 * amplitude rate s of eq:amp_P / eq:amp_SV / eq:amp_SH (without the frame
 * coupling) and grad c. */
static cplx om_rhs_core(const om_medium *m, const om_beam *b, const om_state *y, om_state *dy, double gc_out[3])
{
  const int sp = b->branch == 0 ? 0 : 1;
  const double sg = (double)b->sigma;
  double c, gc[3], H[3][3];
  om_speed(m, sp, b->layer, y->Q, &c, gc, H);
  const double *P = y->P;
  const double np = sqrt(dot3(P, P));

  for (int j = 0; j < 3; ++j) {
    dy->Q[j] = sg * c * P[j] / np;
    dy->P[j] = -sg * gc[j] * np;
  }
  /* eq:DzDt:  d(dzQ)/dt = dzQ (grad c (x) P)/|P| + c dzP (I/|P| - P (x) P/|P|^3)
   *           d(dzP)/dt = -|P| dzQ Hess(c) - dzP (P (x) grad c)/|P|           */
  for (int mm = 0; mm < 3; ++mm)
    for (int j = 0; j < 3; ++j) {
      cplx zq = 0, zp = 0;
      for (int l = 0; l < 3; ++l) {
        double Mq = gc[l] * P[j] / np;
        double Mp = (l == j ? 1.0 / np : 0.0) - P[l] * P[j] / (np * np * np);
        zq += y->ZQ[mm][l] * Mq + c * y->ZP[mm][l] * Mp;
        zp += -np * y->ZQ[mm][l] * H[l][j] - y->ZP[mm][l] * P[l] * gc[j] / np;
      }
      dy->ZQ[mm][j] = sg * zq;
      dy->ZP[mm][j] = sg * zp;
    }
  /* tr(Z^{-1} dZ/dt), Z = dzQ + i dzP */
  cplx Z[3][3], dZ[3][3], X[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      Z[i][j] = y->ZQ[i][j] + I * y->ZP[i][j];
      dZ[i][j] = dy->ZQ[i][j] + I * dy->ZP[i][j];
    }
  csolve3(Z, dZ, X);
  cplx tr = X[0][0] + X[1][1] + X[2][2];
  cplx s = sg * dot3(gc, P) / np + 0.5 * tr;
  dy->S = dot3(P, dy->Q) - sg * c * np;
  for (int i = 0; i < 3; ++i) gc_out[i] = gc[i];
  return s;
}

static void st_from_beam(const om_beam *b, om_state *y)
{
  memcpy(y->Q, b->Q, sizeof(y->Q));
  memcpy(y->P, b->P, sizeof(y->P));
  memcpy(y->ZQ, b->ZQ, sizeof(y->ZQ));
  memcpy(y->ZP, b->ZP, sizeof(y->ZP));
  y->a[0] = b->a[0]; y->a[1] = b->a[1];
  y->S = b->S;
}

static void st_to_beam(const om_state *y, om_beam *b)
{
  memcpy(b->Q, y->Q, sizeof(y->Q));
  memcpy(b->P, y->P, sizeof(y->P));
  memcpy(b->ZQ, y->ZQ, sizeof(y->ZQ));
  memcpy(b->ZP, y->ZP, sizeof(y->ZP));
  b->a[0] = y->a[0]; b->a[1] = y->a[1];
  b->S = y->S;
}

/* out = y + h*k, field by field */
static void st_axpy(om_state *out, const om_state *y, double h, const om_state *k)
{
  for (int i = 0; i < 3; ++i) { out->Q[i] = y->Q[i] + h * k->Q[i]; out->P[i] = y->P[i] + h * k->P[i]; }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      out->ZQ[i][j] = y->ZQ[i][j] + h * k->ZQ[i][j];
      out->ZP[i][j] = y->ZP[i][j] + h * k->ZP[i][j];
    }
  out->a[0] = y->a[0] + h * k->a[0];
  out->a[1] = y->a[1] + h * k->a[1];
  out->S = y->S + h * k->S;
}

/* Classic fourth-order Runge-Kutta step of size dt (Sec. 2.3: fixed-step
 * RK4): y' = y + dt/6 (k1 + 2 k2 + 2 k3 + k4). */
void om_rk4_step(const om_medium *m, om_beam *b, double dt)
{
  om_state y, k1, k2, k3, k4, t;
  st_from_beam(b, &y);
  om_rhs(m, b, &y, &k1);
  st_axpy(&t, &y, 0.5 * dt, &k1);
  om_rhs(m, b, &t, &k2);
  st_axpy(&t, &y, 0.5 * dt, &k2);
  om_rhs(m, b, &t, &k3);
  st_axpy(&t, &y, dt, &k3);
  om_rhs(m, b, &t, &k4);
  om_state out;
  for (int i = 0; i < 3; ++i) {
    out.Q[i] = y.Q[i] + dt / 6.0 * (k1.Q[i] + 2.0 * k2.Q[i] + 2.0 * k3.Q[i] + k4.Q[i]);
    out.P[i] = y.P[i] + dt / 6.0 * (k1.P[i] + 2.0 * k2.P[i] + 2.0 * k3.P[i] + k4.P[i]);
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      out.ZQ[i][j] = y.ZQ[i][j] + dt / 6.0 * (k1.ZQ[i][j] + 2.0 * k2.ZQ[i][j] + 2.0 * k3.ZQ[i][j] + k4.ZQ[i][j]);
      out.ZP[i][j] = y.ZP[i][j] + dt / 6.0 * (k1.ZP[i][j] + 2.0 * k2.ZP[i][j] + 2.0 * k3.ZP[i][j] + k4.ZP[i][j]);
    }
  for (int i = 0; i < 2; ++i)
    out.a[i] = y.a[i] + dt / 6.0 * (k1.a[i] + 2.0 * k2.a[i] + 2.0 * k3.a[i] + k4.a[i]);
  out.S = y.S + dt / 6.0 * (k1.S + 2.0 * k2.S + 2.0 * k3.S + k4.S);
  st_to_beam(&out, b);
}

/* After a step: if an S beam's momentum has come within 10 degrees of its
 * reference axis, switch to the other axis (e_z <-> e_x) and re-express the
 * physical polarisation a_SV N_SV + a_SH N_SH in the new frame. */
void om_reframe(om_beam *b)
{
  if (b->branch == 0) return;
  double np = sqrt(dot3(b->P, b->P));
  if (fabs(dot3(b->P, b->e)) / np <= cos(10.0 * M_PI / 180.0)) return;
  double nsh[3], nsv[3], e2[3] = {0, 0, 0};
  om_s_frame(b->P, b->e, nsh, nsv);
  cplx A[3];
  for (int i = 0; i < 3; ++i) A[i] = b->a[0] * nsv[i] + b->a[1] * nsh[i];
  if (b->e[2] != 0.0 && b->e[0] == 0.0 && b->e[1] == 0.0) e2[0] = 1.0;
  else e2[2] = 1.0;
  memcpy(b->e, e2, sizeof(e2));
  om_s_frame(b->P, b->e, nsh, nsv);
  b->a[0] = A[0] * nsv[0] + A[1] * nsv[1] + A[2] * nsv[2];
  b->a[1] = A[0] * nsh[0] + A[1] * nsh[1] + A[2] * nsh[2];
}

/* Advance n beams by nsteps RK4 steps of size dt (no interfaces). */
void om_evolve(const om_medium *m, om_beam *beams, int64_t n, double dt, int nsteps)
{
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    if (!beams[i].alive) continue;
    for (int s = 0; s < nsteps; ++s) {
      om_rk4_step(m, &beams[i], dt);
      om_reframe(&beams[i]);
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Frame-free S polarisation                                                 */
/* ------------------------------------------------------------------------ */

/* The S amplitude as the physical polarisation vector A = a_SV N_SV + a_SH N_SH
 * (complex, orthogonal to P).  Differentiating that sum under the framed
 * equations (eq:amp_SV, eq:amp_SH, coupling omega = dN_SH/dt . N_SV) leaves
 *   dA/dt = s A - (A . dPhat/dt) Phat,  dPhat/dt = (dP/dt - Phat (Phat . dP/dt))/|P|,
 * with the same scalar rate s: A is carried along the ray by parallel
 * transport and needs no reference axis.  The rest of the state follows the
 * same equations as in om_rhs. */
static void om_rhs_vec(const om_medium *m, const om_beam *b, const om_state *y, const cplx A[3], om_state *dy,
                       cplx dA[3])
{
  double gc[3];
  const cplx s = om_rhs_core(m, b, y, dy, gc);
  dy->a[0] = dy->a[1] = 0;
  const double np = sqrt(dot3(y->P, y->P));
  double ph[3], dph[3];
  for (int i = 0; i < 3; ++i) ph[i] = y->P[i] / np;
  const double pd = dot3(ph, dy->P);
  for (int i = 0; i < 3; ++i) dph[i] = (dy->P[i] - ph[i] * pd) / np;
  const cplx ad = A[0] * dph[0] + A[1] * dph[1] + A[2] * dph[2];
  for (int i = 0; i < 3; ++i) dA[i] = s * A[i] - ad * ph[i];
}

/* One classic RK4 step of an S beam in the frame-free form; afterwards A is
 * projected on the plane orthogonal to the new P (the exact solution stays
 * there; the projection removes the step's truncation drift out of it). */
static void om_rk4_step_vec(const om_medium *m, om_beam *b, cplx A[3], double dt)
{
  om_state y, k[4], t;
  cplx kA[4][3], tA[3];
  st_from_beam(b, &y);
  const double h[4] = {0.0, 0.5 * dt, 0.5 * dt, dt};
  for (int st = 0; st < 4; ++st) {
    if (st == 0) {
      t = y;
      for (int i = 0; i < 3; ++i) tA[i] = A[i];
    } else {
      st_axpy(&t, &y, h[st], &k[st - 1]);
      for (int i = 0; i < 3; ++i) tA[i] = A[i] + h[st] * kA[st - 1][i];
    }
    om_rhs_vec(m, b, &t, tA, &k[st], kA[st]);
  }
  om_state out;
  for (int i = 0; i < 3; ++i) {
    out.Q[i] = y.Q[i] + dt / 6.0 * (k[0].Q[i] + 2.0 * k[1].Q[i] + 2.0 * k[2].Q[i] + k[3].Q[i]);
    out.P[i] = y.P[i] + dt / 6.0 * (k[0].P[i] + 2.0 * k[1].P[i] + 2.0 * k[2].P[i] + k[3].P[i]);
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      out.ZQ[i][j] = y.ZQ[i][j] + dt / 6.0 * (k[0].ZQ[i][j] + 2.0 * k[1].ZQ[i][j] + 2.0 * k[2].ZQ[i][j] + k[3].ZQ[i][j]);
      out.ZP[i][j] = y.ZP[i][j] + dt / 6.0 * (k[0].ZP[i][j] + 2.0 * k[1].ZP[i][j] + 2.0 * k[2].ZP[i][j] + k[3].ZP[i][j]);
    }
  out.a[0] = y.a[0];
  out.a[1] = y.a[1];
  out.S = y.S + dt / 6.0 * (k[0].S + 2.0 * k[1].S + 2.0 * k[2].S + k[3].S);
  for (int i = 0; i < 3; ++i) A[i] += dt / 6.0 * (kA[0][i] + 2.0 * kA[1][i] + 2.0 * kA[2][i] + kA[3][i]);
  st_to_beam(&out, b);
  const double np = sqrt(dot3(b->P, b->P));
  double ph[3];
  for (int i = 0; i < 3; ++i) ph[i] = b->P[i] / np;
  const cplx ap = A[0] * ph[0] + A[1] * ph[1] + A[2] * ph[2];
  for (int i = 0; i < 3; ++i) A[i] -= ap * ph[i];
}

/* Advance n beams by nsteps RK4 steps with S amplitudes in the frame-free
 * form: A is formed from (a_SV, a_SH) and the beam's frame, advanced, and
 * returned to the frame at the end (the axis switched first if P has come
 * within 10 degrees of it, as om_reframe does).  P beams step as in om_evolve. */
void om_evolve_svec(const om_medium *m, om_beam *beams, int64_t n, double dt, int nsteps)
{
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    om_beam *b = &beams[i];
    if (!b->alive) continue;
    if (b->branch == 0) {
      for (int s = 0; s < nsteps; ++s) om_rk4_step(m, b, dt);
      continue;
    }
    double nsh[3], nsv[3];
    om_s_frame(b->P, b->e, nsh, nsv);
    cplx A[3];
    for (int d = 0; d < 3; ++d) A[d] = b->a[0] * nsv[d] + b->a[1] * nsh[d];
    for (int s = 0; s < nsteps; ++s) om_rk4_step_vec(m, b, A, dt);
    const double np = sqrt(dot3(b->P, b->P));
    if (fabs(dot3(b->P, b->e)) / np > cos(10.0 * M_PI / 180.0)) {
      const int was_z = b->e[2] != 0.0 && b->e[0] == 0.0 && b->e[1] == 0.0;
      b->e[0] = was_z ? 1.0 : 0.0;
      b->e[1] = 0.0;
      b->e[2] = was_z ? 0.0 : 1.0;
    }
    om_s_frame(b->P, b->e, nsh, nsv);
    b->a[0] = A[0] * nsv[0] + A[1] * nsv[1] + A[2] * nsv[2];
    b->a[1] = A[0] * nsh[0] + A[1] * nsh[1] + A[2] * nsh[2];
  }
}

/* ------------------------------------------------------------------------ */
/* Initial decomposition (Sec. 2.1, eq:psi, eq:alpha^k)                      */
/* ------------------------------------------------------------------------ */

/* FBI transform of one vector field sampled on the uniform quadrature mesh
 * (ylo + i*yh, x index fastest, array [3][z][y][x]):
 *   Ft_c(q, p) = sum_y yh^3 f_c(y) exp(-i p.(y-q)/eps - |y-q|^2/(2 eps)).
 * The kernel is the product of its three one-dimensional factors, which are
 * tabulated first. */
void om_fbi(const cplx *f, const int yn[3], const double ylo[3], const double yh[3],
            const double q[3], const double p[3], double eps, cplx out[3])
{
  cplx *K[3];
  for (int d = 0; d < 3; ++d) {
    K[d] = (cplx *)malloc(sizeof(cplx) * yn[d]);
    for (int i = 0; i < yn[d]; ++i) {
      double u = ylo[d] + i * yh[d] - q[d];
      K[d][i] = cexp(-I * p[d] * u / eps - u * u / (2.0 * eps));
    }
  }
  const size_t plane = (size_t)yn[0] * yn[1] * yn[2];
  cplx acc[3] = {0, 0, 0};
  for (int iz = 0; iz < yn[2]; ++iz)
    for (int iy = 0; iy < yn[1]; ++iy) {
      cplx kyz = K[2][iz] * K[1][iy];
      for (int ix = 0; ix < yn[0]; ++ix) {
        cplx kk = kyz * K[0][ix];
        size_t o = ((size_t)iz * yn[1] + iy) * yn[0] + ix;
        for (int c = 0; c < 3; ++c) acc[c] += f[c * plane + o] * kk;
      }
    }
  double vol = yh[0] * yh[1] * yh[2];
  for (int c = 0; c < 3; ++c) out[c] = acc[c] * vol;
  for (int d = 0; d < 3; ++d) free(K[d]);
}

/* Unit polarisation of branch b at momentum p with reference axis e. */
static void om_polarisation(int branch, const double p[3], const double e[3], double nh[3])
{
  if (branch == 0) {
    double np = sqrt(dot3(p, p));
    for (int i = 0; i < 3; ++i) nh[i] = p[i] / np;
  } else {
    double nsh[3], nsv[3];
    om_s_frame(p, e, nsh, nsv);
    for (int i = 0; i < 3; ++i) nh[i] = branch == 1 ? nsh[i] : nsv[i];
  }
}

/* Test hook, 0 in every use but one: the pins of the two-way weight set it to
 * plant a known mistake in om_psi (1: the g-term doubled, 2: the g-term's sign
 * flipped, 3: |p|^3 in place of |p|, 4: the 1/2 on f dropped) and check that
 * their test then fails. */
int om_plant_twoway_error = 0;

/* Weight of one beam from the branch projections fn = FBI[f].n_b and
 * gn = FBI[g/c_b].n_b for direction sigma = +-1 (eq:psi with eq:alpha^k read
 * with prefactor 1/(2 k c |p|), k = 1/eps):
 *   psi = (1/2) fn + sigma (i eps / (2 |p|)) gn. */
static cplx om_psi(cplx fn, cplx gn, int sigma, double eps, double np)
{
  double half = 0.5, gscale = 1.0, pden = np;
  switch (om_plant_twoway_error) {
  case 1: gscale = 2.0; break;
  case 2: gscale = -1.0; break;
  case 3: pden = np * np * np; break;
  case 4: half = 1.0; break;
  default: break;
  }
  return half * fn + gscale * sigma * I * eps / (2.0 * pden) * gn;
}

/* Build the beams of one (q, p) mesh point from the FBI transforms Ft = FBI[f]
 * and Gt[b] = FBI[g / c_b] (Gt may be NULL when g = 0).
 *   alpha_{+-} = (1/2)(f +- i g/(k c |p|)) . n_b          (eq:alpha^k read with
 * prefactor 1/(2 k c |p|): with a(0) = 2^{3/2} this is the normalisation under
 * which the summation formula returns f at t = 0; the printed |p|^3 does not)
 *   psi_{b,+-} = (1/2) Ft.n_b +- (i eps/(2|p|)) Gt_b.n_b
 * In one-way mode only "+" beams are made and psi_{b,+} = Ft.n_b, i.e. the
 * data is taken to be the "+"-going part of f.
 *   w = psi * dq * dp * (2 pi eps)^{-9/2}                   (eq:FGA)
 * Returns the number of beams written (<= 6). */
int om_make_beams(const double q[3], const double p[3], const cplx Ft[3], const cplx *Gt,
                  int one_way, double eps, double dq, double dp, int branch_mask,
                  double cull_abs, int64_t lineage_base, int64_t lineage_stride, om_beam *out)
{
  int nb = 0;
  const double np = sqrt(dot3(p, p));
  const double norm = dq * dp * pow(2.0 * M_PI * eps, -4.5);
  for (int br = 0; br < 3; ++br) {
    if (!(branch_mask & (1 << br))) continue;
    for (int si = 0; si < (one_way ? 1 : 2); ++si) {
      int sg = si == 0 ? 1 : -1;
      double e[3], nh[3];
      om_initial_axis(p, e);
      om_polarisation(br, p, e, nh);
      cplx fn = Ft[0] * nh[0] + Ft[1] * nh[1] + Ft[2] * nh[2];
      cplx psi;
      if (one_way) psi = fn;
      else {
        cplx gn = 0.0;
        if (Gt) {
          const cplx *G = Gt + 3 * (br == 0 ? 0 : 1);
          gn = G[0] * nh[0] + G[1] * nh[1] + G[2] * nh[2];
        }
        psi = om_psi(fn, gn, sg, eps, np);
      }
      int64_t lin = lineage_base + (int64_t)(br * 2 + si) * lineage_stride;
      if (cabs(psi) < cull_abs) continue;
      om_beam *b = &out[nb++];
      memset(b, 0, sizeof(*b));
      memcpy(b->Q, q, 3 * sizeof(double));
      memcpy(b->P, p, 3 * sizeof(double));
      for (int i = 0; i < 3; ++i) { b->ZQ[i][i] = 1.0; b->ZP[i][i] = -I; }
      const double a0 = pow(2.0, 1.5);
      if (br == 0) { b->a[0] = a0; b->a[1] = 0; }
      else if (br == 1) { b->a[0] = 0; b->a[1] = a0; }
      else { b->a[0] = a0; b->a[1] = 0; }
      b->S = 0.0;
      b->w = psi * norm;
      memcpy(b->e, e, sizeof(e));
      b->branch = br;
      b->sigma = sg;
      b->layer = 0;
      b->gen = 0;
      b->alive = 1;
      b->lineage = lin;
    }
  }
  return nb;
}

/* ------------------------------------------------------------------------ */
/* Reconstruction (Sec. 2.1, eq:FGA)                                         */
/* ------------------------------------------------------------------------ */

/* Physical amplitude vector A = a_P P/|P| (P beams) or
 * a_SV N_SV + a_SH N_SH (S beams). */
void om_amplitude_vector(const om_beam *b, cplx A[3])
{
  if (b->branch == 0) {
    double np = sqrt(dot3(b->P, b->P));
    for (int i = 0; i < 3; ++i) A[i] = b->a[0] * b->P[i] / np;
  } else {
    double nsh[3], nsv[3];
    om_s_frame(b->P, b->e, nsh, nsv);
    for (int i = 0; i < 3; ++i) A[i] = b->a[0] * nsv[i] + b->a[1] * nsh[i];
  }
}

/* u(x) = sum_b w_b exp(i S_b/eps) A_b exp(i P_b.(x-Q_b)/eps - |x-Q_b|^2/(2 eps))
 * over the beams whose box window max_d |x_d - Q_d| <= sqrt(2 tau eps)
 * contains x; beams summed in array order.  out is [npt][3] complex.
 * Returns the number of (beam, point) terms evaluated. */
int64_t om_sum_points(const om_beam *beams, int64_t nb, const double *x, int64_t npt,
                      double eps, double tau, cplx *out)
{
  const double R = sqrt(2.0 * tau * eps);
  int64_t count = 0;
#pragma omp parallel for schedule(static) reduction(+ : count)
  for (int64_t ip = 0; ip < npt; ++ip) {
    const double *xp = x + 3 * ip;
    cplx u[3] = {0, 0, 0};
    for (int64_t ib = 0; ib < nb; ++ib) {
      const om_beam *b = &beams[ib];
      if (!b->alive) continue;
      double d[3] = {xp[0] - b->Q[0], xp[1] - b->Q[1], xp[2] - b->Q[2]};
      if (fabs(d[0]) > R || fabs(d[1]) > R || fabs(d[2]) > R) continue;
      ++count;
      cplx A[3];
      om_amplitude_vector(b, A);
      cplx g = b->w * cexp(I * b->S / eps) *
               cexp(I * dot3(b->P, d) / eps - dot3(d, d) / (2.0 * eps));
      for (int c = 0; c < 3; ++c) u[c] += g * A[c];
    }
    for (int c = 0; c < 3; ++c) out[3 * ip + c] = u[c];
  }
  return count;
}

/* ------------------------------------------------------------------------ */
/* Point moment-tensor source (initial data for Step 1, closed form)         */
/* ------------------------------------------------------------------------ */

/* The paper's seismic examples use point sources whose decomposition it
 * defers to another paper; the reading used here: an impulsive moment-tensor
 * source is the initial velocity g = -(1/rho0) M grad delta(x - x0), u(0) = 0.
 * Then FBI[g/c_b](q,p) = (1/rho0) M . grad_y [K(y)/c_b(y)] at y = x0
 * (integration by parts), K(y) = exp(-i p.(y-q)/eps - |y-q|^2/(2 eps)), and
 * with f = 0 the weights are psi_{b,+-} = +-(i eps/(2|p|)) FBI[g/c_b].n_b.
 * A Ricker source wavelet multiplies each beam, whose frequency is
 * c_b |p| / eps, by R(w) = (w/w0)^2 exp(1 - (w/w0)^2), w0 = c_P(x0)/eps.
 * Meshes: q on nq^3 cell-centred points of the cube x0 +- qhalf; p on
 * Fibonacci directions times Gauss-Legendre |p| shells on
 * [shell_lo, shell_hi] * c_P(x0)/c_b(x0), measure |p|^2 w_shell 4 pi / ndir. */
typedef struct {
  double eps;
  double x0[3];
  double M[6];           /* xx, yy, zz, xy, xz, yz                       */
  double rho0;
  int nq;
  double qhalf;
  int ndir, nshell;
  double shell_lo, shell_hi;
  int ricker;
  int branch_mask;
  double cull_abs;
} om_point_source;

/* Unit vectors on the golden spiral: z_i = 1 - (2i+1)/n, azimuth i pi (3 - sqrt 5). */
void om_fibonacci_dirs(int n, double *d)
{
  const double ga = M_PI * (3.0 - sqrt(5.0));
  for (int i = 0; i < n; ++i) {
    const double z = 1.0 - (2.0 * i + 1.0) / n;
    const double r = sqrt(fmax(0.0, 1.0 - z * z));
    d[3 * i] = r * cos(ga * i);
    d[3 * i + 1] = r * sin(ga * i);
    d[3 * i + 2] = z;
  }
}

/* Gauss-Legendre nodes and weights on [a, b]: Newton iteration on P_n from
 * the Chebyshev-like guesses cos(pi (i + 3/4)/(n + 1/2)). */
void om_gauss_legendre(int n, double a, double b, double *x, double *w)
{
  for (int i = 0; i < n; ++i) {
    double t = cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = t; p0 = 1.0; }
      dp = n * (t * p1 - p0) / (t * t - 1.0);
      const double dt = p1 / dp;
      t -= dt;
      if (fabs(dt) < 1e-16) break;
    }
    /* recompute the derivative at the converged node */
    double p0 = 1.0, p1 = t;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    if (n == 1) { p1 = t; p0 = 1.0; }
    dp = n * (t * p1 - p0) / (t * t - 1.0);
    x[i] = 0.5 * (a + b) + 0.5 * (b - a) * t;
    w[i] = (b - a) / ((1.0 - t * t) * dp * dp);
  }
}

double om_ricker(double w, double w0)
{
  const double r = (w / w0) * (w / w0);
  return r * exp(1.0 - r);
}

/* The beams of a point source, in lineage order
 * ((branch*2 + dir) * Np + ip) * Nq + iq with ip = shell * ndir + direction;
 * returns the number written (out must hold the candidate count). */
int64_t om_point_source_beams(const om_medium *m, const om_point_source *src, om_beam *out)
{
  const int L0 = om_layer_of(m, src->x0);
  double cP, gP[3], HP[3][3];
  om_speed(m, 0, L0, src->x0, &cP, gP, HP);
  const double rho0 = src->rho0 > 0.0 ? src->rho0
                      : (m->kind == OM_LAYERED ? m->rhol[L0] : (m->rho > 0.0 ? m->rho : 1.0));
  const int nq = src->nq, Nq = nq * nq * nq, Np = src->ndir * src->nshell;
  const double hq = 2.0 * src->qhalf / nq, dq = hq * hq * hq;
  double *dirs = malloc(sizeof(double) * 3 * src->ndir);
  double *xs = malloc(sizeof(double) * src->nshell), *ws = malloc(sizeof(double) * src->nshell);
  om_fibonacci_dirs(src->ndir, dirs);
  const double eps = src->eps, norm = pow(2.0 * M_PI * eps, -4.5);
  int64_t nb = 0;
  for (int br = 0; br < 3; ++br) {
    if (!(src->branch_mask & (1 << br))) continue;
    const int sp = br == 0 ? 0 : 1;
    double cb, gb[3], Hb[3][3];
    om_speed(m, sp, L0, src->x0, &cb, gb, Hb);
    om_gauss_legendre(src->nshell, src->shell_lo * cP / cb, src->shell_hi * cP / cb, xs, ws);
    for (int si = 0; si < 2; ++si) {
      const int sg = si == 0 ? 1 : -1;
      for (int ip = 0; ip < Np; ++ip) {
        const int sh = ip / src->ndir, dj = ip % src->ndir;
        double p[3];
        for (int k = 0; k < 3; ++k) p[k] = xs[sh] * dirs[3 * dj + k];
        const double np = xs[sh];
        const double dp = np * np * ws[sh] * 4.0 * M_PI / src->ndir;
        double e[3], nh[3];
        om_initial_axis(p, e);
        om_polarisation(br, p, e, nh);
        const double rk = src->ricker ? om_ricker(cb * np / eps, cP / eps) : 1.0;
        for (int iq = 0; iq < Nq; ++iq) {
          const int ix = iq % nq, iy = (iq / nq) % nq, iz = iq / (nq * nq);
          double q[3] = {src->x0[0] - src->qhalf + (ix + 0.5) * hq, src->x0[1] - src->qhalf + (iy + 0.5) * hq,
                         src->x0[2] - src->qhalf + (iz + 0.5) * hq};
          double d[3] = {src->x0[0] - q[0], src->x0[1] - q[1], src->x0[2] - q[2]};
          const cplx K = cexp(-I * dot3(p, d) / eps - dot3(d, d) / (2.0 * eps));
          cplx gradKc[3];
          for (int j = 0; j < 3; ++j)
            gradKc[j] = K * (-I * p[j] / eps - d[j] / eps) / cb - K * gb[j] / (cb * cb);
          const double Mm[3][3] = {{src->M[0], src->M[3], src->M[4]},
                                   {src->M[3], src->M[1], src->M[5]},
                                   {src->M[4], src->M[5], src->M[2]}};
          cplx G[3];
          for (int i = 0; i < 3; ++i) {
            G[i] = 0.0;
            for (int j = 0; j < 3; ++j) G[i] += Mm[i][j] * gradKc[j];
            G[i] /= rho0;
          }
          const cplx gn = G[0] * nh[0] + G[1] * nh[1] + G[2] * nh[2];
          const cplx psi = om_psi(0.0, gn, sg, eps, np) * rk;
          if (cabs(psi) < src->cull_abs) continue;
          om_beam *b = &out[nb++];
          memset(b, 0, sizeof(*b));
          memcpy(b->Q, q, sizeof(q));
          memcpy(b->P, p, sizeof(p));
          for (int i = 0; i < 3; ++i) { b->ZQ[i][i] = 1.0; b->ZP[i][i] = -I; }
          const double a0 = pow(2.0, 1.5);
          if (br == 1) { b->a[0] = 0; b->a[1] = a0; }
          else { b->a[0] = a0; b->a[1] = 0; }
          b->w = psi * dq * dp * norm;
          memcpy(b->e, e, sizeof(e));
          b->branch = br;
          b->sigma = sg;
          b->layer = om_layer_of(m, q);
          b->alive = 1;
          b->lineage = ((int64_t)(br * 2 + si) * Np + ip) * Nq + iq;
        }
      }
    }
  }
  free(dirs);
  free(xs);
  free(ws);
  return nb;
}

size_t om_point_source_size(void) { return sizeof(om_point_source); }

/* Point force with a time function (the accuracy experiment of Sec. 2.3,
 * eq:ex_homo): rho u_tt = L u + F(t) d delta(x - x0) with
 * F(t) = cos(Omega (t + T0)) exp(-(t + T0)^2 / width^2).  Reading used here:
 * by Duhamel's principle u(t) = int ds U(t - s; s), U(.; s) the free wave with
 * U = 0, U_t = F(s) d delta(x - x0)/rho0 at its start, whose two-way weights
 * (eq:psi, eq:alpha^k with f = 0) are
 *   psi_{b,+-}(q, p; s) = +-(i eps/(2|p|)) F(s) (d.n_b)/(rho0 c_b) K(x0; q, p),
 * FBI[delta(. - x0)] = K(x0; q, p) = exp(-i p.(x0 - q)/eps - |x0 - q|^2/(2 eps)).
 * A beam launched at time s from (q, p) has, with the speed c = c_b(x0) near
 * the source, the centre a beam launched at the reference time t_ref from
 * q' = q - sigma c (s - t_ref) p/|p| has; the beams are launched at t_ref
 * from (q', p) with the time integral of the weights folded in:
 *   W(q', p) = int ds psi(q' + sigma c (s - t_ref) p/|p|, p; s),
 * which is a Gaussian integral in s (v = s + T0, v0 = T0 + t_ref,
 * D = x0 - q', D_par = D.p/|p|):
 *   W = sigma (i eps/(2|p|)) (d.n_b)/(rho0 c) exp(-i p.D/eps - |D|^2/(2 eps))
 *       (1/2) sum_{+-} sqrt(pi/A) exp(B_+-^2/(4A) + C),
 *   A = 1/width^2 + c^2/(2 eps),
 *   B_+- = c^2 v0/eps + sigma c D_par/eps + i (sigma c |p|/eps +- Omega),
 *   C = -c^2 v0^2/(2 eps) - sigma c D_par v0/eps - i sigma c |p| v0/eps.
 * (The beams' amplitude change over the source duration is left out.)
 * Meshes, frames, cull and lineage as for the moment-tensor source. */
typedef struct {
  double eps;
  double x0[3];
  double d[3];           /* force vector                                  */
  double rho0;
  int nq;
  double qhalf;
  int ndir, nshell;
  double shell_lo, shell_hi;
  double omega, t0, width, t_ref;
  int branch_mask;
  double cull_abs;
} om_point_force;

size_t om_point_force_size(void) { return sizeof(om_point_force); }

/* The time integral of the weights of one beam; see om_point_force. */
static cplx om_force_time_integral(double c, double np, double dpar, int sg, const om_point_force *src)
{
  const double eps = src->eps, v0 = src->t0 + src->t_ref;
  const double A = 1.0 / (src->width * src->width) + c * c / (2.0 * eps);
  const cplx C = -c * c * v0 * v0 / (2.0 * eps) - sg * c * dpar * v0 / eps - I * (sg * c * np * v0 / eps);
  cplx sum = 0.0;
  for (int k = 0; k < 2; ++k) {
    const double om = k == 0 ? src->omega : -src->omega;
    const cplx B = c * c * v0 / eps + sg * c * dpar / eps + I * (sg * c * np / eps + om);
    sum += sqrt(M_PI / A) * cexp(B * B / (4.0 * A) + C);
  }
  return 0.5 * sum;
}

int64_t om_point_force_beams(const om_medium *m, const om_point_force *src, om_beam *out)
{
  const int L0 = om_layer_of(m, src->x0);
  double cP, gP[3], HP[3][3];
  om_speed(m, 0, L0, src->x0, &cP, gP, HP);
  const double rho0 = src->rho0 > 0.0 ? src->rho0
                      : (m->kind == OM_LAYERED ? m->rhol[L0] : (m->rho > 0.0 ? m->rho : 1.0));
  const int nq = src->nq, Nq = nq * nq * nq, Np = src->ndir * src->nshell;
  const double hq = 2.0 * src->qhalf / nq, dq = hq * hq * hq;
  double *dirs = malloc(sizeof(double) * 3 * src->ndir);
  double *xs = malloc(sizeof(double) * src->nshell), *ws = malloc(sizeof(double) * src->nshell);
  om_fibonacci_dirs(src->ndir, dirs);
  const double eps = src->eps, norm = pow(2.0 * M_PI * eps, -4.5);
  int64_t nb = 0;
  for (int br = 0; br < 3; ++br) {
    if (!(src->branch_mask & (1 << br))) continue;
    const int sp = br == 0 ? 0 : 1;
    double cb, gb[3], Hb[3][3];
    om_speed(m, sp, L0, src->x0, &cb, gb, Hb);
    om_gauss_legendre(src->nshell, src->shell_lo * cP / cb, src->shell_hi * cP / cb, xs, ws);
    for (int si = 0; si < 2; ++si) {
      const int sg = si == 0 ? 1 : -1;
      for (int ip = 0; ip < Np; ++ip) {
        const int sh = ip / src->ndir, dj = ip % src->ndir;
        double p[3], ph[3];
        for (int k = 0; k < 3; ++k) {
          p[k] = xs[sh] * dirs[3 * dj + k];
          ph[k] = dirs[3 * dj + k];
        }
        const double np = xs[sh];
        const double dp = np * np * ws[sh] * 4.0 * M_PI / src->ndir;
        double e[3], nh[3];
        om_initial_axis(p, e);
        om_polarisation(br, p, e, nh);
        const double dn = src->d[0] * nh[0] + src->d[1] * nh[1] + src->d[2] * nh[2];
        for (int iq = 0; iq < Nq; ++iq) {
          const int ix = iq % nq, iy = (iq / nq) % nq, iz = iq / (nq * nq);
          double q[3] = {src->x0[0] - src->qhalf + (ix + 0.5) * hq, src->x0[1] - src->qhalf + (iy + 0.5) * hq,
                         src->x0[2] - src->qhalf + (iz + 0.5) * hq};
          double D[3] = {src->x0[0] - q[0], src->x0[1] - q[1], src->x0[2] - q[2]};
          const cplx K = cexp(-I * dot3(p, D) / eps - dot3(D, D) / (2.0 * eps));
          const cplx gn = dn / (rho0 * cb) * K * om_force_time_integral(cb, np, dot3(D, ph), sg, src);
          const cplx psi = om_psi(0.0, gn, sg, eps, np);
          if (cabs(psi) < src->cull_abs) continue;
          om_beam *b = &out[nb++];
          memset(b, 0, sizeof(*b));
          memcpy(b->Q, q, sizeof(q));
          memcpy(b->P, p, sizeof(p));
          for (int i = 0; i < 3; ++i) { b->ZQ[i][i] = 1.0; b->ZP[i][i] = -I; }
          const double a0 = pow(2.0, 1.5);
          if (br == 1) { b->a[0] = 0; b->a[1] = a0; }
          else { b->a[0] = a0; b->a[1] = 0; }
          b->w = psi * dq * dp * norm;
          memcpy(b->e, e, sizeof(e));
          b->branch = br;
          b->sigma = sg;
          b->layer = om_layer_of(m, q);
          b->alive = 1;
          b->lineage = ((int64_t)(br * 2 + si) * Np + ip) * Nq + iq;
        }
      }
    }
  }
  free(dirs);
  free(xs);
  free(ws);
  return nb;
}

/* ------------------------------------------------------------------------ */
/* Interfaces (Sec. 3.1, eq:p:int, eq:Yilmaz, eq:Inter_DzQDzP)               */
/* ------------------------------------------------------------------------ */

/* If Q lies outside layer L, report the interface crossed and the layer on
 * its far side; returns 0 when Q is inside L (points on an interface count
 * as inside).  Flat media: interface i is z = bound[i] between layer i
 * (below) and i+1 (above).  Spherical media: interface i is |x| = bound[i]
 * between layer i (outside) and i+1 (inside). */
int om_layer_exit(const om_medium *m, int L, const double Q[3], int *iface, int *newL)
{
  if (m->kind != OM_LAYERED) return 0;
  const double v = m->geometry == 1 ? sqrt(dot3(Q, Q)) : Q[2];
  const int nl = m->nlayer;
  if (m->geometry == 1) {
    if (L < nl - 1 && v < m->bound[L]) { *iface = L; *newL = L + 1; return 1; }
    if (L > 0 && v > m->bound[L - 1]) { *iface = L - 1; *newL = L - 1; return 1; }
    if (L == 0 && m->surface > 0.0 && v > m->surface) { *iface = OM_SURFACE; *newL = 0; return 1; }
  } else {
    if (L < nl - 1 && v > m->bound[L]) { *iface = L; *newL = L + 1; return 1; }
    if (L > 0 && v < m->bound[L - 1]) { *iface = L - 1; *newL = L - 1; return 1; }
    if (L == nl - 1 && m->surface > 0.0 && v > m->surface) { *iface = OM_SURFACE; *newL = L; return 1; }
  }
  return 0;
}

/* Level (z or radius) of interface iface, or of the free surface. */
static double om_iface_level(const om_medium *m, int iface) { return iface == OM_SURFACE ? m->surface : m->bound[iface]; }

/* Fraction theta in [0, 1] of the straight segment Q0 -> Q1 at which it meets
 * interface `iface` (layers are homogeneous, so a ray inside one is a
 * straight line and an RK4 step moves Q along it exactly). */
double om_crossing_fraction(const om_medium *m, int iface, const double Q0[3], const double Q1[3])
{
  const double r = om_iface_level(m, iface);
  double th;
  if (m->geometry == 1) {
    /* |Q0 + th D| = r: a th^2 + 2 b th + c = 0; the root where the segment
       first meets the sphere */
    double D[3] = {Q1[0] - Q0[0], Q1[1] - Q0[1], Q1[2] - Q0[2]};
    const double a = dot3(D, D), b = dot3(Q0, D), c = dot3(Q0, Q0) - r * r;
    double disc = b * b - a * c;
    if (disc < 0.0) disc = 0.0;
    const double sq = sqrt(disc);
    /* c > 0: Q0 outside, entering; c <= 0: Q0 inside, leaving */
    th = c > 0.0 ? (-b - sq) / a : (-b + sq) / a;
  } else {
    th = (r - Q0[2]) / (Q1[2] - Q0[2]);
  }
  return th < 0.0 ? 0.0 : (th > 1.0 ? 1.0 : th);
}

/* Complex linear solve A x = b (n <= 4) by Gaussian elimination with partial
 * pivoting; A and b are overwritten. */
static void csolve_n(int n, cplx A[4][4], cplx b[4], cplx x[4])
{
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (cabs(A[r][col]) > cabs(A[piv][col])) piv = r;
    if (piv != col) {
      for (int j = 0; j < n; ++j) { cplx t = A[col][j]; A[col][j] = A[piv][j]; A[piv][j] = t; }
      cplx t = b[col]; b[col] = b[piv]; b[piv] = t;
    }
    for (int r = col + 1; r < n; ++r) {
      cplx f = A[r][col] / A[col][col];
      for (int j = col; j < n; ++j) A[r][j] -= f * A[col][j];
      b[r] -= f * b[col];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    cplx s = b[r];
    for (int j = r + 1; j < n; ++j) s -= A[r][j] * x[j];
    x[r] = s / A[r][r];
  }
}

/* One outgoing plane-wave mode at the interface. */
typedef struct {
  int exists;     /* propagating (not evanescent)                          */
  int sp;         /* 0 = P, 1 = S                                          */
  int side;       /* 0 = reflected (incident layer), 1 = transmitted       */
  double P[3];    /* momentum (global frame)                               */
  cplx A[3];      /* displacement amplitude vector (global frame)          */
} om_mode;

/* Snell's law and the elastic transmission/reflection problem for a plane
 * wave with momentum Pin and complex displacement amplitude vector Ain
 * (polarised along Pin for sp_in = 0, orthogonal to it for sp_in = 1)
 * arriving from layer L at an interface with unit normal n (pointing into
 * the transmission layer newL).
 *   Snell (eq:p:int): every outgoing mode keeps the tangential momentum and
 *   the frequency H = c_in |Pin|, so |P_out| = H / c_out; transmitted modes
 *   keep the sign of the normal component, reflected modes flip it.  A mode
 *   whose normal component would be imaginary is evanescent: it enters the
 *   boundary problem with the decaying imaginary normal component but is not
 *   returned as a beam (the paper is silent on post-critical incidence).
 *   Amplitudes: the paper's printed Zoeppritz system (eq:Yilmaz) is for
 *   potentials and has a misprint in its last right-hand-side entry; here
 *   the same physics is solved directly for displacements: continuity of the
 *   displacement u and of the traction sigma.n across the interface, with
 *   sigma_ij = lambda div(u) delta_ij + mu (d_i u_j + d_j u_i), lambda =
 *   rho (c_P^2 - 2 c_S^2), mu = rho c_S^2, for plane waves u = A d exp(i k.x/eps)
 *   with k = P (the common factor i/eps drops out).  P modes are polarised
 *   along k/|k|, in-plane S modes along e2 x k/|k| and SH modes along e2,
 *   in the local frame e3 = n, e1 = tangential momentum direction,
 *   e2 = e3 x e1.
 * out[0..3] = (P reflected, S reflected, P transmitted, S transmitted). */
void om_interface_modes(const om_medium *m, int L, int newL, const double xc[3], const double n[3], int sp_in,
                        const double Pin[3], const cplx Ain[3], om_mode out[4])
{
  /* speeds of both wave types on both sides at the crossing point xc (the
     layer constants where the layers are homogeneous) */
  double cP[2], cS[2];
  {
    double gdum[3], Hdum[3][3];
    om_speed(m, 0, L, xc, &cP[0], gdum, Hdum);
    om_speed(m, 1, L, xc, &cS[0], gdum, Hdum);
    om_speed(m, 0, newL, xc, &cP[1], gdum, Hdum);
    om_speed(m, 1, newL, xc, &cS[1], gdum, Hdum);
  }
  const double c_in = sp_in == 0 ? cP[0] : cS[0];
  const double H = c_in * sqrt(dot3(Pin, Pin));
  const double pn = dot3(Pin, n);
  double pt[3] = {Pin[0] - pn * n[0], Pin[1] - pn * n[1], Pin[2] - pn * n[2]};
  const double p1 = sqrt(dot3(pt, pt));
  double e1[3], e2[3];
  if (p1 > 1e-12 * sqrt(dot3(Pin, Pin))) {
    for (int i = 0; i < 3; ++i) e1[i] = pt[i] / p1;
  } else {
    /* normal incidence: any tangent direction (the problem is symmetric) */
    double t[3] = {1.0, 0.0, 0.0};
    if (fabs(n[0]) > 0.9) { t[0] = 0.0; t[1] = 1.0; }
    const double tn = dot3(t, n);
    for (int i = 0; i < 3; ++i) t[i] -= tn * n[i];
    const double nt = sqrt(dot3(t, t));
    for (int i = 0; i < 3; ++i) e1[i] = t[i] / nt;
  }
  cross3(n, e1, e2);
  const double sgn = pn >= 0.0 ? 1.0 : -1.0;
  /* media of the two sides */
  const double rho[2] = {m->rhol[L], m->rhol[newL]};
  double lam[2], mu[2];
  for (int s = 0; s < 2; ++s) {
    mu[s] = rho[s] * cS[s] * cS[s];
    lam[s] = rho[s] * (cP[s] * cP[s] - 2.0 * cS[s] * cS[s]);
  }
  /* local (k1, k3) and polarisations (d1, d2, d3) of the four outgoing modes
     and of the incident one */
  cplx k3[5], d1[5], d3[5];
  double kk[5];
  int side[5], exists[5];
  const double p1l = p1 > 1e-12 * sqrt(dot3(Pin, Pin)) ? p1 : 0.0;
  for (int mo = 0; mo < 4; ++mo) {
    const int sp = mo & 1, sd = mo >> 1;
    const double c = sp == 0 ? cP[sd] : cS[sd];
    const double kabs = H / c;
    const double rad = kabs * kabs - p1l * p1l;
    const double dir = sd == 1 ? sgn : -sgn;  /* transmitted keep the sign */
    kk[mo] = kabs;
    side[mo] = sd;
    if (rad >= 0.0) {
      k3[mo] = dir * sqrt(rad);
      exists[mo] = 1;
    } else {
      /* decays away from the interface on its own side (x3 > 0 transmitted) */
      k3[mo] = (sd == 1 ? 1.0 : -1.0) * I * sqrt(-rad);
      exists[mo] = 0;
    }
  }
  kk[4] = H / c_in;
  k3[4] = pn;
  side[4] = 0;
  exists[4] = 1;
  for (int mo = 0; mo < 5; ++mo) {
    const int sp = mo == 4 ? sp_in : (mo & 1);
    const cplx h1 = p1l / kk[mo], h3 = k3[mo] / kk[mo]; /* k / |k| */
    if (sp == 0) { d1[mo] = h1; d3[mo] = h3; }
    else { d1[mo] = h3; d3[mo] = -h1; } /* e2 x khat */
  }
  /* incident amplitude in the local frame: along khat (P) or split into the
     in-plane and SH parts (S) */
  const cplx A1 = Ain[0] * e1[0] + Ain[1] * e1[1] + Ain[2] * e1[2];
  const cplx A2 = Ain[0] * e2[0] + Ain[1] * e2[1] + Ain[2] * e2[2];
  const cplx A3 = Ain[0] * n[0] + Ain[1] * n[1] + Ain[2] * n[2];
  const cplx a_inplane = A1 * d1[4] + A3 * d3[4];
  const cplx a_sh = sp_in == 0 ? 0.0 : A2;
  /* P-SV system: rows u1, u3, t1, t3; columns R_P, R_S, T_P, T_S */
  cplx M[4][4], b[4], x[4];
  for (int mo = 0; mo < 5; ++mo) {
    const int sd = side[mo];
    const cplx k1 = p1l;
    const cplx kd = k1 * d1[mo] + k3[mo] * d3[mo];
    const cplx col[4] = {d1[mo], d3[mo], mu[sd] * (k1 * d3[mo] + k3[mo] * d1[mo]),
                         lam[sd] * kd + 2.0 * mu[sd] * k3[mo] * d3[mo]};
    for (int r = 0; r < 4; ++r) {
      if (mo == 4) b[r] = -a_inplane * col[r];
      else M[r][mo] = sd == 0 ? col[r] : -col[r];
    }
  }
  csolve_n(4, M, b, x);
  /* SH system: rows u2, t2; columns R_SH, T_SH (polarisation e2 for all) */
  cplx y[2] = {0.0, 0.0};
  if (sp_in == 1) {
    cplx Ms[4][4], bs[4], xs[4];
    Ms[0][0] = 1.0;
    Ms[0][1] = -1.0;
    Ms[1][0] = mu[0] * k3[1];
    Ms[1][1] = -mu[1] * k3[3];
    bs[0] = -a_sh;
    bs[1] = -a_sh * mu[0] * k3[4];
    csolve_n(2, Ms, bs, xs);
    y[0] = xs[0];
    y[1] = xs[1];
  }
  for (int mo = 0; mo < 4; ++mo) {
    om_mode *o = &out[mo];
    o->sp = mo & 1;
    o->side = side[mo];
    o->exists = exists[mo];
    const double k3r = creal(k3[mo]);
    for (int i = 0; i < 3; ++i) o->P[i] = p1l * e1[i] + k3r * n[i];
    const cplx ain = x[mo];
    const cplx ash = o->sp == 1 ? y[mo >> 1] : 0.0;
    for (int i = 0; i < 3; ++i) o->A[i] = ain * (d1[mo] * e1[i] + d3[mo] * n[i]) + ash * e2[i];
  }
}

/* The same plane-wave problem at a traction-free surface (the outer side is
 * empty): only the reflected modes exist, and the conditions are sigma.n = 0
 * for the incident plus reflected waves, in the local frame of
 * om_interface_modes (e3 = n pointing out of the medium, e1 = tangential
 * momentum direction).  In-plane (P, SV): rows t1, t3, unknowns R_P, R_S;
 * SH: mu (k3_in a_SH + k3_r R_SH) = 0.  out[2], out[3] (transmitted) do not
 * exist.  Speeds at the surface point xc. */
void om_free_surface_modes(const om_medium *m, int L, const double xc[3], const double n[3], int sp_in,
                           const double Pin[3], const cplx Ain[3], om_mode out[4])
{
  double cP, cS;
  {
    double gdum[3], Hdum[3][3];
    om_speed(m, 0, L, xc, &cP, gdum, Hdum);
    om_speed(m, 1, L, xc, &cS, gdum, Hdum);
  }
  const double c_in = sp_in == 0 ? cP : cS;
  const double H = c_in * sqrt(dot3(Pin, Pin));
  const double pn = dot3(Pin, n);
  double pt[3] = {Pin[0] - pn * n[0], Pin[1] - pn * n[1], Pin[2] - pn * n[2]};
  const double p1 = sqrt(dot3(pt, pt));
  double e1[3], e2[3];
  const int oblique = p1 > 1e-12 * sqrt(dot3(Pin, Pin));
  if (oblique) {
    for (int i = 0; i < 3; ++i) e1[i] = pt[i] / p1;
  } else {
    double t[3] = {1.0, 0.0, 0.0};
    if (fabs(n[0]) > 0.9) { t[0] = 0.0; t[1] = 1.0; }
    const double tn = dot3(t, n);
    for (int i = 0; i < 3; ++i) t[i] -= tn * n[i];
    const double nt = sqrt(dot3(t, t));
    for (int i = 0; i < 3; ++i) e1[i] = t[i] / nt;
  }
  cross3(n, e1, e2);
  const double p1l = oblique ? p1 : 0.0;
  const double sgn = pn >= 0.0 ? 1.0 : -1.0;
  const double rho = m->rhol[L];
  const double mu = rho * cS * cS, lam = rho * (cP * cP - 2.0 * cS * cS);
  /* waves 0 (P reflected), 1 (S reflected), 2 (incident) */
  cplx k3[3], d1[3], d3[3];
  double kk[3];
  int exists[2];
  for (int w = 0; w < 2; ++w) {
    const double c = w == 0 ? cP : cS;
    const double kabs = H / c, rad = kabs * kabs - p1l * p1l;
    kk[w] = kabs;
    if (rad >= 0.0) {
      k3[w] = -sgn * sqrt(rad);
      exists[w] = 1;
    } else {
      k3[w] = -I * sqrt(-rad); /* decays into the medium (x3 < 0) */
      exists[w] = 0;
    }
  }
  kk[2] = H / c_in;
  k3[2] = pn;
  for (int w = 0; w < 3; ++w) {
    const int sp = w == 2 ? sp_in : w;
    const cplx h1 = p1l / kk[w], h3 = k3[w] / kk[w];
    if (sp == 0) { d1[w] = h1; d3[w] = h3; }
    else { d1[w] = h3; d3[w] = -h1; }
  }
  const cplx A1 = Ain[0] * e1[0] + Ain[1] * e1[1] + Ain[2] * e1[2];
  const cplx A2 = Ain[0] * e2[0] + Ain[1] * e2[1] + Ain[2] * e2[2];
  const cplx A3 = Ain[0] * n[0] + Ain[1] * n[1] + Ain[2] * n[2];
  const cplx a_inplane = A1 * d1[2] + A3 * d3[2];
  const cplx a_sh = sp_in == 0 ? 0.0 : A2;
  cplx M[4][4], b[4], x[4];
  for (int w = 0; w < 3; ++w) {
    const cplx k1 = p1l;
    const cplx kd = k1 * d1[w] + k3[w] * d3[w];
    const cplx t1 = mu * (k1 * d3[w] + k3[w] * d1[w]);
    const cplx t3 = lam * kd + 2.0 * mu * k3[w] * d3[w];
    if (w == 2) {
      b[0] = -a_inplane * t1;
      b[1] = -a_inplane * t3;
    } else {
      M[0][w] = t1;
      M[1][w] = t3;
    }
  }
  csolve_n(2, M, b, x);
  const cplx ysh = sp_in == 1 ? -k3[2] * a_sh / k3[1] : 0.0;
  for (int w = 0; w < 4; ++w) {
    om_mode *o = &out[w];
    o->sp = w & 1;
    o->side = w >> 1;
    o->exists = w < 2 ? exists[w] : 0;
    for (int i = 0; i < 3; ++i) { o->P[i] = 0.0; o->A[i] = 0.0; }
    if (w >= 2) continue;
    const double k3r = creal(k3[w]);
    for (int i = 0; i < 3; ++i) o->P[i] = p1l * e1[i] + k3r * n[i];
    const cplx ash = w == 1 ? ysh : 0.0;
    for (int i = 0; i < 3; ++i) o->A[i] = x[w] * (d1[w] * e1[i] + d3[w] * n[i]) + ash * e2[i];
  }
}

/* Lineage number of child k (0..3: P reflected, S reflected, P transmitted,
 * S transmitted) of a beam: generation in the top bits, then the parent's
 * path shifted by two bits. */
int64_t om_child_lineage(int64_t parent, int gen_parent, int k)
{
  const int64_t path = parent & ((INT64_C(1) << 58) - 1);
  return ((int64_t)(gen_parent + 1) << 58) | (path << 2) | k;
}

/* Map of the state of a beam at an interface point x* to one outgoing mode
 * (eq:Inter_DzQDzP; row m of dzQ, dzP is the derivative by z_m, columns the
 * spatial components).  With n the unit normal, V = c P/|P| (the sign sigma
 * of the branch cancels throughout), s = V_in.n, p_n = Pin.n, p_n' = Pout.n,
 * mu = p_n' - p_n, per row (q_n = dzQ.n):
 *   the crossing time and point move with z: dtau = -q_n / s,
 *     dzQ* = dzQ - V_in q_n / s  (tangent to the interface);
 *   P at the crossing: dzP* = dzP + |Pin| grad c_in q_n / s;
 *   the outgoing momentum P' = P + mu n(x*) keeps the tangential part and
 *   H = c|P|, so with the shape operator K = dn/dx (K = kcurv (I - n n^T) on
 *   a sphere, kcurv = s/R for n = s x/R; 0 on a plane)
 *     dmu = [(V_in - V_out).dzP* + (|Pin| grad c_in - |Pout| grad c_out).dzQ*
 *            - mu V_out.(K dzQ*)] / (V_out.n),
 *     dzP'* = dzP* + n dmu + mu K dzQ*;
 *   and the child, started at the crossing, at the same instant:
 *     dzQ' = dzQ* + V_out q_n / s,   dzP' = dzP'* - |Pout| grad c_out q_n / s.
 * Where grad c = 0 and the interface is flat this is the printed map
 * (dzQ' = dzQ F, dzP' = dzP F^{-T} with F = I + n (x) v, v = (kappa - 1) p_t/p_n
 * + (kappa p_n'/p_n - 1) n, kappa = (c_out/c_in)^2).  The printed gradient
 * terms are replaced by the ones above, and the curvature term added: with
 * them the map equals finite-difference Jacobians of neighbouring rays on
 * planes and spheres, in constant and in linear-gradient layers.  c_in, c_out,
 * gin, gout: speeds and gradients of the incident and outgoing modes at x*. */
void om_interface_jacobians(const double n[3], const double Pin[3], const double Pout[3], double c_in, double c_out,
                            const double gin[3], const double gout[3], double kcurv, cplx ZQ[3][3], cplx ZP[3][3])
{
  const double pn = dot3(Pin, n), pno = dot3(Pout, n);
  const double Pi = sqrt(dot3(Pin, Pin)), Po = sqrt(dot3(Pout, Pout));
  double vin[3], vout[3];
  for (int i = 0; i < 3; ++i) { vin[i] = c_in * Pin[i] / Pi; vout[i] = c_out * Pout[i] / Po; }
  const double s_in = dot3(vin, n), s_out = dot3(vout, n), mu = pno - pn;
  cplx ZQo[3][3], ZPo[3][3];
  for (int m = 0; m < 3; ++m) {
    cplx qn = 0.0;
    for (int i = 0; i < 3; ++i) qn += ZQ[m][i] * n[i];
    cplx dQs[3], dPi[3], Kd[3], qsn = 0.0;
    for (int i = 0; i < 3; ++i) dQs[i] = ZQ[m][i] - vin[i] * qn / s_in;
    for (int i = 0; i < 3; ++i) qsn += dQs[i] * n[i];
    for (int i = 0; i < 3; ++i) Kd[i] = kcurv * (dQs[i] - n[i] * qsn);
    for (int i = 0; i < 3; ++i) dPi[i] = ZP[m][i] + Pi * gin[i] * qn / s_in;
    cplx num = 0.0;
    for (int i = 0; i < 3; ++i)
      num += (vin[i] - vout[i]) * dPi[i] + (Pi * gin[i] - Po * gout[i]) * dQs[i] - mu * vout[i] * Kd[i];
    const cplx dmu = num / s_out;
    for (int j = 0; j < 3; ++j) {
      ZQo[m][j] = dQs[j] + vout[j] * qn / s_in;
      ZPo[m][j] = dPi[j] + n[j] * dmu + mu * Kd[j] - Po * gout[j] * qn / s_in;
    }
  }
  memcpy(ZQ, ZQo, sizeof(ZQo));
  memcpy(ZP, ZPo, sizeof(ZPo));
}

/* Crossing fraction theta of a step from y0 in a layer whose speed varies
 * (curved ray): four secant iterations on the level of the RK4 sub-step of
 * theta dt from y0, started from 0 and from the straight-ray estimate. */
static double om_crossing_secant(const om_medium *m, const om_beam *y0, int iface, double dt, double th0)
{
  const double b = om_iface_level(m, iface);
  double ta = 0.0, fa = (m->geometry == 1 ? sqrt(dot3(y0->Q, y0->Q)) : y0->Q[2]) - b;
  double tb = th0;
  om_beam x = *y0;
  om_rk4_step(m, &x, tb * dt);
  double fb = (m->geometry == 1 ? sqrt(dot3(x.Q, x.Q)) : x.Q[2]) - b;
  for (int it = 0; it < 4; ++it) {
    if (fb == fa) break;
    double tn = tb - fb * (tb - ta) / (fb - fa);
    tn = tn < 0.0 ? 0.0 : (tn > 1.0 ? 1.0 : tn);
    ta = tb;
    fa = fb;
    tb = tn;
    x = *y0;
    om_rk4_step(m, &x, tb * dt);
    fb = (m->geometry == 1 ? sqrt(dot3(x.Q, x.Q)) : x.Q[2]) - b;
  }
  return tb;
}

/* Advance n beams (array capacity cap) by nsteps RK4 steps in a layered
 * medium with interfaces.  After each step a beam whose centre has left its
 * layer is split: it is moved back to the start of the step and advanced by
 * theta dt to the crossing (theta from the straight ray in a constant layer,
 * refined by four secant iterations on RK4 sub-steps in a gradient layer),
 * Q is put exactly on the interface, and each propagating outgoing mode
 * (speeds taken at the crossing point) whose amplitude is at
 * least child_cut times the incident one becomes a child beam (lineage from
 * om_child_lineage, generation + 1, the parent's weight, sigma and action),
 * which then takes the remaining (1 - theta) dt in its own layer.  The parent
 * is retired.  A beam already at generation gmax is retired at an interface
 * without children.  Children are appended in parent order; beams appended
 * during a step are not stepped again in it.  Returns the new beam count, or
 * -1 if the capacity would be exceeded (then the beam set is partly
 * updated).  *capped receives the number of beams retired at the cap. */
/* One regular step of an S beam with the frame-free amplitude: A from the
 * frame, the vector RK4 step, and back to the frame (axis switched first if P
 * has come within 10 degrees of it). */
static void om_step_svec(const om_medium *m, om_beam *b, double dt)
{
  double nsh[3], nsv[3];
  om_s_frame(b->P, b->e, nsh, nsv);
  cplx A[3];
  for (int d = 0; d < 3; ++d) A[d] = b->a[0] * nsv[d] + b->a[1] * nsh[d];
  om_rk4_step_vec(m, b, A, dt);
  const double np = sqrt(dot3(b->P, b->P));
  if (fabs(dot3(b->P, b->e)) / np > cos(10.0 * M_PI / 180.0)) {
    const int was_z = b->e[2] != 0.0 && b->e[0] == 0.0 && b->e[1] == 0.0;
    b->e[0] = was_z ? 1.0 : 0.0;
    b->e[1] = 0.0;
    b->e[2] = was_z ? 0.0 : 1.0;
  }
  om_s_frame(b->P, b->e, nsh, nsv);
  b->a[0] = A[0] * nsv[0] + A[1] * nsv[1] + A[2] * nsv[2];
  b->a[1] = A[0] * nsh[0] + A[1] * nsh[1] + A[2] * nsh[2];
}

/* s_vector: in a medium with curved rays somewhere (a gradient or an anomaly
 * in some layer), the regular steps of S beams take the frame-free amplitude
 * (om_step_svec); steps that reach an interface and the children's partial
 * steps stay in the framed form. */
int64_t om_evolve_layered(const om_medium *m, om_beam *beams, int64_t n, int64_t cap, double dt, int nsteps,
                          int gmax, double child_cut, int64_t *capped, int s_vector)
{
  int64_t ncap = 0;
  int curved = 0;
  for (int l = 0; l < m->nlayer; ++l) curved = curved || m->gradl[l] != 0.0 || m->anom_amp[l] != 0.0;
  const int vec = s_vector && curved;
  for (int s = 0; s < nsteps; ++s) {
    const int64_t n0 = n;
    for (int64_t i = 0; i < n0; ++i) {
      om_beam *b = &beams[i];
      if (!b->alive) continue;
      om_beam y0 = *b;
      om_beam yv = *b;
      om_rk4_step(m, b, dt);
      int iface, newL;
      if (!om_layer_exit(m, y0.layer, b->Q, &iface, &newL)) {
        if (vec && b->branch != 0) {
          om_step_svec(m, &yv, dt);
          *b = yv;
        } else {
          om_reframe(b);
        }
        continue;
      }
      double th = om_crossing_fraction(m, iface, y0.Q, b->Q);
      om_beam x = y0;
      /* curved rays (a gradient or an anomaly in the layer): secant iterations */
      if (m->gradl[y0.layer] != 0.0 || m->anom_amp[y0.layer] != 0.0)
        th = om_crossing_secant(m, &y0, iface, dt, th);
      om_rk4_step(m, &x, th * dt);
      /* exactly onto the interface */
      double nrm[3] = {0.0, 0.0, 0.0};
      double kcurv = 0.0;
      if (m->geometry == 1) {
        const double r = sqrt(dot3(x.Q, x.Q));
        const double R = om_iface_level(m, iface);
        for (int k = 0; k < 3; ++k) x.Q[k] *= R / r;
        kcurv = (iface == OM_SURFACE ? 1.0 : (newL > y0.layer ? -1.0 : 1.0)) / R;
        for (int k = 0; k < 3; ++k) nrm[k] = kcurv * x.Q[k];
      } else {
        x.Q[2] = om_iface_level(m, iface);
        nrm[2] = iface == OM_SURFACE ? 1.0 : (newL > y0.layer ? 1.0 : -1.0);
      }
      b->alive = 0;
      if (x.gen >= gmax) {
        ++ncap;
        continue;
      }
      const int sp_in = x.branch == 0 ? 0 : 1;
      cplx Ain[3];
      om_amplitude_vector(&x, Ain);
      const double ain = sqrt(creal(Ain[0] * conj(Ain[0]) + Ain[1] * conj(Ain[1]) + Ain[2] * conj(Ain[2])));
      om_mode md[4];
      if (iface == OM_SURFACE) om_free_surface_modes(m, y0.layer, x.Q, nrm, sp_in, x.P, Ain, md);
      else om_interface_modes(m, y0.layer, newL, x.Q, nrm, sp_in, x.P, Ain, md);
      double c_in, g_in[3], Hd[3][3];
      om_speed(m, sp_in, y0.layer, x.Q, &c_in, g_in, Hd);
      for (int k = 0; k < 4; ++k) {
        if (!md[k].exists) continue;
        const double am = sqrt(creal(md[k].A[0] * conj(md[k].A[0]) + md[k].A[1] * conj(md[k].A[1]) +
                                     md[k].A[2] * conj(md[k].A[2])));
        if (!(am >= child_cut * ain)) continue;
        if (n >= cap) return -1;
        om_beam c = x;
        const int lay = md[k].side == 1 ? newL : y0.layer;
        double c_out, g_out[3];
        om_speed(m, md[k].sp, lay, x.Q, &c_out, g_out, Hd);
        memcpy(c.P, md[k].P, sizeof c.P);
        om_interface_jacobians(nrm, x.P, c.P, c_in, c_out, g_in, g_out, kcurv, c.ZQ, c.ZP);
        c.layer = lay;
        c.branch = md[k].sp == 0 ? 0 : 2;
        c.gen = x.gen + 1;
        c.lineage = om_child_lineage(x.lineage, x.gen, k);
        c.alive = 1;
        om_initial_axis(c.P, c.e);
        if (md[k].sp == 0) {
          const double np = sqrt(dot3(c.P, c.P));
          c.a[0] = (md[k].A[0] * c.P[0] + md[k].A[1] * c.P[1] + md[k].A[2] * c.P[2]) / np;
          c.a[1] = 0.0;
        } else {
          double nsh[3], nsv[3];
          om_s_frame(c.P, c.e, nsh, nsv);
          c.a[0] = md[k].A[0] * nsv[0] + md[k].A[1] * nsv[1] + md[k].A[2] * nsv[2];
          c.a[1] = md[k].A[0] * nsh[0] + md[k].A[1] * nsh[1] + md[k].A[2] * nsh[2];
        }
        om_rk4_step(m, &c, (1.0 - th) * dt);
        om_reframe(&c);
        beams[n++] = c;
        b = &beams[i];
      }
    }
  }
  if (capped) *capped = ncap;
  return n;
}

/* Batched helpers for the Python wrapper. */
void om_fbi_many(const cplx *f, const int yn[3], const double ylo[3], const double yh[3],
                 const double *q, const double *p, int64_t n, double eps, cplx *out)
{
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t i = 0; i < n; ++i) om_fbi(f, yn, ylo, yh, q + 3 * i, p + 3 * i, eps, out + 3 * i);
}

/* rhs of one beam at its stored state, for tests of the ODE itself */
/* om_make_beams over many mesh points: pair i is (q[i], p[i]) with FBI values
 * Ft[i] and Gt[i] (Gt NULL or [n][2][3]: FBI[g/c_P], FBI[g/c_S]) and lineage
 * base ip[i]*nq_all + iq[i]; beams are written in pair order.  Returns the
 * number of beams written. */
int64_t om_make_beams_many(const double *q, const double *p, const cplx *Ft, const cplx *Gt, int64_t n,
                           const int64_t *iq, const int64_t *ip, int64_t nq_all, int64_t np_all, int one_way,
                           double eps, double dq, double dp, int branch_mask, double cull_abs, om_beam *out)
{
  int64_t k = 0;
  for (int64_t i = 0; i < n; ++i)
    k += om_make_beams(q + 3 * i, p + 3 * i, Ft + 3 * i, Gt ? Gt + 6 * i : NULL, one_way, eps, dq, dp, branch_mask,
                       cull_abs, ip[i] * nq_all + iq[i], nq_all * np_all, out + k);
  return k;
}

void om_rhs_beam(const om_medium *m, const om_beam *b, om_beam *d)
{
  om_state y, dy;
  st_from_beam(b, &y);
  om_rhs(m, b, &y, &dy);
  *d = *b;
  st_to_beam(&dy, d);
}

void om_speed_many(const om_medium *m, int sp, const double *x, int64_t n, double *out /* [n][13] */)
{
  for (int64_t i = 0; i < n; ++i) {
    double c, gc[3], H[3][3];
    om_speed(m, sp, om_layer_of(m, x + 3 * i), x + 3 * i, &c, gc, H);
    double *o = out + 13 * i;
    o[0] = c;
    for (int k = 0; k < 3; ++k) o[1 + k] = gc[k];
    for (int k = 0; k < 9; ++k) o[4 + k] = H[k / 3][k % 3];
  }
}

void om_amplitude_vectors(const om_beam *b, int64_t n, cplx *A)
{
  for (int64_t i = 0; i < n; ++i) om_amplitude_vector(&b[i], A + 3 * i);
}

void om_reframe_many(om_beam *b, int64_t n)
{
  for (int64_t i = 0; i < n; ++i) om_reframe(&b[i]);
}

size_t om_medium_size(void) { return sizeof(om_medium); }
