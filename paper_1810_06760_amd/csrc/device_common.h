// Device-side helpers shared by the gfx950 kernels: medium evaluation and
// polarisation frames.
#pragma once

#include "fga_internal.h"

namespace fga {

// Medium kinds a kernel is specialised for.
// MK_GRID: trilinear node records; MK_GRID3: cubic B-spline of the node values.
enum { MK_HOMOG = 0, MK_GRID = 1, MK_LAYERED = 2, MK_GRID3 = 3 };

// Layered media: if Q lies outside layer L, the interface crossed and the
// layer beyond it (points on an interface count as inside).  Flat: interface
// i is z = bound[i] between layer i (below) and i+1; spherical: |x| = bound[i]
// between layer i (outside) and i+1 (inside).  The free surface, if any, is
// interface IFACE_SURFACE with the beam's own layer beyond it.
constexpr int IFACE_SURFACE = -1;
__device__ __forceinline__ bool layer_exit(const DevMedium &m, int L, const double Q[3], int &iface, int &newL)
{
  const int nl = m.nlayer;
  if (m.geometry == 1) {
    const double r = sqrt(Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2]);
    if (L < nl - 1 && r < m.bound[L]) { iface = L; newL = L + 1; return true; }
    if (L > 0 && r > m.bound[L - 1]) { iface = L - 1; newL = L - 1; return true; }
    if (L == 0 && m.surface > 0.0 && r > m.surface) { iface = IFACE_SURFACE; newL = 0; return true; }
  } else {
    if (L < nl - 1 && Q[2] > m.bound[L]) { iface = L; newL = L + 1; return true; }
    if (L > 0 && Q[2] < m.bound[L - 1]) { iface = L - 1; newL = L - 1; return true; }
    if (L == nl - 1 && m.surface > 0.0 && Q[2] > m.surface) { iface = IFACE_SURFACE; newL = L; return true; }
  }
  return false;
}

// Level (z or radius) of interface iface, or of the free surface.
__device__ __forceinline__ double iface_level(const DevMedium &m, int iface)
{
  return iface == IFACE_SURFACE ? m.surface : m.bound[iface];
}

// Speed of wave type sp (0 = P, 1 = S) at x: c, gradient g and Hessian H
// (xx, yy, zz, xy, xz, yz).  Grid media interpolate the ten precomputed node
// fields trilinearly (periodic); each node is one 128-byte record.
// A block of MEDBLK^3 grid nodes held in LDS by a workgroup: the ten fields
// of node (o + l) (periodic) at lds[10 (l_z MEDBLK^2 + l_y MEDBLK + l_x)].
constexpr int MEDBLK = 12;
// Cubic media: a block of MEDBLK3^3 spline coefficients per node field, the
// c_S field (two_fields) MEDBLK3^3 doubles after the c_P field.
constexpr int MEDBLK3 = 16;
struct MedBlock {
  const double *lds;  // NULL: no block
  int o[3];
};

// Cubic B-spline weights of the nodes i-1 .. i+2 at the fraction t of cell i,
// and their first and second derivatives in x (ih = 1/h).
__device__ __forceinline__ void bspline_weights(double t, double ih, double w[4], double d1[4], double d2[4])
{
  const double s = 1.0 - t, t2 = t * t, t3 = t2 * t, i6 = 1.0 / 6.0, ih2 = ih * ih;
  w[0] = s * s * s * i6;
  w[1] = (3.0 * t3 - 6.0 * t2 + 4.0) * i6;
  w[2] = (-3.0 * t3 + 3.0 * t2 + 3.0 * t + 1.0) * i6;
  w[3] = t3 * i6;
  d1[0] = -0.5 * s * s * ih;
  d1[1] = (1.5 * t2 - 2.0 * t) * ih;
  d1[2] = (-1.5 * t2 + t + 0.5) * ih;
  d1[3] = 0.5 * t2 * ih;
  d2[0] = s * ih2;
  d2[1] = (3.0 * t - 2.0) * ih2;
  d2[2] = (1.0 - 3.0 * t) * ih2;
  d2[3] = t * ih2;
}

// Tensor-product sum of the 4x4x4 coefficients ld(a, b, c) (x, y, z offsets)
// giving c, grad c and the Hessian (xx, yy, zz, xy, xz, yz) in v[10]: the x
// sums first (value, first, second derivative per row), then y, then z.
template <class Load>
__device__ __forceinline__ void bspline_sum(const double w[3][4], const double d1[3][4], const double d2[3][4],
                                            Load ld, double v[10])
{
#pragma unroll
  for (int k = 0; k < 10; ++k) v[k] = 0.0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double y00 = 0.0, y10 = 0.0, y01 = 0.0, y20 = 0.0, y11 = 0.0, y02 = 0.0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      double x0 = 0.0, x1 = 0.0, x2 = 0.0;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const double q = ld(a, b, c);
        x0 += w[0][a] * q;
        x1 += d1[0][a] * q;
        x2 += d2[0][a] * q;
      }
      y00 += w[1][b] * x0;
      y10 += w[1][b] * x1;
      y20 += w[1][b] * x2;
      y01 += d1[1][b] * x0;
      y11 += d1[1][b] * x1;
      y02 += d2[1][b] * x0;
    }
    v[0] += w[2][c] * y00;
    v[1] += w[2][c] * y10;
    v[2] += w[2][c] * y01;
    v[3] += d1[2][c] * y00;
    v[4] += w[2][c] * y20;
    v[5] += w[2][c] * y02;
    v[6] += d2[2][c] * y00;
    v[7] += w[2][c] * y11;
    v[8] += d1[2][c] * y10;
    v[9] += d1[2][c] * y01;
  }
}

template <int MK>
__device__ __forceinline__ void medium_eval(const DevMedium &m, int sp, int layer, const double *x,
                                            double &c, double g[3], double H[6], const MedBlock *blk = nullptr)
{
  if constexpr (MK == MK_HOMOG) {
    c = sp == 0 ? m.cp : m.cs;
    g[0] = g[1] = g[2] = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) H[i] = 0.0;
  } else if constexpr (MK == MK_LAYERED) {
    const double c0 = sp == 0 ? m.cpl[layer] : m.csl[layer];
    const double gm = m.gradl[layer];
    g[0] = g[1] = g[2] = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) H[i] = 0.0;
    c = c0;
    if (gm != 0.0) {
      if (m.geometry == 1) {
        // c = c0 (1 + gm r): grad c = c0 gm x/r, Hess c = c0 gm (I - x x^T/r^2)/r
        const double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        const double k = c0 * gm / r;
        c = c0 * (1.0 + gm * r);
#pragma unroll
        for (int d = 0; d < 3; ++d) g[d] = k * x[d];
        const double ir2 = 1.0 / (r * r);
        H[0] = k * (1.0 - x[0] * x[0] * ir2);
        H[1] = k * (1.0 - x[1] * x[1] * ir2);
        H[2] = k * (1.0 - x[2] * x[2] * ir2);
        H[3] = -k * x[0] * x[1] * ir2;
        H[4] = -k * x[0] * x[2] * ir2;
        H[5] = -k * x[1] * x[2] * ir2;
      } else {
        c = c0 * (1.0 + gm * x[2]);
        g[2] = c0 * gm;
      }
    }
    const double al = m.anom_amp[layer];
    if (al != 0.0) {
      // times f = 1 - al E, E = exp(-beta q), q = sum_d w_d d_d^2: grad f = 2 al beta E w d,
      // Hess f = al E (2 beta diag(w) - 4 beta^2 (w d)(w d)^T); the product rule for c f
      const double be = m.anom_beta[layer];
      double wd[3], q = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double dd = x[d] - m.anom_x[layer][d];
        wd[d] = m.anom_w[layer][d] * dd;
        q += wd[d] * dd;
      }
      const double E = exp(-be * q);
      const double f = 1.0 - al * E;
      const double k1 = 2.0 * al * be * E, k2 = 4.0 * al * be * be * E;
      const double gf[3] = {k1 * wd[0], k1 * wd[1], k1 * wd[2]};
      const int ii[6] = {0, 1, 2, 0, 0, 1}, jj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        const int i = ii[t], j = jj[t];
        const double hf = (i == j ? al * E * 2.0 * be * m.anom_w[layer][i] : 0.0) - k2 * wd[i] * wd[j];
        H[t] = f * H[t] + g[i] * gf[j] + gf[i] * g[j] + c * hf;
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) g[d] = f * g[d] + c * gf[d];
      c *= f;
    }
  } else if constexpr (MK == MK_GRID3) {
    const double *cf = m.coef;
    double scale = 1.0;
    if (sp) {
      if (m.two_fields) cf += m.coef_stride;
      else scale = m.cs_ratio;
    }
    int i0[3];
    double w[3][4], d1[3][4], d2[3][4];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double u = (x[d] - m.lo[d]) * m.ih[d];
      const double fl = floor(u);
      int ii = (int)fl;
      if (ii < 0 || ii >= m.n[d]) ii = ((ii % m.n[d]) + m.n[d]) % m.n[d];  // periodic (rare)
      i0[d] = ii;
      bspline_weights(u - fl, m.ih[d], w[d], d1[d], d2[d]);
    }
    // the 4x4x4 stencil from the LDS block when it lies in it for every lane
    bool inblk = blk != nullptr && blk->lds != nullptr;
    int l[3] = {0, 0, 0};
    if (inblk) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        int li = i0[d] - 1 - blk->o[d];
        if (li < 0) li += m.n[d];
        l[d] = li;
        inblk = inblk && li <= MEDBLK3 - 4;
      }
    }
    double v[10];
    if (__all(inblk)) {
      const double *b0 = blk->lds + ((sp && m.two_fields) ? MEDBLK3 * MEDBLK3 * MEDBLK3 : 0) +
                         (l[2] * MEDBLK3 + l[1]) * MEDBLK3 + l[0];
      bspline_sum(w, d1, d2, [&](int ia, int ib, int ic) { return b0[(ic * MEDBLK3 + ib) * MEDBLK3 + ia]; }, v);
    } else {
      int ix[4], iy[4], iz[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        ix[k] = i0[0] - 1 + k;
        iy[k] = i0[1] - 1 + k;
        iz[k] = i0[2] - 1 + k;
        ix[k] += ix[k] < 0 ? m.n[0] : (ix[k] >= m.n[0] ? -m.n[0] : 0);
        iy[k] += iy[k] < 0 ? m.n[1] : (iy[k] >= m.n[1] ? -m.n[1] : 0);
        iz[k] += iz[k] < 0 ? m.n[2] : (iz[k] >= m.n[2] ? -m.n[2] : 0);
      }
      bspline_sum(w, d1, d2,
                  [&](int ia, int ib, int ic) { return cf[((size_t)iz[ic] * m.n[1] + iy[ib]) * m.n[0] + ix[ia]]; }, v);
    }
    c = scale * v[0];
#pragma unroll
    for (int k = 0; k < 3; ++k) g[k] = scale * v[1 + k];
#pragma unroll
    for (int k = 0; k < 6; ++k) H[k] = scale * v[4 + k];
  } else {
    const double *tab = m.table;
    double scale = 1.0;
    if (sp) {
      if (m.two_fields) tab += m.field_stride;
      else scale = m.cs_ratio;
    }
    int i0[3], i1[3];
    double t[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double u = (x[d] - m.lo[d]) * m.ih[d];
      double fl = floor(u);
      t[d] = u - fl;
      int ii = (int)fl;
      if (ii < 0 || ii >= m.n[d]) ii = ((ii % m.n[d]) + m.n[d]) % m.n[d];  // periodic (rare)
      i0[d] = ii;
      i1[d] = ii + 1 == m.n[d] ? 0 : ii + 1;
    }
    double v[10];
#pragma unroll
    for (int f = 0; f < 10; ++f) v[f] = 0.0;
    // the cell's eight nodes from the LDS block when they all lie in it
    bool inblk = blk != nullptr && blk->lds != nullptr;
    int l[3] = {0, 0, 0};
    if (inblk) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        int li = i0[d] - blk->o[d];
        if (li < 0) li += m.n[d];
        l[d] = li;
        inblk = inblk && li <= MEDBLK - 2;
      }
    }
    // LDS path when every lane of the wavefront has its cell in the block
    // (the common case: Morton-ordered neighbours), else global memory for all
    if (__all(inblk)) {
#pragma unroll 8
      for (int corner = 0; corner < 8; ++corner) {
        const int lx = l[0] + (corner & 1), ly = l[1] + ((corner >> 1) & 1), lz = l[2] + ((corner >> 2) & 1);
        const double w = ((corner & 1) ? t[0] : 1.0 - t[0]) * ((corner & 2) ? t[1] : 1.0 - t[1]) *
                         ((corner & 4) ? t[2] : 1.0 - t[2]);
        const double2 *p = reinterpret_cast<const double2 *>(blk->lds + 10 * ((lz * MEDBLK + ly) * MEDBLK + lx));
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          const double2 a = p[k];
          v[2 * k] += w * a.x;
          v[2 * k + 1] += w * a.y;
        }
      }
    } else {
#pragma unroll 2
      for (int corner = 0; corner < 8; ++corner) {
        const int ix = (corner & 1) ? i1[0] : i0[0];
        const int iy = (corner & 2) ? i1[1] : i0[1];
        const int iz = (corner & 4) ? i1[2] : i0[2];
        const double w = ((corner & 1) ? t[0] : 1.0 - t[0]) * ((corner & 2) ? t[1] : 1.0 - t[1]) *
                         ((corner & 4) ? t[2] : 1.0 - t[2]);
        const double2 *p = reinterpret_cast<const double2 *>(
            tab + (size_t)FGA_GRID_NODE_DOUBLES * (((size_t)iz * m.n[1] + iy) * m.n[0] + ix));
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          const double2 a = p[k];
          v[2 * k] += w * a.x;
          v[2 * k + 1] += w * a.y;
        }
      }
    }
    c = scale * v[0];
#pragma unroll
    for (int k = 0; k < 3; ++k) g[k] = scale * v[1 + k];
#pragma unroll
    for (int k = 0; k < 6; ++k) H[k] = scale * v[4 + k];
  }
}

// SH/SV frame: N_SH = (e x P)/|e x P|, N_SV = (P/|P|) x N_SH.
__device__ __forceinline__ void s_frame(const double P[3], const double e[3], double nsh[3], double nsv[3])
{
  double x0 = e[1] * P[2] - e[2] * P[1];
  double x1 = e[2] * P[0] - e[0] * P[2];
  double x2 = e[0] * P[1] - e[1] * P[0];
  double in = 1.0 / sqrt(x0 * x0 + x1 * x1 + x2 * x2);
  nsh[0] = x0 * in; nsh[1] = x1 * in; nsh[2] = x2 * in;
  double ip = 1.0 / sqrt(P[0] * P[0] + P[1] * P[1] + P[2] * P[2]);
  double p0 = P[0] * ip, p1 = P[1] * ip, p2 = P[2] * ip;
  nsv[0] = p1 * nsh[2] - p2 * nsh[1];
  nsv[1] = p2 * nsh[0] - p0 * nsh[2];
  nsv[2] = p0 * nsh[1] - p1 * nsh[0];
}

// Rank of this lane among the lanes of its 256-thread block with keep = true,
// and the block total.  Uses wavefront ballots; must be called by all threads.
__device__ __forceinline__ int block_rank(bool keep, int *total)
{
  __shared__ int wsum[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned long long m = __ballot(keep);
  const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  const int r = __popcll(m & lt);
  if (lane == 0) wsum[w] = __popcll(m);
  __syncthreads();
  int off = 0;
  for (int k = 0; k < w; ++k) off += wsum[k];
  *total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
  __syncthreads();
  return off + r;
}

}  // namespace fga
