// Device-side helpers shared by the gfx950 kernels: medium evaluation and
// polarisation frames.
#pragma once

#include "fga_internal.h"

namespace fga {

// Medium kinds a kernel is specialised for.
enum { MK_HOMOG = 0, MK_GRID = 1, MK_LAYERED = 2 };

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
struct MedBlock {
  const double *lds;  // NULL: no block
  int o[3];
};

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
