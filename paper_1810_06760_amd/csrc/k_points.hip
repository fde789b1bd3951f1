// Step 3 at scattered points (eq:FGA): receivers and seismograms.
//
// Layout.  Points are pre-sorted along a Morton curve and split into groups
// of 16; a wavefront owns one group, its lanes being (point ri = lane % 16,
// beam slot bs = lane / 16).  The workgroup (4 groups, 64 points) walks a
// range of beams in tiles of 64 emission records (Q, P/eps, B = w e^{iS/eps} A)
// staged in LDS; lane (ri, bs) evaluates beams bs, bs + 4, ... of each tile
// against its point.  Beams of a tile are spatially close and so are the 16
// points of a group, so the window test is nearly uniform across a
// wavefront, and a tile whose bounding box is farther than the window from
// the group's box is skipped as a whole.  Each point's sum is reduced over
// its four beam slots with lane shuffles and written once per workgroup and
// sample; workgroup partials are reduced afterwards in a fixed order, so the
// sums are bitwise reproducible and need no atomics.
#include "device_common.h"
#include "fastmath.h"

namespace fga {
namespace {

constexpr int TILE = 64;   // beam records per LDS stage
constexpr int GROUP = 16;  // points per wavefront

__global__ __launch_bounds__(256) void k_sum_points(PointsArgs a)
{
  __shared__ double rec[12][TILE];
  __shared__ double tbox[6];
  __shared__ TrigTables tab;
  fill_tables(tab);

  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ri = lane & (GROUP - 1), bs = lane / GROUP;
  const int64_t r = (int64_t)blockIdx.y * 64 + w * GROUP + ri;
  const bool rv = r < a.n;
  double x0 = 1.0e300, x1 = 1.0e300, x2 = 1.0e300;
  if (rv) {
    x0 = a.xyz[3 * r];
    x1 = a.xyz[3 * r + 1];
    x2 = a.xyz[3 * r + 2];
  }
  // bounding box of the group's points (lanes of a wavefront share the group)
  double gb[6] = {rv ? x0 : 1e300, rv ? x1 : 1e300, rv ? x2 : 1e300,
                  rv ? x0 : -1e300, rv ? x1 : -1e300, rv ? x2 : -1e300};
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      gb[d] = fmin(gb[d], __shfl_xor(gb[d], off));
      gb[3 + d] = fmax(gb[3 + d], __shfl_xor(gb[3 + d], off));
    }
  }
  const double R = sqrt(2.0 * a.tau * a.eps);
  const double hieps = 0.5 / a.eps;
  const int64_t b0 = (int64_t)blockIdx.x * a.beams_per_block;
  const int64_t b1 = b0 + a.beams_per_block < a.nb ? b0 + a.beams_per_block : a.nb;
  unsigned long long cnt = 0;
  __syncthreads();  // tables
  for (int s = 0; s < a.m; ++s) {
    const double *E = a.emit + (int64_t)s * 12 * a.nb;
    double u[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t t0 = b0; t0 < b1; t0 += TILE) {
      for (int k = threadIdx.x; k < 12 * TILE; k += 256) {
        const int f = k / TILE, jj = k % TILE;
        // padding beams sit at -1e300, points of idle lanes at +1e300: never in window
        rec[f][jj] = t0 + jj < b1 ? E[f * a.nb + t0 + jj] : (f < 3 ? -1.0e300 : 0.0);
      }
      if (w == 0) {
        // tile bounding box of the beam centres
        const bool bv = t0 + lane < b1;
        double q[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) q[d] = bv ? E[d * a.nb + t0 + lane] : 0.0;
        double tb[6] = {bv ? q[0] : 1e300, bv ? q[1] : 1e300, bv ? q[2] : 1e300,
                        bv ? q[0] : -1e300, bv ? q[1] : -1e300, bv ? q[2] : -1e300};
        for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            tb[d] = fmin(tb[d], __shfl_xor(tb[d], off));
            tb[3 + d] = fmax(tb[3 + d], __shfl_xor(tb[3 + d], off));
          }
        }
        if (lane < 6) tbox[lane] = tb[lane];
      }
      __syncthreads();
      const bool near = tbox[0] - R <= gb[3] && gb[0] <= tbox[3] + R && tbox[1] - R <= gb[4] &&
                        gb[1] <= tbox[4] + R && tbox[2] - R <= gb[5] && gb[2] <= tbox[5] + R;
      if (near) {
#pragma unroll 2
        for (int jb = bs; jb < TILE; jb += 64 / GROUP) {
          const double d0 = x0 - rec[0][jb], d1 = x1 - rec[1][jb], d2 = x2 - rec[2][jb];
          if (fmax(fabs(d0), fmax(fabs(d1), fabs(d2))) > R) continue;
          ++cnt;
          const double g = (d0 * d0 + d1 * d1 + d2 * d2) * hieps;
          const double ph = rec[3][jb] * d0 + rec[4][jb] * d1 + rec[5][jb] * d2;
          double er, ei;
          cexp_neg(tab, g, ph, er, ei);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const double br = rec[6 + 2 * c][jb], bi = rec[7 + 2 * c][jb];
            u[2 * c] = fma(er, br, fma(-ei, bi, u[2 * c]));
            u[2 * c + 1] = fma(er, bi, fma(ei, br, u[2 * c + 1]));
          }
        }
      }
      __syncthreads();
    }
    // sum the four beam slots of each point (fixed order: slot 0+1, 2+3, then both)
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      u[c] += __shfl_xor(u[c], 16);
      u[c] += __shfl_xor(u[c], 32);
    }
    if (rv && bs == 0) {
      double *o = a.partial + (((int64_t)blockIdx.x * a.m + s) * a.n + r) * 6;
#pragma unroll
      for (int c = 0; c < 6; ++c) o[c] = u[c];
    }
  }
  if (a.evals) {
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_down(cnt, off);
    if (lane == 0 && cnt) atomicAdd(a.evals, cnt);
  }
}

// out[perm[r]][s0 + s][c] (+)= sum over blocks of partial[blk][s][r][c], blocks in order.
__global__ __launch_bounds__(256) void k_reduce_points(const double *__restrict__ partial, int nblk, int m, int64_t n,
                                                       const int32_t *__restrict__ perm, double *__restrict__ out,
                                                       int64_t out_samples, int s0, int accumulate)
{
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;  // (s, r, c6)
  const int64_t total = (int64_t)m * n * 6;
  if (id >= total) return;
  const int c6 = (int)(id % 6);
  const int64_t r = (id / 6) % n;
  const int s = (int)(id / (6 * n));
  double v = 0.0;
  for (int b = 0; b < nblk; ++b) v += partial[(((int64_t)b * m + s) * n + r) * 6 + c6];
  const int64_t ro = perm ? perm[r] : r;
  double *o = out + (ro * out_samples + s0 + s) * 6 + c6;
  *o = accumulate ? *o + v : v;
}

}  // namespace

hipError_t launch_sum_points(const PointsArgs &a, int *nblk_out, hipStream_t st)
{
  const int64_t nblk = (a.nb + a.beams_per_block - 1) / a.beams_per_block;
  *nblk_out = (int)nblk;
  if (a.nb == 0 || a.n == 0 || a.m == 0) return hipSuccess;
  dim3 grid((unsigned)nblk, (unsigned)((a.n + 63) / 64));
  ProfScope prof(FGA_K_SUM_POINTS, st);
  hipLaunchKernelGGL(k_sum_points, grid, 256, 0, st, a);
  return hipGetLastError();
}

hipError_t launch_reduce_points(const double *partial, int nblk, int m, int64_t n, const int32_t *perm, double *out,
                                int64_t out_samples, int s0, int accumulate, hipStream_t st)
{
  const int64_t total = (int64_t)m * n * 6;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_points, (unsigned)((total + 255) / 256), 256, 0, st, partial, nblk, m, n, perm, out,
                     out_samples, s0, accumulate);
  return hipGetLastError();
}

}  // namespace fga
