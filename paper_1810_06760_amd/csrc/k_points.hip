// Step 3 at scattered points (eq:FGA): receivers and seismograms.
//
// Work is organised receiver-major: each thread owns one receiver and keeps
// its three complex sums in registers, while the workgroup walks a range of
// beams whose emission records (Q, P, B = w e^{iS/eps} A) are staged through
// LDS and read as broadcasts.  No two threads ever add into the same output,
// so the sums need no atomics; per-workgroup partials are reduced afterwards
// in a fixed order, which keeps the result bitwise reproducible.
#include "device_common.h"

namespace fga {
namespace {

constexpr int TILE = 64;  // beam records per LDS stage

__global__ __launch_bounds__(256) void k_sum_points(PointsArgs a)
{
  __shared__ double rec[12][TILE];
  const int64_t r = (int64_t)blockIdx.y * 256 + threadIdx.x;
  const bool rv = r < a.n;
  double x0 = 0.0, x1 = 0.0, x2 = 0.0;
  if (rv) {
    x0 = a.xyz[3 * r];
    x1 = a.xyz[3 * r + 1];
    x2 = a.xyz[3 * r + 2];
  }
  const double R = sqrt(2.0 * a.tau * a.eps);
  const double ieps = 1.0 / a.eps, hieps = 0.5 / a.eps;
  const int64_t b0 = (int64_t)blockIdx.x * a.beams_per_block;
  const int64_t b1 = b0 + a.beams_per_block < a.nb ? b0 + a.beams_per_block : a.nb;
  unsigned long long cnt = 0;
  for (int s = 0; s < a.m; ++s) {
    const double *E = a.emit + (int64_t)s * 12 * a.nb;
    double u[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t t0 = b0; t0 < b1; t0 += TILE) {
      for (int k = threadIdx.x; k < 12 * TILE; k += 256) {
        const int f = k / TILE, jj = k % TILE;
        rec[f][jj] = t0 + jj < b1 ? E[f * a.nb + t0 + jj] : (f < 3 ? 1.0e300 : 0.0);
      }
      __syncthreads();
      if (rv) {
        for (int jj = 0; jj < TILE; ++jj) {
          const double d0 = x0 - rec[0][jj], d1 = x1 - rec[1][jj], d2 = x2 - rec[2][jj];
          if (fabs(d0) > R || fabs(d1) > R || fabs(d2) > R) continue;
          ++cnt;
          const double ph = (rec[3][jj] * d0 + rec[4][jj] * d1 + rec[5][jj] * d2) * ieps;
          const double gm = exp(-(d0 * d0 + d1 * d1 + d2 * d2) * hieps);
          double sn, cs;
          sincos(ph, &sn, &cs);
          const double er = gm * cs, ei = gm * sn;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const double br = rec[6 + 2 * c][jj], bi = rec[7 + 2 * c][jj];
            u[2 * c] += er * br - ei * bi;
            u[2 * c + 1] += er * bi + ei * br;
          }
        }
      }
      __syncthreads();
    }
    if (rv) {
      double *o = a.partial + (((int64_t)blockIdx.x * a.m + s) * a.n + r) * 6;
#pragma unroll
      for (int c = 0; c < 6; ++c) o[c] = u[c];
    }
  }
  if (a.evals) {
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_down(cnt, off);
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(a.evals, cnt);
  }
}

// out[r][s0 + s][c] (+)= sum over blocks of partial[blk][s][r][c], blocks in order.
__global__ __launch_bounds__(256) void k_reduce_points(const double *__restrict__ partial, int nblk, int m, int64_t n,
                                                       double *__restrict__ out, int64_t out_samples, int s0,
                                                       int accumulate)
{
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;  // (s, r, c6)
  const int64_t total = (int64_t)m * n * 6;
  if (id >= total) return;
  const int c6 = (int)(id % 6);
  const int64_t r = (id / 6) % n;
  const int s = (int)(id / (6 * n));
  double v = 0.0;
  for (int b = 0; b < nblk; ++b) v += partial[(((int64_t)b * m + s) * n + r) * 6 + c6];
  double *o = out + (r * out_samples + s0 + s) * 6 + c6;
  *o = accumulate ? *o + v : v;
}

}  // namespace

hipError_t launch_sum_points(const PointsArgs &a, int *nblk_out, hipStream_t st)
{
  const int64_t nblk = (a.nb + a.beams_per_block - 1) / a.beams_per_block;
  *nblk_out = (int)nblk;
  if (a.nb == 0 || a.n == 0 || a.m == 0) return hipSuccess;
  dim3 grid((unsigned)nblk, (unsigned)((a.n + 255) / 256));
  ProfScope prof(FGA_K_SUM_POINTS, st);
  hipLaunchKernelGGL(k_sum_points, grid, 256, 0, st, a);
  return hipGetLastError();
}

hipError_t launch_reduce_points(const double *partial, int nblk, int m, int64_t n, double *out, int64_t out_samples,
                                int s0, int accumulate, hipStream_t st)
{
  const int64_t total = (int64_t)m * n * 6;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_points, (unsigned)((total + 255) / 256), 256, 0, st, partial, nblk, m, n, out,
                     out_samples, s0, accumulate);
  return hipGetLastError();
}

}  // namespace fga
