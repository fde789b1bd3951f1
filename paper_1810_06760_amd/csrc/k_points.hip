// Step 3 at scattered points (eq:FGA): receivers and seismograms.
//
// Beam-major layout.  A wavefront owns RW points and walks a range of beams
// 64 at a time, one beam per lane, each lane holding its beam's emission
// record (Q, P/eps, B = w e^{iS/eps} A) in registers and RW complex 3-vector
// sums.  The beam set is kept in Morton order of Q, so the 64 beams of a
// lane group are close together and the window test against one point is
// (nearly) the same on every lane: evaluation is divergence-free and a point
// whose window misses all 64 beams costs one test.  After the beam range the
// sums are reduced over the lanes in a fixed order and written once per
// wavefront and sample; per-workgroup partials are then reduced in a fixed
// order, so the sums are bitwise reproducible and need no atomics.
#include "device_common.h"
#include "fastmath.h"

namespace fga {
namespace {

constexpr int RW = 8;  // points per wavefront

__global__ __launch_bounds__(256) void k_sum_points(PointsArgs a)
{
  __shared__ TrigTables tab;
  fill_tables(tab);
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: points live in SGPRs
  // blockIdx.x: point group (fastest, so workgroups sharing a beam range run
  // together and re-read its records from L2); blockIdx.y: beam range
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + w) * RW;
  double xr[RW][3];
#pragma unroll
  for (int k = 0; k < RW; ++k)
#pragma unroll
    for (int d = 0; d < 3; ++d) xr[k][d] = r0 + k < a.n ? a.xyz[3 * (r0 + k) + d] : 1.0e300;
  const double R = sqrt(2.0 * a.tau * a.eps);
  const double hieps = 0.5 / a.eps;
  const int64_t b0 = (int64_t)blockIdx.y * a.beams_per_block;
  const int64_t b1 = b0 + a.beams_per_block < a.nb ? b0 + a.beams_per_block : a.nb;
  unsigned long long cnt = 0;
  for (int s = 0; s < a.m; ++s) {
    const double *E = a.emit + (int64_t)s * 12 * a.nb;
    double u[RW][6];
#pragma unroll
    for (int k = 0; k < RW; ++k)
#pragma unroll
      for (int c = 0; c < 6; ++c) u[k][c] = 0.0;
    // records of the lane's beam, software-pipelined one tile ahead so the
    // global loads overlap the previous tile's arithmetic
    double nq[3], npe[3], nB[6];
    auto fetch = [&](int64_t t0) {
      const int64_t j = t0 + lane;
      const bool v = j < b1;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        nq[d] = v ? E[d * a.nb + j] : -1.0e300;
        npe[d] = v ? E[(3 + d) * a.nb + j] : 0.0;
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) nB[c] = v ? E[(6 + c) * a.nb + j] : 0.0;
    };
    fetch(b0);
    for (int64_t t0 = b0; t0 < b1; t0 += 64) {
      double q[3], pe[3], B[6];
#pragma unroll
      for (int d = 0; d < 3; ++d) { q[d] = nq[d]; pe[d] = npe[d]; }
#pragma unroll
      for (int c = 0; c < 6; ++c) B[c] = nB[c];
      if (t0 + 64 < b1) fetch(t0 + 64);
      // points two at a time: two independent exponential chains per lane;
      // a pair no lane's window reaches is skipped by the whole wavefront,
      // and a lane outside one window contributes an exact zero
#pragma unroll
      for (int k = 0; k < RW; k += 2) {
        double dd[2][3];
        bool in[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
          for (int d = 0; d < 3; ++d) dd[h][d] = xr[k + h][d] - q[d];
          in[h] = !(fmax(fabs(dd[h][0]), fmax(fabs(dd[h][1]), fabs(dd[h][2]))) > R);
        }
        if (!__any(in[0] || in[1])) continue;
        double er[2], ei[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          cnt += in[h] ? 1 : 0;
          const double g = in[h] ? (dd[h][0] * dd[h][0] + dd[h][1] * dd[h][1] + dd[h][2] * dd[h][2]) * hieps : 0.0;
          const double ph = in[h] ? pe[0] * dd[h][0] + pe[1] * dd[h][1] + pe[2] * dd[h][2] : 0.0;
          cexp_neg(tab, g, ph, er[h], ei[h]);
          er[h] = in[h] ? er[h] : 0.0;
          ei[h] = in[h] ? ei[h] : 0.0;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            u[k + h][2 * c] = fma(er[h], B[2 * c], fma(-ei[h], B[2 * c + 1], u[k + h][2 * c]));
            u[k + h][2 * c + 1] = fma(er[h], B[2 * c + 1], fma(ei[h], B[2 * c], u[k + h][2 * c + 1]));
          }
      }
    }
    // lane reduction in a fixed butterfly order; every lane ends with the total
#pragma unroll
    for (int k = 0; k < RW; ++k)
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        double v = u[k][c];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        u[k][c] = v;
      }
    if (lane < RW * 6) {
      const int k = lane / 6, c = lane % 6;
      double v = 0.0;
#pragma unroll
      for (int kk = 0; kk < RW; ++kk)
#pragma unroll
        for (int cc = 0; cc < 6; ++cc)
          if (kk == k && cc == c) v = u[kk][cc];
      if (r0 + k < a.n) a.partial[(((int64_t)blockIdx.y * a.m + s) * a.n + r0 + k) * 6 + c] = v;
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
  dim3 grid((unsigned)((a.n + 4 * RW - 1) / (4 * RW)), (unsigned)nblk);
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
