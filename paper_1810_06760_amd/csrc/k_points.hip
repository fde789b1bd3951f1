// Step 3 at scattered points (eq:FGA): receivers and seismograms.
//
// Beam-major layout.  A wavefront owns RW = 4 points and walks a range of
// beams 64 at a time, one beam per lane, each lane holding its beam's
// emission record (Q, P 128/(pi eps), B = w e^{iS/eps} A) in registers and
// RW complex 3-vector sums; of the four points, only those whose window
// holds some beam of the tile are evaluated.  The beam set is kept in
// Morton order of Q, so the 64 beams of a tile are close together and the
// window test against one point is (nearly) the same on every lane; a tile
// whose bounding box lies out of reach of all the wavefront's points is
// skipped without loading its records.  A workgroup covers one sample, 8 points
// (two wavefronts) and one beam range; workgroups sharing a beam range are
// dealt to one XCD so its records are read from HBM once.  After the beam
// range the sums are reduced over the lanes in a fixed order and written
// once per wavefront; per-workgroup partials are then reduced in a fixed
// order, so the sums are bitwise reproducible and need no atomics.
#include <type_traits>

#include "device_common.h"
#include "fastmath.h"

namespace fga {
namespace {

constexpr int RW = 4;  // points per wavefront
constexpr int GRP = RW < 4 ? RW : 4;  // points evaluated together
// Two wavefronts per workgroup: a new workgroup needs a free wavefront slot
// on as many SIMDs as it has wavefronts, and the wavefronts of one finish at
// different times (their points skip different tiles), so smaller workgroups
// keep more of the four slots per SIMD busy (6 % faster than four, as fast
// as one; the sums are identical).
constexpr int WPW = 2;        // wavefronts per workgroup
constexpr int PG = WPW * RW;  // points per workgroup

// Workgroup -> (point group, beam range, sample).  Workgroups are dealt to
// the 8 XCDs round-robin by id; the point groups of one (beam range, sample)
// unit get consecutive ids on the same XCD, so that unit's records come from
// HBM once and are then served by that XCD's L2.
struct PointsWork {
  int pg;
  int64_t blk;
  int s;
  bool valid;
};
__device__ __forceinline__ PointsWork points_work(int64_t id, int groups, int64_t nblk, int m)
{
  PointsWork w;
  const int64_t xcd = id & 7, j = id >> 3;
  w.pg = (int)(j % groups);
  const int64_t unit = (j / groups) * 8 + xcd;
  w.blk = unit % nblk;
  w.s = (int)(unit / nblk);
  w.valid = w.s < m;
  return w;
}

constexpr double LOG2E = 1.4426950408889634;

// Summation modes: FP64 throughout; MIXED (FP32 exp / sin / cos, FP64
// products and sums); MIXED32 (FP32 exp / sin / cos, products and per-lane
// sums, the lane and block reductions in FP64).
enum { SUM_FP64 = 0, SUM_MIXED = 1, SUM_MIXED32 = 2 };

// One term's complex factor exp(-|d|^2/(2 eps) + i P.d/eps), zero outside
// the window (in false).  Mixed modes: the exponent and the phase (in
// revolutions, reduced to [-1/2, 1/2]) are formed in FP64, then exp2 / sin /
// cos run on the FP32 transcendental unit.  FP64: the table-driven
// exponential.  T is the accumulation type (float only for MIXED32).
template <int MODE, typename T>
__device__ __forceinline__ void point_term(const TrigTables &tab, const double (&dd)[3], const double (&pe)[3],
                                           bool in, double hieps, T &er, T &ei)
{
  const double g = (dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]) * hieps;
  const double v = pe[0] * dd[0] + pe[1] * dd[1] + pe[2] * dd[2];  // phase in units of pi/128
  if constexpr (MODE != SUM_FP64) {
    const double rev = v * (1.0 / 256.0);
    const float r = (float)(rev - rint(rev));
    const float amp = in ? __builtin_amdgcn_exp2f((float)(-g * LOG2E)) : 0.0f;
    er = (T)(amp * __builtin_amdgcn_cosf(r));
    ei = (T)(amp * __builtin_amdgcn_sinf(r));
  } else {
    cexp_neg_units(tab, g, v, in, er, ei);
  }
}

// u_c += (er + i ei) B_c, c = 0..2 (complex)
template <typename T>
__device__ __forceinline__ void accumulate_term(T (&u)[6], const T (&B)[6], T er, T ei)
{
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    u[2 * c] = fma(er, B[2 * c], fma(-ei, B[2 * c + 1], u[2 * c]));
    u[2 * c + 1] = fma(er, B[2 * c + 1], fma(ei, B[2 * c], u[2 * c + 1]));
  }
}

// MODE: SUM_FP64, SUM_MIXED or SUM_MIXED32 (the term and its sum as stated
// at point_term; MIXED32 holds the tile's records B and the sums in FP32).
template <int MODE>
__global__ __launch_bounds__(64 * WPW) __attribute__((amdgpu_waves_per_eu(4))) void k_sum_points(PointsArgs a, int groups, int64_t nblk)
{
  using Acc = typename std::conditional<MODE == SUM_MIXED32, float, double>::type;
  __shared__ TrigTables tab;
  fill_tables(tab);
  __syncthreads();

  const PointsWork wk = points_work(blockIdx.x, groups, nblk, a.m);
  if (!wk.valid) return;  // whole workgroup: padding of the last XCD round
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: points live in SGPRs
  const int64_t r0 = (int64_t)wk.pg * PG + w * RW;
  double xr[RW][3];
#pragma unroll
  for (int k = 0; k < RW; ++k)
#pragma unroll
    for (int d = 0; d < 3; ++d) xr[k][d] = r0 + k < a.n ? a.xyz[3 * (r0 + k) + d] : 1.0e30;
  const double R = sqrt(2.0 * a.tau * a.eps);
  const double hieps = 0.5 / a.eps;
  const int64_t b0 = wk.blk * a.beams_per_block;
  const int64_t b1 = b0 + a.beams_per_block < a.nb ? b0 + a.beams_per_block : a.nb;
  const int s = wk.s;
  const double *E = a.emit + (int64_t)s * 12 * a.nb;
  uint64_t cnt = 0;          // wave-uniform in-window count
  Acc u[RW][6];
#pragma unroll
  for (int k = 0; k < RW; ++k)
#pragma unroll
    for (int c = 0; c < 6; ++c) u[k][c] = (Acc)0;

  // bounding box of the wavefront's points; a beam tile whose box lies more
  // than R away from it along some axis holds no term for any of them (the
  // rounded differences are monotone, so this agrees with the per-lane test)
  double plo[3], phi[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    plo[d] = xr[0][d];
    phi[d] = xr[0][d];
#pragma unroll
    for (int k = 1; k < RW; ++k)
      if (r0 + k < a.n) {
        plo[d] = fmin(plo[d], xr[k][d]);
        phi[d] = fmax(phi[d], xr[k][d]);
      }
  }
  const double *TB = a.tile_box + (int64_t)s * a.ntiles * 6;
  // The range's tiles are tested 64 at a time, one per lane (box loads in
  // parallel), and walked through the ballot of the live ones; a tile whose
  // box lies more than R from the points' box along an axis is skipped.
  const int64_t tb0 = b0 >> 6, tb1 = (b1 + 63) >> 6;  // b0 is a multiple of 64
  int64_t mbase = -1;
  uint64_t mask = 0;
  auto next_live = [&](int64_t t0) {  // first beam of the next live tile at or after t0, else b1
    int64_t t = t0 >> 6;
    while (t < tb1) {
      const int64_t base = t & ~(int64_t)63;
      if (base != mbase) {
        const int64_t tt = base + lane;
        bool ok = false;
        if (tt >= tb0 && tt < tb1) {
          const double *tb = TB + tt * 6;  // lo[3], hi[3]
          ok = true;
#pragma unroll
          for (int d = 0; d < 3; ++d) ok = ok && !(tb[d] - phi[d] > R) && !(plo[d] - tb[3 + d] > R);
        }
        mask = __ballot(ok);
        mbase = base;
      }
      const uint64_t rest = mask >> (t - base);
      if (rest) return (t + __ffsll((long long)rest) - 1) << 6;
      t = base + 64;
    }
    return b1;
  };
  // records of the lane's beam for the current tile
  double q[3], pe[3];
  Acc B[6];
  auto fetch = [&](int64_t t0) {
    const int64_t j = t0 + lane;
    const bool v = j < b1;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      q[d] = v ? E[d * a.nb + j] : -1.0e300;
      pe[d] = v ? E[(3 + d) * a.nb + j] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) B[c] = v ? (Acc)E[(6 + c) * a.nb + j] : (Acc)0;
  };
  for (int64_t t0 = next_live(b0); t0 < b1; t0 = next_live(t0 + 64)) {
    fetch(t0);
    // points four at a time: when every one of the four windows holds some
    // lane's beam, the four terms are evaluated together (four independent
    // exponential chains per lane hide each other's latency); otherwise only
    // the points whose window holds a beam of the tile, one chain each.
    // Outside its window a term's magnitude is replaced by zero, so skipping
    // a point no lane reaches changes no sum.
#pragma unroll
    for (int k = 0; k < RW; k += GRP) {
      double dd[GRP][3];
      bool in[GRP];
      unsigned need = 0;  // wave-uniform: points with at least one lane in window
#pragma unroll
      for (int h = 0; h < GRP; ++h) {
#pragma unroll
        for (int d = 0; d < 3; ++d) dd[h][d] = xr[k + h][d] - q[d];
        in[h] = fmax(fabs(dd[h][0]), fmax(fabs(dd[h][1]), fabs(dd[h][2]))) <= R;  // false for an all-NaN offset
        const uint64_t bal = __ballot(in[h]);
        cnt += __popcll(bal);
        need |= bal ? 1u << h : 0u;
      }
      if (!need) continue;
#pragma unroll
      for (int h = 0; h < GRP; ++h)
        if (need & (1u << h)) {
          Acc er, ei;
          point_term<MODE>(tab, dd[h], pe, in[h], hieps, er, ei);
          accumulate_term(u[k + h], B, er, ei);
        }
    }
  }
  // lane reduction in FP64 in a fixed butterfly order; every lane ends with the total
  double ud[RW][6];
#pragma unroll
  for (int k = 0; k < RW; ++k)
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      double v = (double)u[k][c];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      ud[k][c] = v;
    }
  if (lane < RW * 6) {
    const int k = lane / 6, c = lane % 6;
    double v = 0.0;
#pragma unroll
    for (int kk = 0; kk < RW; ++kk)
#pragma unroll
      for (int cc = 0; cc < 6; ++cc)
        if (kk == k && cc == c) v = ud[kk][cc];
    if (r0 + k < a.n) a.partial[((wk.blk * a.m + s) * a.n + r0 + k) * 6 + c] = v;
  }
  if (a.evals && lane == 0 && cnt) atomicAdd(a.evals, (unsigned long long)cnt);
}

// Per sample and 64-beam tile: bounding box of the live beams' centres Q
// (lo[3], hi[3]; an all-dead tile gets an empty box +inf / -inf).
__global__ __launch_bounds__(256) void k_tile_box(const double *__restrict__ emit, int64_t nb, int64_t ntiles,
                                                  double *__restrict__ box)
{
  const int lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int s = blockIdx.y;
  if (t >= ntiles) return;
  const double *E = emit + (int64_t)s * 12 * nb;
  const int64_t j = t * 64 + lane;
  double lo[3], hi[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double q = j < nb ? E[d * nb + j] : -1.0e300;
    const bool dead = !(q > -1.0e299);
    lo[d] = dead ? INFINITY : q;
    hi[d] = dead ? -INFINITY : q;
  }
#pragma unroll
  for (int d = 0; d < 3; ++d)
    for (int off = 32; off > 0; off >>= 1) {
      lo[d] = fmin(lo[d], __shfl_xor(lo[d], off));
      hi[d] = fmax(hi[d], __shfl_xor(hi[d], off));
    }
  if (lane < 6) {
    double v = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (lane == d) v = lo[d];
      if (lane == 3 + d) v = hi[d];
    }
    box[((int64_t)s * ntiles + t) * 6 + lane] = v;
  }
}

// out[perm[r]][s0 + s][c] (+)= sum over blocks of partial[blk][s][r][c].
// A workgroup takes 64 consecutive outputs (one per lane, so every block row
// is read coalesced); its RG wavefronts sum the blocks b = w, w + RG, ... in
// order, and lane l of wavefront 0 adds the RG partial sums in order: a
// fixed summation order, bitwise reproducible, with RG times the parallelism
// of one thread per output.
constexpr int RG = 16;
__global__ __launch_bounds__(64 * RG) void k_reduce_points(const double *__restrict__ partial, int nblk, int m,
                                                           int64_t n, const int32_t *__restrict__ perm,
                                                           double *__restrict__ out, int64_t out_samples, int s0,
                                                           int accumulate)
{
  __shared__ double part[RG][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t id = (int64_t)blockIdx.x * 64 + lane;  // (s, r, c6)
  const int64_t total = (int64_t)m * n * 6;
  const int64_t row = (int64_t)m * n * 6;  // doubles per block
  double v = 0.0;
  if (id < total)
    for (int b = w; b < nblk; b += RG) v += partial[(int64_t)b * row + id];
  part[w][lane] = v;
  __syncthreads();
  if (w == 0 && id < total) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < RG; ++k) t += part[k][lane];
    const int c6 = (int)(id % 6);
    const int64_t r = (id / 6) % n;
    const int s = (int)(id / (6 * n));
    const int64_t ro = perm ? perm[r] : r;
    double *o = out + (ro * out_samples + s0 + s) * 6 + c6;
    *o = accumulate ? *o + t : t;
  }
}

}  // namespace

int points_beams_per_block(int64_t nb, int64_t n, int m)
{
  // enough workgroups (about 8192) that the last partial round of resident
  // workgroups is a small fraction of the launch; ranges are whole 64-beam tiles
  const int64_t groups = (n + PG - 1) / PG;
  const int64_t pairs = nb * groups * (m > 0 ? m : 1);
  int64_t bpb = (pairs + 8191) / 8192;
  bpb = (bpb + 63) / 64 * 64;
  if (bpb < 1024) bpb = 1024;
  if (bpb > 8192) bpb = 8192;
  return (int)bpb;
}

hipError_t launch_sum_points(const PointsArgs &a, int *nblk_out, hipStream_t st)
{
  const int64_t nblk = (a.nb + a.beams_per_block - 1) / a.beams_per_block;
  *nblk_out = (int)nblk;
  if (a.nb == 0 || a.n == 0 || a.m == 0) return hipSuccess;
  if (a.m > 65535) return hipErrorInvalidConfiguration;
  const int64_t ntiles = (a.nb + 63) / 64;
  if (ntiles != a.ntiles) return hipErrorInvalidValue;
  if (!a.boxes_ready) {
    hipLaunchKernelGGL(k_tile_box, dim3((unsigned)((ntiles + 3) / 4), (unsigned)a.m), 256, 0, st, a.emit, a.nb,
                       ntiles, a.tile_box);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int groups = (int)((a.n + PG - 1) / PG);
  const int64_t units = (nblk * a.m + 7) / 8 * 8;
  const int64_t nwg = units * groups;
  if (nwg > 0x7fffffff) return hipErrorInvalidConfiguration;
  ProfScope prof(FGA_K_SUM_POINTS, st);
  if (a.precision == FGA_FP32)
    hipLaunchKernelGGL(k_sum_points<SUM_MIXED>, dim3((unsigned)nwg), 64 * WPW, 0, st, a, groups, nblk);
  else if (a.precision == FGA_FP32_ACC32)
    hipLaunchKernelGGL(k_sum_points<SUM_MIXED32>, dim3((unsigned)nwg), 64 * WPW, 0, st, a, groups, nblk);
  else
    hipLaunchKernelGGL(k_sum_points<SUM_FP64>, dim3((unsigned)nwg), 64 * WPW, 0, st, a, groups, nblk);
  return hipGetLastError();
}

hipError_t launch_reduce_points(const double *partial, int nblk, int m, int64_t n, const int32_t *perm, double *out,
                                int64_t out_samples, int s0, int accumulate, hipStream_t st)
{
  const int64_t total = (int64_t)m * n * 6;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_points, (unsigned)((total + 63) / 64), 64 * RG, 0, st, partial, nblk, m, n, perm, out,
                     out_samples, s0, accumulate);
  return hipGetLastError();
}

}  // namespace fga
