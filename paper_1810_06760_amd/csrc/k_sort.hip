// Spatial ordering of the beam set.
//
// Beams are independent, so their order in memory is free.  Sorting them
// along a Morton curve of their centres Q puts beams that share medium cells
// into the same wavefronts and workgroups: the trilinear gathers of the
// integrator then hit the same cache lines, and the receiver sums see
// compact beam tiles.  Dead beams sort last and are dropped, which is also
// the compaction step.  The radix sort is stable, so the order (and every
// result) is reproducible run to run.
#include <hipcub/hipcub.hpp>

#include "device_common.h"

namespace fga {
namespace {

__global__ __launch_bounds__(256) void k_bbox_partial(const double *__restrict__ F, const int32_t *__restrict__ I,
                                                      int64_t cap, int64_t n, double *__restrict__ part)
{
  __shared__ double red[6][4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double b[6] = {HUGE_VAL, HUGE_VAL, HUGE_VAL, -HUGE_VAL, -HUGE_VAL, -HUGE_VAL};
  if (i < n && (I[FGA_FLAGS * cap + i] & FGA_FLAG_ALIVE)) {
    for (int d = 0; d < 3; ++d) {
      const double q = F[(FGA_Q + d) * cap + i];
      b[d] = q;
      b[3 + d] = q;
    }
  }
  for (int off = 32; off > 0; off >>= 1)
    for (int d = 0; d < 3; ++d) {
      b[d] = fmin(b[d], __shfl_xor(b[d], off));
      b[3 + d] = fmax(b[3 + d], __shfl_xor(b[3 + d], off));
    }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 6; ++k) red[k][w] = b[k];
  __syncthreads();
  if (threadIdx.x < 6) {
    const int k = threadIdx.x;
    double v = red[k][0];
    for (int ww = 1; ww < 4; ++ww) v = k < 3 ? fmin(v, red[k][ww]) : fmax(v, red[k][ww]);
    part[(int64_t)blockIdx.x * 6 + k] = v;
  }
}

__global__ __launch_bounds__(256) void k_bbox_final(const double *__restrict__ part, int64_t nblk,
                                                    double *__restrict__ box)
{
  __shared__ double red[6][256];
  double b[6] = {HUGE_VAL, HUGE_VAL, HUGE_VAL, -HUGE_VAL, -HUGE_VAL, -HUGE_VAL};
  for (int64_t k = threadIdx.x; k < nblk; k += 256)
    for (int d = 0; d < 6; ++d) b[d] = d < 3 ? fmin(b[d], part[k * 6 + d]) : fmax(b[d], part[k * 6 + d]);
  for (int d = 0; d < 6; ++d) red[d][threadIdx.x] = b[d];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int d = 0; d < 6; ++d)
        red[d][threadIdx.x] = d < 3 ? fmin(red[d][threadIdx.x], red[d][threadIdx.x + s])
                                    : fmax(red[d][threadIdx.x], red[d][threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x < 6) box[threadIdx.x] = red[threadIdx.x][0];
}

__device__ __forceinline__ uint32_t spread3(uint32_t v)
{
  v &= 0x3ff;
  v = (v | (v << 16)) & 0x030000ff;
  v = (v | (v << 8)) & 0x0300f00f;
  v = (v | (v << 4)) & 0x030c30c3;
  v = (v | (v << 2)) & 0x09249249;
  return v;
}

__global__ __launch_bounds__(256) void k_morton(const double *__restrict__ F, const int32_t *__restrict__ I,
                                                int64_t cap, int64_t n, const double *__restrict__ box,
                                                uint32_t *__restrict__ keys, int32_t *__restrict__ vals)
{
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  uint32_t key = 0xffffffffu;
  if (I[FGA_FLAGS * cap + i] & FGA_FLAG_ALIVE) {
    uint32_t c[3];
    for (int d = 0; d < 3; ++d) {
      const double span = box[3 + d] - box[d];
      double u = span > 0 ? (F[(FGA_Q + d) * cap + i] - box[d]) / span * 1023.0 : 0.0;
      u = u < 0.0 ? 0.0 : (u > 1023.0 ? 1023.0 : u);
      c[d] = (uint32_t)u;
    }
    key = spread3(c[0]) | (spread3(c[1]) << 1) | (spread3(c[2]) << 2);
  }
  keys[i] = key;
  vals[i] = (int32_t)i;
}

__global__ __launch_bounds__(256) void k_count_alive(const uint32_t *__restrict__ keys, int64_t n,
                                                     int64_t *__restrict__ out)
{
  // keys are sorted: the first dead key marks the end of the live beams
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const bool live = keys[i] != 0xffffffffu;
  const bool next_dead = i + 1 == n || keys[i + 1] == 0xffffffffu;
  if (i == 0 && !live) *out = 0;
  if (live && next_dead) *out = i + 1;
}

template <class T>
__global__ __launch_bounds__(256) void k_gather(const T *__restrict__ src, const int32_t *__restrict__ perm,
                                                int64_t n, T *__restrict__ dst)
{
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = src[perm[i]];
}

struct SortBufs {
  uint32_t *k1, *k2;
  int32_t *v1, *v2;
  double *part, *box, *tmp;
  int64_t *alive;
  void *sort_tmp;
  size_t sort_bytes;
};

SortBufs sort_layout(int64_t n, Arena &ar)
{
  SortBufs b{};
  const int64_t nblk = (n + 255) / 256;
  b.k1 = ar.take<uint32_t>(n + 1);
  b.k2 = ar.take<uint32_t>(n + 1);
  b.v1 = ar.take<int32_t>(n + 1);
  b.v2 = ar.take<int32_t>(n + 1);
  b.part = ar.take<double>(6 * nblk + 6);
  b.box = ar.take<double>(6);
  b.tmp = ar.take<double>(n + 1);
  b.alive = ar.take<int64_t>(1);
  b.sort_bytes = 0;
  // size query only (no device work): the bytes come back in sort_bytes
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, b.sort_bytes, b.k1, b.k2, b.v1, b.v2, (int)(n > 0 ? n : 1), 0,
                                           32);
  b.sort_tmp = ar.take<char>(b.sort_bytes + 1);
  return b;
}

}  // namespace

fga_status sort_beams_spatial(fga_beams *b, Arena &ar, hipStream_t st, bool size_only, size_t *need)
{
  const int64_t n = b->count;
  SortBufs s = sort_layout(n, ar);
  if (size_only) {
    *need = ar.used;
    return FGA_OK;
  }
  if (!s.k1 || !s.k2 || !s.v1 || !s.v2 || !s.part || !s.box || !s.tmp || !s.alive || !s.sort_tmp)
    return fail(FGA_ENOMEM, "beam sort workspace too small (%zu bytes given)", ar.size);
  if (n == 0) return FGA_OK;
  if (n > 0x7fffffff) return fail(FGA_EUNSUPPORTED, "more than 2^31 beams in one sort");
  const int64_t nblk = (n + 255) / 256;
  const int64_t cap = b->capacity;
  hipLaunchKernelGGL(k_bbox_partial, (unsigned)nblk, 256, 0, st, b->f64, b->i32, cap, n, s.part);
  FGA_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_bbox_final, 1, 256, 0, st, s.part, nblk, s.box);
  FGA_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_morton, (unsigned)nblk, 256, 0, st, b->f64, b->i32, cap, n, s.box, s.k1, s.v1);
  FGA_LAUNCH_CHECK();
  // dead beams carry key 0xffffffff: sort all 32 bits so they land last
  size_t bytes = s.sort_bytes;
  FGA_HIP(hipcub::DeviceRadixSort::SortPairs(s.sort_tmp, bytes, s.k1, s.k2, s.v1, s.v2, (int)n, 0, 32, st));
  FGA_HIP(hipMemsetAsync(s.alive, 0, sizeof(int64_t), st));
  hipLaunchKernelGGL(k_count_alive, (unsigned)nblk, 256, 0, st, s.k2, n, s.alive);
  FGA_LAUNCH_CHECK();
  for (int p = 0; p < FGA_NF64; ++p) {
    double *pl = b->f64 + (int64_t)p * cap;
    hipLaunchKernelGGL(k_gather<double>, (unsigned)nblk, 256, 0, st, pl, s.v2, n, s.tmp);
    FGA_HIP(hipMemcpyAsync(pl, s.tmp, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  for (int p = 0; p < FGA_NI32; ++p) {
    int32_t *pl = b->i32 + (int64_t)p * cap;
    hipLaunchKernelGGL(k_gather<int32_t>, (unsigned)nblk, 256, 0, st, pl, s.v2, n, (int32_t *)s.tmp);
    FGA_HIP(hipMemcpyAsync(pl, s.tmp, n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
  }
  hipLaunchKernelGGL(k_gather<int64_t>, (unsigned)nblk, 256, 0, st, b->lineage, s.v2, n, (int64_t *)s.tmp);
  FGA_HIP(hipMemcpyAsync(b->lineage, s.tmp, n * sizeof(int64_t), hipMemcpyDeviceToDevice, st));
  FGA_LAUNCH_CHECK();
  int64_t alive = 0;
  FGA_HIP(hipMemcpyAsync(&alive, s.alive, sizeof alive, hipMemcpyDeviceToHost, st));
  FGA_HIP(hipStreamSynchronize(st));
  b->count = alive;
  return FGA_OK;
}

}  // namespace fga
