// Order-preserving stream compaction helpers: per-block counts, a
// single-workgroup exclusive scan of the block counts, and the stable
// compaction of the beam planes (a6: culling keeps beams in lineage order).
#include "device_common.h"

namespace fga {

// Exclusive scan of n int64 values by one workgroup of 1024 threads; each
// thread scans a contiguous chunk.  total (device) receives the sum.
namespace {
__global__ __launch_bounds__(1024) void k_scan_exclusive(const int64_t *__restrict__ in, int64_t *__restrict__ out,
                                                         int64_t n, int64_t *__restrict__ total)
{
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t per = (n + 1023) / 1024;
  const int64_t b = t * per, e = b + per < n ? b + per : n;
  int64_t s = 0;
  for (int64_t i = b; i < e; ++i) s += in[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int64_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = part[t] - s;
  for (int64_t i = b; i < e; ++i) {
    const int64_t v = in[i];
    out[i] = run;
    run += v;
  }
  if (t == 1023) *total = part[1023];
}

}  // namespace

hipError_t launch_scan(const int64_t *in, int64_t *out, int64_t n, int64_t *total, hipStream_t st)
{
  hipLaunchKernelGGL(k_scan_exclusive, 1, 1024, 0, st, in, out, n, total);
  return hipGetLastError();
}

namespace {

__global__ __launch_bounds__(256) void k_alive_counts(const int32_t *__restrict__ flags, int64_t n,
                                                      int64_t *__restrict__ counts)
{
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool keep = i < n && (flags[i] & FGA_FLAG_ALIVE);
  int total;
  block_rank(keep, &total);
  if (threadIdx.x == 0) counts[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void k_alive_dest(const int32_t *__restrict__ flags, int64_t n,
                                                    const int64_t *__restrict__ offs, int64_t *__restrict__ dest)
{
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool keep = i < n && (flags[i] & FGA_FLAG_ALIVE);
  int total;
  const int r = block_rank(keep, &total);
  if (i < n) dest[i] = keep ? offs[blockIdx.x] + r : -1;
}

template <class T>
__global__ __launch_bounds__(256) void k_scatter(const T *__restrict__ src, const int64_t *__restrict__ dest,
                                                 int64_t n, T *__restrict__ dst)
{
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    const int64_t d = dest[i];
    if (d >= 0) dst[d] = src[i];
  }
}

}  // namespace

// Beam-set counts for fga_beams_info: ctr[0] alive, [1] quarantined, [2..4]
// alive per branch, [5] alive children (generation > 0); one ballot per
// wavefront and counter, one atomic per wavefront.
__global__ __launch_bounds__(64) void k_zero_counters(unsigned long long *ctr, int n)
{
  if ((int)threadIdx.x < n) ctr[threadIdx.x] = 0ull;
}

__global__ __launch_bounds__(256) void k_beams_info(const int32_t *__restrict__ i32, int64_t cap, int64_t n,
                                                    unsigned long long *__restrict__ ctr)
{
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int32_t flags = 0, br = -1, gen = 0;
  if (i < n) {
    flags = i32[FGA_FLAGS * cap + i];
    br = i32[FGA_BRANCH * cap + i];
    gen = i32[FGA_GEN * cap + i];
  }
  const bool alive = i < n && (flags & FGA_FLAG_ALIVE);
  const bool pred[6] = {alive, i < n && (flags & FGA_FLAG_QUARANTINED) != 0, alive && br == 0, alive && br == 1,
                        alive && br == 2, alive && gen > 0};
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const unsigned long long m = __ballot(pred[k]);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(ctr + k, (unsigned long long)__popcll(m));
  }
}

hipError_t launch_beams_info(const fga_beams *b, unsigned long long *ctr, hipStream_t st)
{
  hipLaunchKernelGGL(k_zero_counters, 1, 64, 0, st, ctr, 6);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || b->count <= 0) return e;
  hipLaunchKernelGGL(k_beams_info, (unsigned)((b->count + 255) / 256), 256, 0, st, b->i32, b->capacity, b->count,
                     ctr);
  return hipGetLastError();
}

fga_status compact_beams(fga_beams *b, Arena &ar, hipStream_t st, bool size_only, size_t *need)
{
  const int64_t n = b->count;
  const int64_t nblk = (n + 255) / 256;
  int64_t *counts = ar.take<int64_t>(nblk + 1);
  int64_t *offs = ar.take<int64_t>(nblk + 1);
  int64_t *total = ar.take<int64_t>(1);
  int64_t *dest = ar.take<int64_t>(n + 1);
  double *tmp = ar.take<double>(n + 1);
  if (size_only) {
    *need = ar.used;
    return FGA_OK;
  }
  if (!counts || !offs || !total || !dest || !tmp)
    return fail(FGA_ENOMEM, "compaction workspace too small (%zu bytes given)", ar.size);
  if (n == 0) return FGA_OK;
  const int32_t *flags = b->i32 + (int64_t)FGA_FLAGS * b->capacity;
  hipLaunchKernelGGL(k_alive_counts, (unsigned)nblk, 256, 0, st, flags, n, counts);
  FGA_LAUNCH_CHECK();
  FGA_HIP(launch_scan(counts, offs, nblk, total, st));
  hipLaunchKernelGGL(k_alive_dest, (unsigned)nblk, 256, 0, st, flags, n, offs, dest);
  FGA_LAUNCH_CHECK();
  int64_t kept = 0;
  FGA_HIP(hipMemcpyAsync(&kept, total, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  FGA_HIP(hipStreamSynchronize(st));
  if (kept == n) return FGA_OK;
  for (int p = 0; p < FGA_NF64; ++p) {
    double *pl = b->f64 + (int64_t)p * b->capacity;
    hipLaunchKernelGGL(k_scatter<double>, (unsigned)nblk, 256, 0, st, pl, dest, n, tmp);
    FGA_HIP(hipMemcpyAsync(pl, tmp, kept * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  for (int p = 0; p < FGA_NI32; ++p) {
    int32_t *pl = b->i32 + (int64_t)p * b->capacity;
    hipLaunchKernelGGL(k_scatter<int32_t>, (unsigned)nblk, 256, 0, st, pl, dest, n, (int32_t *)tmp);
    FGA_HIP(hipMemcpyAsync(pl, tmp, kept * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
  }
  hipLaunchKernelGGL(k_scatter<int64_t>, (unsigned)nblk, 256, 0, st, b->lineage, dest, n, (int64_t *)tmp);
  FGA_HIP(hipMemcpyAsync(b->lineage, tmp, kept * sizeof(int64_t), hipMemcpyDeviceToDevice, st));
  FGA_LAUNCH_CHECK();
  b->count = kept;
  return FGA_OK;
}

}  // namespace fga
