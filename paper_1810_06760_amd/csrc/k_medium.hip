// Grid media: per-node derived fields (c, grad c, Hessian) by second-order
// periodic central differences, one 128-byte record per node so that a
// trilinear gather touches one cache line per corner; and the coefficients of
// the periodic cubic B-spline through the node values.
#include "device_common.h"

namespace fga {
namespace {

__global__ __launch_bounds__(256) void k_grid_build(const double *__restrict__ c, int nx, int ny, int nz,
                                                    double hx, double hy, double hz, double *__restrict__ tab)
{
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = (int64_t)nx * ny * nz;
  if (id >= total) return;
  const int i = (int)(id % nx), j = (int)((id / nx) % ny), k = (int)(id / ((int64_t)nx * ny));
  auto at = [&](int a, int b, int d) -> double {
    a = (a + nx) % nx; b = (b + ny) % ny; d = (d + nz) % nz;
    return c[((int64_t)d * ny + b) * nx + a];
  };
  const double c0 = at(i, j, k);
  double *o = tab + (int64_t)FGA_GRID_NODE_DOUBLES * id;
  o[0] = c0;
  o[1] = (at(i + 1, j, k) - at(i - 1, j, k)) / (2.0 * hx);
  o[2] = (at(i, j + 1, k) - at(i, j - 1, k)) / (2.0 * hy);
  o[3] = (at(i, j, k + 1) - at(i, j, k - 1)) / (2.0 * hz);
  o[4] = (at(i + 1, j, k) - 2.0 * c0 + at(i - 1, j, k)) / (hx * hx);
  o[5] = (at(i, j + 1, k) - 2.0 * c0 + at(i, j - 1, k)) / (hy * hy);
  o[6] = (at(i, j, k + 1) - 2.0 * c0 + at(i, j, k - 1)) / (hz * hz);
  o[7] = (at(i + 1, j + 1, k) - at(i + 1, j - 1, k) - at(i - 1, j + 1, k) + at(i - 1, j - 1, k)) / (4.0 * hx * hy);
  o[8] = (at(i + 1, j, k + 1) - at(i + 1, j, k - 1) - at(i - 1, j, k + 1) + at(i - 1, j, k - 1)) / (4.0 * hx * hz);
  o[9] = (at(i, j + 1, k + 1) - at(i, j + 1, k - 1) - at(i, j - 1, k + 1) + at(i, j - 1, k - 1)) / (4.0 * hy * hz);
  for (int f = 10; f < FGA_GRID_NODE_DOUBLES; ++f) o[f] = 0.0;
}

// Periodic cubic B-spline coefficients along one axis: the interpolation
// condition (a[i-1] + 4 a[i] + a[i+1]) / 6 = f[i] is inverted by the filter
// 6 / (q^-1 + 4 + q) = -6 zp / ((1 - zp q^-1)(1 - zp q)), zp = sqrt(3) - 2, run
// as a causal and an anti-causal first-order recursion (Unser, Aldroubi and
// Eden 1993); on a periodic line each recursion starts from its geometric sum
// over one whole period.  One thread per line of nodes along `axis`, read from
// src and written to dst (dst may be src: every value is read before it is
// overwritten).
__global__ __launch_bounds__(256) void k_spline_lines(const double *src, double *dst, int nx, int ny, int nz,
                                                      int axis)
{
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int len;
  int64_t stride, base, nlines;
  if (axis == 0) {
    len = nx; stride = 1; nlines = (int64_t)ny * nz; base = id * nx;
  } else if (axis == 1) {
    len = ny; stride = nx; nlines = (int64_t)nx * nz;
    base = (id / nx) * (int64_t)nx * ny + id % nx;
  } else {
    len = nz; stride = (int64_t)nx * ny; nlines = (int64_t)nx * ny; base = id;
  }
  if (id >= nlines) return;
  const double zp = sqrt(3.0) - 2.0;
  // causal: c+[k] = f[k] + zp c+[k-1], c+[0] = sum_j zp^j f[-j mod len] / (1 - zp^len)
  double zj = 1.0, acc = src[base];
  for (int j = 1; j < len; ++j) {
    zj *= zp;
    acc += zj * src[base + (len - j) * stride];
  }
  const double zn = zj * zp;
  double cp = acc / (1.0 - zn);
  dst[base] = cp;
  for (int k = 1; k < len; ++k) {
    cp = src[base + k * stride] + zp * cp;
    dst[base + k * stride] = cp;
  }
  // anti-causal: d[k] = c+[k] + zp d[k+1], d[len-1] = sum_j zp^j c+[(len-1+j) mod len] / (1 - zp^len);
  // a = -6 zp d
  zj = 1.0;
  acc = dst[base + (len - 1) * stride];
  for (int j = 1; j < len; ++j) {
    zj *= zp;
    acc += zj * dst[base + (j - 1) * stride];
  }
  double d = acc / (1.0 - zn);
  const double gain = -6.0 * zp;
  dst[base + (len - 1) * stride] = gain * d;
  for (int k = len - 2; k >= 0; --k) {
    d = dst[base + k * stride] + zp * d;
    dst[base + k * stride] = gain * d;
  }
}

}  // namespace

hipError_t launch_spline_coefficients(const int n[3], const double *c, double *coef, hipStream_t st)
{
  const int64_t lines[3] = {(int64_t)n[1] * n[2], (int64_t)n[0] * n[2], (int64_t)n[0] * n[1]};
  for (int axis = 0; axis < 3; ++axis) {
    hipLaunchKernelGGL(k_spline_lines, (unsigned)((lines[axis] + 255) / 256), 256, 0, st, axis == 0 ? c : coef,
                       coef, n[0], n[1], n[2], axis);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_grid_build(const int n[3], const double h[3], const double *c, double *table, hipStream_t st)
{
  const int64_t total = (int64_t)n[0] * n[1] * n[2];
  hipLaunchKernelGGL(k_grid_build, (unsigned)((total + 255) / 256), 256, 0, st, c, n[0], n[1], n[2], h[0], h[1],
                     h[2], table);
  return hipGetLastError();
}

// Receivers given in spherical coordinates (r, theta, phi) with theta the
// longitude and phi the latitude (the coordinates of the Earth examples,
// opening of Sec. 3): x = (r cos theta cos phi, r sin theta cos phi, r sin phi).
__global__ __launch_bounds__(256) void k_spherical_to_cartesian(const double *__restrict__ rtp, int64_t n,
                                                                double *__restrict__ xyz)
{
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double r = rtp[3 * i], th = rtp[3 * i + 1], ph = rtp[3 * i + 2];
  double st, ct, sp, cp;
  sincos(th, &st, &ct);
  sincos(ph, &sp, &cp);
  xyz[3 * i] = r * ct * cp;
  xyz[3 * i + 1] = r * st * cp;
  xyz[3 * i + 2] = r * sp;
}

hipError_t launch_spherical_to_cartesian(const double *rtp, int64_t n, double *xyz, hipStream_t st)
{
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_spherical_to_cartesian, (unsigned)((n + 255) / 256), 256, 0, st, rtp, n, xyz);
  return hipGetLastError();
}

}  // namespace fga
