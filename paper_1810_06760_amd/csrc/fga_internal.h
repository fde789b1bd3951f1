// Internal declarations of the gfx950 FGA library (host launchers, device
// helpers, error reporting).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "fga.h"

namespace fga {

// ---------------------------------------------------------------- errors --
void set_error(const char *fmt, ...);
fga_status fail(fga_status st, const char *fmt, ...);

#define FGA_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return ::fga::fail(FGA_EDEVICE, "%s failed: %s (%s:%d)", #call,                  \
                         hipGetErrorString(e_), __FILE__, __LINE__);                   \
  } while (0)

#define FGA_LAUNCH_CHECK()                                                             \
  do {                                                                                 \
    hipError_t e_ = hipGetLastError();                                                 \
    if (e_ != hipSuccess)                                                              \
      return ::fga::fail(FGA_EDEVICE, "kernel launch failed: %s (%s:%d)",              \
                         hipGetErrorString(e_), __FILE__, __LINE__);                   \
  } while (0)

// --------------------------------------------------------------- timing --
// Records a start event on construction and a stop event on destruction
// (around one kernel launch) when profiling is enabled.
struct ProfScope {
  int k;
  hipStream_t st;
  hipEvent_t a = nullptr;
  ProfScope(int kernel, hipStream_t s);
  ~ProfScope();
};

// ------------------------------------------------------------- workspace --
// Bump allocator over a caller workspace; every sub-buffer is 256-byte aligned.
struct Arena {
  char *base = nullptr;
  size_t size = 0, used = 0;
  Arena(void *b, size_t s) : base(static_cast<char *>(b)), size(s) {}
  template <class T> T *take(size_t n) {
    size_t off = (used + 255) & ~size_t(255);
    used = off + n * sizeof(T);
    if (base == nullptr || used > size) return nullptr;
    return reinterpret_cast<T *>(base + off);
  }
  static size_t need(size_t bytes) { return (bytes + 255) & ~size_t(255); }
};

// ----------------------------------------------------------- media (GPU) --
// Device view of a medium; passed by value to kernels.
struct DevMedium {
  int kind;
  double cp, cs;
  // grid
  const double *table;
  int n[3];
  double lo[3], ih[3];
  int64_t field_stride;   // doubles between the c_P and c_S tables
  int two_fields;
  double cs_ratio;
  int smooth;             // 1: cubic B-spline of the node values (coef), 0: trilinear records
  const double *coef;     // spline coefficients, c_P then c_S (coef_stride apart)
  int64_t coef_stride;
  // layered
  int geometry, nlayer;
  double bound[FGA_MAX_LAYERS];
  double cpl[FGA_MAX_LAYERS], csl[FGA_MAX_LAYERS], rhol[FGA_MAX_LAYERS];
  double gradl[FGA_MAX_LAYERS];  // relative speed gradient per layer (0: constant)
  double anom_amp[FGA_MAX_LAYERS], anom_beta[FGA_MAX_LAYERS];  // Gaussian anomaly per layer (0: none)
  double anom_x[FGA_MAX_LAYERS][3], anom_w[FGA_MAX_LAYERS][3];
  int any_grad;                  // some layer has a gradient: the general RK4 step
  double surface;                // > 0: traction-free surface closing the outermost region
};

fga_status make_dev_medium(const fga_medium *m, DevMedium *out);

// -------------------------------------------------------------- launchers --
hipError_t launch_grid_build(const int n[3], const double h[3], const double *c, double *table,
                             hipStream_t st);
hipError_t launch_spline_coefficients(const int n[3], const double *c, double *coef, hipStream_t st);

struct IntegrateArgs {
  double *f64;
  int32_t *i32;
  int64_t cap;
  int64_t beg, end;          // beams [beg, end)
  double dt;
  int nsteps;
  int step0;                 // global index of the first step of this launch
  int stride;                // emit after steps with (step+1) % stride == 0 (0: never)
  double *emit;              // [n_emit][12][end-beg]
  double eps_emit;
  double cutoff_abs;
  unsigned long long *counters;  // [0] beam-steps, [1] culled, [2] quarantined
  int s_vector;              // 1: frame-free S amplitudes (grid media)
};
hipError_t launch_integrate(const DevMedium &m, const IntegrateArgs &a, hipStream_t st);

struct PointsArgs {
  const double *emit;        // [m][12][nb] records
  int64_t nb;                // beams in the batch
  int m;                     // samples in the batch
  const double *xyz;         // [n][3]
  int64_t n;
  double eps, tau;
  double *partial;           // [nblk][m][n][6]
  int beams_per_block;
  unsigned long long *evals;
  double *tile_box;          // scratch [m][ntiles][6], ntiles = ceil(nb / 64)
  int64_t ntiles;
  int boxes_ready;           // tile_box already holds the boxes (written with the records)
  int precision;             // FGA_FP64, or FGA_FP32: FP32 exp/sin/cos of FP64-reduced arguments
};
hipError_t launch_sum_points(const PointsArgs &a, int *nblk_out, hipStream_t st);
// beams walked by one point-sum workgroup for nb beams, n points and m samples
// per launch (a multiple of 64 in [1024, 8192]); partial holds
// ceil(nb / that) * m * n * 6 doubles
int points_beams_per_block(int64_t nb, int64_t n, int m);
// seis[perm[r]][s0 + s][c] (+)= sum_blk partial[blk][s][r][c]   (perm NULL: identity)
hipError_t launch_reduce_points(const double *partial, int nblk, int m, int64_t n, const int32_t *perm,
                                double *out, int64_t out_samples, int s0, int accumulate, hipStream_t st);
// Copies n points (device [n][3]) into xyz_sorted in Morton order of their
// positions and sets perm[k] = original index of sorted point k.  Synchronises st.
fga_status sort_points(const double *xyz, int64_t n, double *xyz_sorted, int32_t *perm, hipStream_t st);
// rtp (device [n][3]: radius, longitude, latitude) -> xyz (device [n][3])
hipError_t launch_spherical_to_cartesian(const double *rtp, int64_t n, double *xyz, hipStream_t st);

// beams -> emission records (current state, one sample)
// box (may be NULL): also the tile boxes of the records, [ceil((end - beg) / 64)][6]
hipError_t launch_emit(const double *f64, const int32_t *i32, int64_t cap, int64_t beg, int64_t end,
                       double eps, double *emit, double *box, hipStream_t st);

// decomposition
struct DecompArgs {
  const fga_mesh *mesh;
  const double *Ft;          // complex [3][nz*npz][ny*npy][nx*npx] (see k_decompose)
  const double *Gt;          // NULL or complex [2][3][...] (FBI[g/c_P], FBI[g/c_S])
  double *f64;
  int32_t *i32;
  int64_t *lineage;
  int64_t cap;
};
fga_status decompose_impl(const DevMedium &dm, const fga_mesh *mesh, const double *f, const double *g,
                          fga_beams *beams, Arena &ar, hipStream_t st, bool size_only, size_t *need);

// Interface step of a layered medium after one integrator step: beams that
// left their layer during the step (flag FGA_FLAG_CROSS, state still at the
// start of the step) are split into children (Snell, elastic boundary
// problem, Jacobian map) which finish the step in their own layers.
struct InterfaceArgs {
  double *f64;
  int32_t *i32;
  int64_t *lineage;
  int64_t cap;
  int64_t n;                 // beams in the set before the step
  const int32_t *list;       // [nlist] the crossing beams' slots, increasing
  int64_t nlist;
  double dt;
  int gen_max;
  double child_cut;
  int64_t *blk_extra;        // [ceil(nlist / 256)] extra slots per workgroup (pass 1 output)
  int64_t *blk_off;          // [ceil(nlist / 256)] exclusive scan of blk_extra (pass 2 input)
  unsigned long long *counters;  // [0] crossings, [1] children, [2] retired at the generation cap
};
// pass 1 (write = 0): per-workgroup counts of extra slots; pass 2 (write = 1):
// children written (first child in the parent's slot, the others appended at
// n + blk_off + rank)
hipError_t launch_interface(const DevMedium &m, const InterfaceArgs &a, int write, hipStream_t st);
// The slots of [0, n) flagged FGA_FLAG_CROSS, in increasing order, into
// sorted[0, *ncross) (list: unordered scratch of the same size; count: one
// device counter; tmp: cross_sort_bytes(cap) bytes).  Synchronises st.
size_t cross_sort_bytes(int64_t cap);
hipError_t collect_crossers(const int32_t *flags, int64_t n, int32_t *list, int32_t *sorted,
                            unsigned long long *count, void *tmp, size_t tmp_bytes, hipStream_t st,
                            int64_t *ncross);

// exclusive scan of n int64 values (one workgroup); total = sum
hipError_t launch_scan(const int64_t *in, int64_t *out, int64_t n, int64_t *total, hipStream_t st);

// Morton-order the beam set by Q (dead beams dropped; count updated; synchronises st)
fga_status sort_beams_spatial(fga_beams *b, Arena &ar, hipStream_t st, bool size_only, size_t *need);

// stable compaction of the beam set by FLAGS & ALIVE
fga_status compact_beams(fga_beams *b, Arena &ar, hipStream_t st, bool size_only, size_t *need);
// counts for fga_beams_info into ctr[6] (device)
hipError_t launch_beams_info(const fga_beams *b, unsigned long long *ctr, hipStream_t st);

// grid summation
fga_status grid_sum_impl(const fga_beams *b, double eps, double tau, const int n[3], const double lo[3],
                         const double h[3], int precision, double *out, Arena &ar, hipStream_t st,
                         bool size_only, size_t *need, int64_t *evals, bool add = false);

}  // namespace fga
