// C ABI of the gfx950 FGA library: argument validation, workspace layout and
// the host-side sequencing of the kernels.  See include/fga.h.
#include <cmath>
#include <cstring>
#include <string>
#include <algorithm>
#include <mutex>
#include <vector>

#include "device_common.h"

namespace fga {

static thread_local std::string g_err;

void set_error(const char *fmt, ...)
{
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

fga_status fail(fga_status st, const char *fmt, ...)
{
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

int64_t decompose_candidates(const fga_mesh *m);

// ------------------------------------------------------------ kernel timing --
namespace {
struct ProfRec {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
};
bool g_prof_on = false;
ProfRec g_prof[FGA_K_COUNT];

void prof_clear()
{
  for (auto &r : g_prof) {
    for (auto &p : r.ev) {
      (void)hipEventDestroy(p.first);
      (void)hipEventDestroy(p.second);
    }
    r.ev.clear();
  }
}
}  // namespace

ProfScope::ProfScope(int kernel, hipStream_t s) : k(kernel), st(s)
{
  if (g_prof_on && hipEventCreate(&a) == hipSuccess) {
    if (hipEventRecord(a, st) != hipSuccess) {
      (void)hipEventDestroy(a);
      a = nullptr;
    }
  } else {
    a = nullptr;
  }
}

ProfScope::~ProfScope()
{
  if (!a) return;
  hipEvent_t b;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return;
  }
  if (hipEventRecord(b, st) != hipSuccess) {  // an unrecorded pair would time nothing
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return;
  }
  g_prof[k].ev.emplace_back(a, b);
}

fga_status make_dev_medium(const fga_medium *m, DevMedium *o)
{
  if (!m) return fail(FGA_EINVAL, "medium is NULL");
  std::memset(o, 0, sizeof(*o));
  o->kind = m->kind;
  switch (m->kind) {
  case FGA_MEDIUM_HOMOGENEOUS:
    if (!(m->cp > 0) || !(m->cs > 0)) return fail(FGA_EINVAL, "homogeneous medium needs cp > 0 and cs > 0");
    o->cp = m->cp;
    o->cs = m->cs;
    return FGA_OK;
  case FGA_MEDIUM_GRID:
    if (!m->table) return fail(FGA_EINVAL, "grid medium table is NULL");
    for (int d = 0; d < 3; ++d) {
      if (m->n[d] < 3) return fail(FGA_EINVAL, "grid medium needs n >= 3 per axis");
      if (!(m->h[d] > 0)) return fail(FGA_EINVAL, "grid medium needs h > 0");
      o->n[d] = m->n[d];
      o->lo[d] = m->lo[d];
      o->ih[d] = 1.0 / m->h[d];
    }
    o->table = m->table;
    o->two_fields = m->two_fields ? 1 : 0;
    o->cs_ratio = m->cs_ratio;
    o->field_stride = (int64_t)FGA_GRID_NODE_DOUBLES * m->n[0] * m->n[1] * m->n[2];
    o->smooth = m->smooth ? 1 : 0;
    o->coef_stride = (int64_t)m->n[0] * m->n[1] * m->n[2];
    o->coef = m->table + o->field_stride * (o->two_fields ? 2 : 1);
    if (!o->two_fields && !(m->cs_ratio > 0)) return fail(FGA_EINVAL, "grid medium needs cs_ratio > 0");
    return FGA_OK;
  case FGA_MEDIUM_LAYERED:
    if (m->nlayer < 1 || m->nlayer > FGA_MAX_LAYERS) return fail(FGA_EINVAL, "layered medium needs 1..8 layers");
    if (m->geometry != 0 && m->geometry != 1) return fail(FGA_EINVAL, "layered geometry must be 0 or 1");
    o->geometry = m->geometry;
    o->nlayer = m->nlayer;
    o->any_grad = 0;
    for (int l = 0; l < FGA_MAX_LAYERS; ++l) {
      o->bound[l] = m->bound[l];
      o->cpl[l] = m->cpl[l];
      o->csl[l] = m->csl[l];
      o->rhol[l] = m->rhol[l];
      o->gradl[l] = l < m->nlayer ? m->gradl[l] : 0.0;
      if (l < m->nlayer && m->gradl[l] != 0.0) o->any_grad = 1;
      // a Gaussian anomaly curves the rays too: the same general step and crossing
      o->anom_amp[l] = l < m->nlayer ? m->anom_amp[l] : 0.0;
      o->anom_beta[l] = m->anom_beta[l];
      for (int d = 0; d < 3; ++d) {
        o->anom_x[l][d] = m->anom_x[l][d];
        o->anom_w[l][d] = m->anom_w[l][d];
      }
      if (l < m->nlayer && m->anom_amp[l] != 0.0) o->any_grad = 1;
    }
    for (int l = 0; l < m->nlayer; ++l) {
      if (!std::isfinite(m->gradl[l])) return fail(FGA_EINVAL, "layer %d has a non-finite gradient", l);
      if (m->anom_amp[l] != 0.0) {
        bool ok = std::isfinite(m->anom_amp[l]) && std::isfinite(m->anom_beta[l]) && m->anom_beta[l] >= 0.0;
        for (int d = 0; d < 3; ++d)
          ok = ok && std::isfinite(m->anom_x[l][d]) && std::isfinite(m->anom_w[l][d]) && m->anom_w[l][d] >= 0.0;
        if (!ok)
          return fail(FGA_EINVAL, "layer %d: the anomaly needs finite values, beta >= 0 and weights >= 0", l);
      }
    }
    if (m->geometry == 1 && m->gradl[m->nlayer - 1] != 0.0)
      return fail(FGA_EINVAL, "the innermost spherical layer must have a constant speed");
    o->surface = m->surface;
    if (!(m->surface >= 0.0)) return fail(FGA_EINVAL, "surface must be >= 0 (0: none)");
    if (m->surface > 0.0 && m->nlayer > 1 &&
        (m->geometry == 1 ? !(m->surface > m->bound[0]) : !(m->surface > m->bound[m->nlayer - 2])))
      return fail(FGA_EINVAL, "the free surface must lie outside every interface");
    for (int l = 0; l < m->nlayer; ++l)
      if (!(m->cpl[l] > 0) || !(m->csl[l] > 0) || !(m->rhol[l] > 0))
        return fail(FGA_EINVAL, "layer %d has non-positive speed or density", l);
    for (int l = 0; l + 1 < m->nlayer - 1; ++l)
      if (m->geometry == 0 ? !(m->bound[l] < m->bound[l + 1]) : !(m->bound[l] > m->bound[l + 1] && m->bound[l + 1] > 0))
        return fail(FGA_EINVAL, "layer bounds must be increasing (flat) or decreasing and positive (spherical)");
    return FGA_OK;
  default:
    return fail(FGA_EINVAL, "unknown medium kind %d", m->kind);
  }
}

fga_status sort_points(const double *xyz, int64_t n, double *xyz_sorted, int32_t *perm, hipStream_t st)
{
  std::vector<double> h((size_t)3 * n);
  FGA_HIP(hipMemcpyAsync(h.data(), xyz, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  FGA_HIP(hipStreamSynchronize(st));
  double lo[3] = {HUGE_VAL, HUGE_VAL, HUGE_VAL}, hi[3] = {-HUGE_VAL, -HUGE_VAL, -HUGE_VAL};
  for (int64_t i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) {
      const double v = h[3 * i + d];
      if (!std::isfinite(v)) return fail(FGA_EINVAL, "point %lld is not finite", (long long)i);
      lo[d] = v < lo[d] ? v : lo[d];
      hi[d] = v > hi[d] ? v : hi[d];
    }
  // 10-bit Morton key of each point within the points' bounding box
  std::vector<std::pair<uint32_t, int32_t>> key((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    uint32_t k = 0;
    uint32_t c[3];
    for (int d = 0; d < 3; ++d) {
      const double span = hi[d] > lo[d] ? hi[d] - lo[d] : 1.0;
      double u = (h[3 * i + d] - lo[d]) / span * 1023.0;
      c[d] = (uint32_t)(u < 0 ? 0 : (u > 1023 ? 1023 : u));
    }
    for (int b = 9; b >= 0; --b)
      for (int d = 2; d >= 0; --d) k = (k << 1) | ((c[d] >> b) & 1u);
    key[(size_t)i] = {k, (int32_t)i};
  }
  std::stable_sort(key.begin(), key.end(),
                   [](const std::pair<uint32_t, int32_t> &a, const std::pair<uint32_t, int32_t> &b) {
                     return a.first < b.first;
                   });
  std::vector<double> hs((size_t)3 * n);
  std::vector<int32_t> hp((size_t)n);
  for (int64_t k = 0; k < n; ++k) {
    const int32_t i = key[(size_t)k].second;
    hp[(size_t)k] = i;
    for (int d = 0; d < 3; ++d) hs[3 * k + d] = h[3 * (size_t)i + d];
  }
  FGA_HIP(hipMemcpyAsync(xyz_sorted, hs.data(), hs.size() * sizeof(double), hipMemcpyHostToDevice, st));
  FGA_HIP(hipMemcpyAsync(perm, hp.data(), hp.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
  FGA_HIP(hipStreamSynchronize(st));
  return FGA_OK;
}

static bool point_precision_ok(int p) { return p == FGA_FP64 || p == FGA_FP32 || p == FGA_FP32_ACC32; }

static fga_status check_beams(const fga_beams *b)
{
  if (!b) return fail(FGA_EINVAL, "beams is NULL");
  if (b->capacity < 0 || b->count < 0 || b->count > b->capacity) return fail(FGA_EINVAL, "beam count/capacity invalid");
  if (b->capacity > 0 && (!b->f64 || !b->i32 || !b->lineage)) return fail(FGA_EINVAL, "beam planes are NULL");
  return FGA_OK;
}

static fga_status check_mesh(const fga_mesh *m)
{
  if (!m) return fail(FGA_EINVAL, "mesh is NULL");
  if (!(m->eps > 0)) return fail(FGA_EINVAL, "eps must be > 0");
  for (int d = 0; d < 3; ++d) {
    if (m->nq[d] < 1 || m->np[d] < 1 || m->ny[d] < 1) return fail(FGA_EINVAL, "mesh sizes must be >= 1");
    if (!(m->qh[d] > 0) || !(m->ph[d] > 0) || !(m->yh[d] > 0)) return fail(FGA_EINVAL, "mesh spacings must be > 0");
  }
  if (m->branch_mask < 1 || m->branch_mask > 7) return fail(FGA_EINVAL, "branch_mask must be in 1..7");
  // |p| must not vanish on the p mesh: p_d = lo + i h is zero only if lo/h is a non-positive integer > -n
  bool zero = true;
  for (int d = 0; d < 3; ++d) {
    const double u = -m->plo[d] / m->ph[d];
    zero = zero && u >= 0 && u <= m->np[d] - 1 && std::fabs(u - std::round(u)) < 1e-12;
  }
  if (zero) return fail(FGA_EINVAL, "the p mesh contains p = 0");
  const double ncand = 6.0 * m->nq[0] * m->nq[1] * m->nq[2] * (double)m->np[0] * m->np[1] * m->np[2];
  if (ncand > 4.0e9) return fail(FGA_EUNSUPPORTED, "more than 4e9 candidate beams");
  return FGA_OK;
}

}  // namespace fga

using namespace fga;

fga_status fga_beams_info(const fga_beams *beams, fga_beams_stats *out, void *workspace, size_t workspace_bytes,
                          void *stream)
{
  fga_status s;
  if ((s = check_beams(beams)) != FGA_OK) return s;
  if (!out) return fail(FGA_EINVAL, "stats output is NULL");
  if (!workspace || workspace_bytes < FGA_BEAMS_INFO_WORKSPACE || ((uintptr_t)workspace & 7))
    return fail(FGA_EINVAL, "fga_beams_info needs %d bytes of 8-byte aligned device workspace",
                FGA_BEAMS_INFO_WORKSPACE);
  hipStream_t st = (hipStream_t)stream;
  unsigned long long *ctr = static_cast<unsigned long long *>(workspace);
  FGA_HIP(launch_beams_info(beams, ctr, st));
  unsigned long long h[6];
  FGA_HIP(hipMemcpyAsync(h, ctr, sizeof(h), hipMemcpyDeviceToHost, st));
  FGA_HIP(hipStreamSynchronize(st));
  out->count = beams->count;
  out->alive = (int64_t)h[0];
  out->quarantined = (int64_t)h[1];
  for (int b = 0; b < 3; ++b) out->by_branch[b] = (int64_t)h[2 + b];
  out->children = (int64_t)h[5];
  return FGA_OK;
}

// Plane-by-plane copies between a beam set and [plane][n] arrays (host or
// device: hipMemcpyDefault lets the runtime tell them apart).
template <typename T>
static hipError_t copy_planes(T *dst, size_t dpitch, const T *src, size_t spitch, int64_t n, int planes,
                              hipStream_t st)
{
  // one copy per plane (a 2-D copy's pitch would be limited to 2^31 bytes)
  for (int f = 0; f < planes && n > 0; ++f) {
    const hipError_t e =
        hipMemcpyAsync(dst + f * dpitch, src + f * spitch, (size_t)n * sizeof(T), hipMemcpyDefault, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

fga_status fga_beams_export(const fga_beams *beams, double *f64, int32_t *i32, int64_t *lineage, void *stream)
{
  fga_status s;
  if ((s = check_beams(beams)) != FGA_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = beams->count;
  const size_t cap = (size_t)beams->capacity;
  if (f64) FGA_HIP(copy_planes(f64, (size_t)n, beams->f64, cap, n, FGA_NF64, st));
  if (i32) FGA_HIP(copy_planes(i32, (size_t)n, beams->i32, cap, n, FGA_NI32, st));
  if (lineage) FGA_HIP(copy_planes(lineage, (size_t)n, beams->lineage, cap, n, 1, st));
  FGA_HIP(hipStreamSynchronize(st));
  return FGA_OK;
}

fga_status fga_beams_import(fga_beams *beams, int64_t n, const double *f64, const int32_t *i32,
                            const int64_t *lineage, void *stream)
{
  fga_status s;
  if ((s = check_beams(beams)) != FGA_OK) return s;
  if (n < 0) return fail(FGA_EINVAL, "n < 0");
  if (n > beams->capacity) return fail(FGA_ECAPACITY, "%lld beams do not fit a capacity of %lld", (long long)n,
                                       (long long)beams->capacity);
  if (n > 0 && (!f64 || !i32 || !lineage)) return fail(FGA_EINVAL, "import arrays are NULL");
  hipStream_t st = (hipStream_t)stream;
  const size_t cap = (size_t)beams->capacity;
  FGA_HIP(copy_planes(beams->f64, cap, f64, (size_t)n, n, FGA_NF64, st));
  FGA_HIP(copy_planes(beams->i32, cap, i32, (size_t)n, n, FGA_NI32, st));
  FGA_HIP(copy_planes(beams->lineage, cap, lineage, (size_t)n, n, 1, st));
  FGA_HIP(hipStreamSynchronize(st));
  beams->count = n;
  return FGA_OK;
}

extern "C" {

const char *fga_last_error(void) { return g_err.c_str(); }

fga_status fga_profile_enable(int on)
{
  prof_clear();
  g_prof_on = on != 0;
  return FGA_OK;
}

fga_status fga_profile_read(int k, int64_t *launches, double *total_ms, int reset)
{
  if (k < 0 || k >= FGA_K_COUNT) return fail(FGA_EINVAL, "unknown kernel id %d", k);
  double tot = 0.0;
  for (auto &p : g_prof[k].ev) {
    FGA_HIP(hipEventSynchronize(p.second));
    float ms = 0.0f;
    FGA_HIP(hipEventElapsedTime(&ms, p.first, p.second));
    tot += ms;
  }
  if (launches) *launches = (int64_t)g_prof[k].ev.size();
  if (total_ms) *total_ms = tot;
  if (reset) {
    for (auto &p : g_prof[k].ev) {
      (void)hipEventDestroy(p.first);
      (void)hipEventDestroy(p.second);
    }
    g_prof[k].ev.clear();
  }
  return FGA_OK;
}
const char *fga_version(void) { return "fga-gfx950 0.1"; }

size_t fga_medium_grid_table_bytes(const int n[3], int two_fields)
{
  if (!n || n[0] < 1 || n[1] < 1 || n[2] < 1) return 0;
  return sizeof(double) * (FGA_GRID_NODE_DOUBLES + 1) * (size_t)n[0] * n[1] * n[2] * (two_fields ? 2 : 1);
}

fga_status fga_medium_grid_build(const int n[3], const double h[3], const double *cp_nodes, const double *cs_nodes,
                                 double *table, void *stream)
{
  if (!n || !h || !cp_nodes || !table) return fail(FGA_EINVAL, "NULL argument");
  for (int d = 0; d < 3; ++d) {
    if (n[d] < 3) return fail(FGA_EINVAL, "grid needs n >= 3 per axis");
    if (!(h[d] > 0)) return fail(FGA_EINVAL, "grid needs h > 0");
  }
  hipStream_t st = (hipStream_t)stream;
  const size_t N = (size_t)n[0] * n[1] * n[2];
  const int nf = cs_nodes ? 2 : 1;
  double *coef = table + (size_t)FGA_GRID_NODE_DOUBLES * N * nf;
  FGA_HIP(launch_grid_build(n, h, cp_nodes, table, st));
  FGA_HIP(launch_spline_coefficients(n, cp_nodes, coef, st));
  if (cs_nodes) {
    FGA_HIP(launch_grid_build(n, h, cs_nodes, table + (size_t)FGA_GRID_NODE_DOUBLES * N, st));
    FGA_HIP(launch_spline_coefficients(n, cs_nodes, coef + N, st));
  }
  return FGA_OK;
}

int64_t fga_decompose_candidates(const fga_mesh *mesh)
{
  if (check_mesh(mesh) != FGA_OK) return -1;
  return decompose_candidates(mesh);
}

size_t fga_decompose_workspace_bytes(const fga_mesh *mesh, int with_g)
{
  if (check_mesh(mesh) != FGA_OK) return 0;
  Arena ar(nullptr, 0);
  size_t need = 0;
  DevMedium dm{};
  fga_beams b{};
  double dummy;
  decompose_impl(dm, mesh, &dummy, with_g ? &dummy : nullptr, &b, ar, nullptr, true, &need);
  return need;
}

fga_status fga_decompose(const fga_medium *med, const fga_mesh *mesh, const double *f, const double *g,
                         fga_beams *beams, void *workspace, size_t workspace_bytes, void *stream)
{
  fga_status s;
  DevMedium dm;
  if ((s = make_dev_medium(med, &dm)) != FGA_OK) return s;
  if ((s = check_mesh(mesh)) != FGA_OK) return s;
  if ((s = check_beams(beams)) != FGA_OK) return s;
  if (!f) return fail(FGA_EINVAL, "f is NULL");
  Arena ar(workspace, workspace_bytes);
  size_t need = 0;
  return decompose_impl(dm, mesh, f, g, beams, ar, (hipStream_t)stream, false, &need);
}

// ------------------------------------------------------------------ evolve --

namespace {

struct EvolvePlan {
  int chunk;
  int64_t batch;
  int nsamp;        // total samples
  int bpb;          // beams per receiver workgroup
  int resort;       // steps between spatial reorderings (0: never)
};

EvolvePlan evolve_plan(const fga_beams *b, int nsteps, const fga_evolve_opts *o, const fga_receivers *r)
{
  EvolvePlan p;
  p.chunk = (o && o->chunk > 0) ? o->chunk : (r ? 16 : 50);
  if (p.chunk > nsteps) p.chunk = nsteps > 0 ? nsteps : 1;
  p.batch = (o && o->batch > 0) ? o->batch : ((int64_t)1 << 22);
  if (p.batch > b->capacity) p.batch = b->capacity > 0 ? b->capacity : 1;
  p.nsamp = r ? nsteps / r->stride : 0;
  p.bpb = r ? points_beams_per_block(p.batch, r->n, (p.chunk + r->stride - 1) / r->stride + 1) : 1024;
  // with receivers: every 32 steps for large sets (the sort's cost wins over
  // lost locality: 36.0 -> 35.6 s on the 49 M-beam workload), every 16 for
  // small ones (serving requests of 0.1-2.5 M beams)
  p.resort = (o && o->resort < 0) ? 0 : ((o && o->resort > 0) ? o->resort : (r ? (b->count >= (1 << 23) ? 32 : 16) : 64));
  if (p.resort > 0 && p.resort < p.chunk) p.resort = p.chunk;
  return p;
}

struct EvolveBufs {
  unsigned long long *ctr = nullptr;
  double *emit = nullptr, *partial = nullptr, *xs = nullptr, *box = nullptr, *xc = nullptr;
  int32_t *perm = nullptr;
  int64_t *blk_extra = nullptr, *blk_off = nullptr, *total = nullptr;  // interface step
  int32_t *cross_list = nullptr, *cross_sorted = nullptr;
  unsigned long long *cross_count = nullptr;
  void *cross_tmp = nullptr;
  size_t cross_tmp_bytes = 0;
};

static EvolveBufs evolve_layout(const EvolvePlan &p, const fga_receivers *r, int64_t cap, Arena &ar)
{
  EvolveBufs b;
  b.ctr = ar.take<unsigned long long>(8);
  const int64_t nblk_all = (cap + 255) / 256 + 1;
  b.blk_extra = ar.take<int64_t>(nblk_all);
  b.blk_off = ar.take<int64_t>(nblk_all);
  b.total = ar.take<int64_t>(1);
  b.cross_list = ar.take<int32_t>(cap + 1);
  b.cross_sorted = ar.take<int32_t>(cap + 1);
  b.cross_count = ar.take<unsigned long long>(1);
  b.cross_tmp_bytes = cross_sort_bytes(cap);
  b.cross_tmp = ar.take<char>(b.cross_tmp_bytes);
  if (r) {
    const int m = (p.chunk + r->stride - 1) / r->stride + 1;
    b.emit = ar.take<double>((size_t)m * 12 * p.batch);
    const int64_t nblk = (p.batch + p.bpb - 1) / p.bpb;
    b.partial = ar.take<double>((size_t)nblk * m * r->n * 6);
    b.box = ar.take<double>((size_t)m * ((p.batch + 63) / 64) * 6);
    b.xs = ar.take<double>((size_t)3 * r->n + 1);
    b.perm = ar.take<int32_t>((size_t)r->n + 1);
    if (r->coords == FGA_COORDS_SPHERICAL) b.xc = ar.take<double>((size_t)3 * r->n + 1);
  }
  return b;
}

}  // namespace

size_t fga_evolve_workspace_bytes(const fga_beams *beams, int nsteps, const fga_evolve_opts *opts,
                                  const fga_receivers *rec)
{
  if (check_beams(beams) != FGA_OK || nsteps < 0) return 0;
  if (rec && rec->stride < 1) return 0;
  const EvolvePlan p = evolve_plan(beams, nsteps, opts, rec);
  Arena ar(nullptr, 0);
  evolve_layout(p, rec, beams->capacity, ar);
  // the re-sort and the compaction work behind the evolution's buffers (the
  // counters among them stay intact), sized for a full beam set: interface
  // splitting can grow it up to capacity
  const size_t base = Arena::need(ar.used);
  size_t need = ar.used;
  fga_beams bb = *beams;
  bb.count = bb.capacity;
  if (p.resort > 0) {
    Arena sa(nullptr, 0);
    size_t ns = 0;
    sort_beams_spatial(&bb, sa, nullptr, true, &ns);
    need = need > base + ns ? need : base + ns;
  }
  if (opts && opts->compact) {
    Arena a2(nullptr, 0);
    size_t n2 = 0;
    compact_beams(&bb, a2, nullptr, true, &n2);
    need = need > base + n2 ? need : base + n2;
  }
  return need;
}

fga_status fga_evolve(const fga_medium *med, fga_beams *beams, double dt, int nsteps, const fga_evolve_opts *opts,
                      const fga_receivers *rec, double *seis, void *workspace, size_t workspace_bytes, void *stream,
                      fga_evolve_stats *stats)
{
  fga_status s;
  DevMedium dm;
  if ((s = make_dev_medium(med, &dm)) != FGA_OK) return s;
  if ((s = check_beams(beams)) != FGA_OK) return s;
  if (nsteps < 0) return fail(FGA_EINVAL, "nsteps < 0");
  if (!(dt > 0) && nsteps > 0) return fail(FGA_EINVAL, "dt must be > 0");
  if (rec) {
    if (rec->stride < 1) return fail(FGA_EINVAL, "receiver stride must be >= 1");
    if (rec->n < 0 || (rec->n > 0 && !rec->xyz)) return fail(FGA_EINVAL, "receiver positions invalid");
    if (!(rec->eps > 0) || !(rec->tau > 0)) return fail(FGA_EINVAL, "receiver eps and tau must be > 0");
    if (!point_precision_ok(rec->precision))
      return fail(FGA_EUNSUPPORTED, "receiver precision %d not built (FGA_FP64, FGA_FP32, FGA_FP32_ACC32)",
                  rec->precision);
    if (!seis && rec->n > 0 && nsteps / rec->stride > 0) return fail(FGA_EINVAL, "seis is NULL");
    if (rec->coords != FGA_COORDS_CARTESIAN && rec->coords != FGA_COORDS_SPHERICAL)
      return fail(FGA_EINVAL, "receiver coords must be FGA_COORDS_CARTESIAN or FGA_COORDS_SPHERICAL");
  }
  const int s_vector = opts && opts->s_vector ? 1 : 0;
  hipStream_t st = (hipStream_t)stream;
  EvolvePlan p = evolve_plan(beams, nsteps, opts, rec);
  // layered media step one step per launch and re-sort a beam set grown by
  // interface children: re-sorting every 64 steps costs less than it saves
  // (152 -> 148 s per step on the layered Earth with 16); the workspace does
  // not depend on the interval
  if (dm.kind == FGA_MEDIUM_LAYERED && p.resort > 0 && !(opts && opts->resort > 0)) p.resort = 64;
  Arena ar(workspace, workspace_bytes);
  const EvolveBufs wb = evolve_layout(p, rec, beams->capacity, ar);
  unsigned long long *ctr = wb.ctr;
  double *emit = wb.emit, *partial = wb.partial;
  if (!ctr || !wb.blk_extra || !wb.blk_off || !wb.total || !wb.cross_list || !wb.cross_sorted ||
      !wb.cross_count || !wb.cross_tmp ||
      (rec && (!emit || !partial || !wb.box || !wb.xs || !wb.perm ||
               (rec->coords == FGA_COORDS_SPHERICAL && !wb.xc))))
    return fail(FGA_ENOMEM, "evolve workspace too small (%zu bytes given, %zu needed)", workspace_bytes, ar.used);
  const size_t sort_base = Arena::need(ar.used);  // re-sort and compaction work here, behind the counters
  const size_t sub_bytes = workspace_bytes > sort_base ? workspace_bytes - sort_base : 0;
  FGA_HIP(hipMemsetAsync(ctr, 0, 8 * sizeof(unsigned long long), st));
  if (rec && rec->n > 0) {
    const double *xyz = rec->xyz;
    if (rec->coords == FGA_COORDS_SPHERICAL) {
      FGA_HIP(launch_spherical_to_cartesian(rec->xyz, rec->n, wb.xc, st));
      xyz = wb.xc;
    }
    if ((s = sort_points(xyz, rec->n, wb.xs, wb.perm, st)) != FGA_OK) return s;
  }

  const double cutoff = opts ? opts->cutoff_abs : 0.0;
  int last_sort = -1;
  if (dm.kind == FGA_MEDIUM_LAYERED) {
    // one step at a time: integrator, interface split, then the sample
    const int gen_max = (opts && opts->gen_max > 0) ? opts->gen_max : 3;
    const double child_cut = (opts && opts->child_cut != 0.0) ? (opts->child_cut < 0.0 ? 0.0 : opts->child_cut) : 1e-3;
    for (int s0 = 0; s0 < nsteps; ++s0) {
      if (p.resort > 0 && (last_sort < 0 || s0 - last_sort >= p.resort)) {
        Arena sa(static_cast<char *>(workspace) + sort_base, sub_bytes);
        size_t need = 0;
        if ((s = sort_beams_spatial(beams, sa, st, false, &need)) != FGA_OK) return s;
        last_sort = s0;
      }
      const int64_t n = beams->count;
      IntegrateArgs a{};
      a.f64 = beams->f64;
      a.i32 = beams->i32;
      a.cap = beams->capacity;
      a.beg = 0;
      a.end = n;
      a.dt = dt;
      a.nsteps = 1;
      a.step0 = s0;
      a.stride = 0;
      a.eps_emit = 1.0;
      a.cutoff_abs = cutoff;
      a.counters = ctr;
      a.s_vector = s_vector;
      FGA_HIP(launch_integrate(dm, a, st));
      InterfaceArgs ia{};
      ia.f64 = beams->f64;
      ia.i32 = beams->i32;
      ia.lineage = beams->lineage;
      ia.cap = beams->capacity;
      ia.n = n;
      ia.dt = dt;
      ia.gen_max = gen_max;
      ia.child_cut = child_cut;
      ia.blk_extra = wb.blk_extra;
      ia.blk_off = wb.blk_off;
      ia.counters = ctr + 4;
      // the crossing beams, in slot order (children slots as if every beam
      // were visited in order)
      int64_t ncross = 0;
      FGA_HIP(collect_crossers(beams->i32 + FGA_FLAGS * beams->capacity, n, wb.cross_list, wb.cross_sorted,
                               wb.cross_count, wb.cross_tmp, wb.cross_tmp_bytes, st, &ncross));
      ia.list = wb.cross_sorted;
      ia.nlist = ncross;
      if (ncross > 0) {
        FGA_HIP(launch_interface(dm, ia, 0, st));
        FGA_HIP(launch_scan(wb.blk_extra, wb.blk_off, (ncross + 255) / 256, wb.total, st));
        int64_t extra = 0;
        FGA_HIP(hipMemcpyAsync(&extra, wb.total, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        FGA_HIP(hipStreamSynchronize(st));
        if (n + extra > beams->capacity)
          return fail(FGA_ECAPACITY, "step %d: %lld beams after interface splitting exceed the capacity %lld", s0,
                      (long long)(n + extra), (long long)beams->capacity);
        FGA_HIP(launch_interface(dm, ia, 1, st));
        beams->count = n + extra;
      }
      if (rec && (s0 + 1) % rec->stride == 0 && rec->n > 0) {
        const int sample = (s0 + 1) / rec->stride - 1;
        const int64_t nb = beams->count;
        if (nb == 0) FGA_HIP(launch_reduce_points(partial, 0, 1, rec->n, wb.perm, seis, p.nsamp, sample, 0, st));
        // one sample per step here: the records, boxes and partials laid out
        // for m samples of p.batch beams hold one sample of m * p.batch beams
        // (with the same beams per workgroup, which depends on beams x samples)
        const int64_t lbatch = p.batch * (int64_t)((p.chunk + rec->stride - 1) / rec->stride + 1);
        for (int64_t b0 = 0; b0 < nb; b0 += lbatch) {
          const int64_t b1 = b0 + lbatch < nb ? b0 + lbatch : nb;
          FGA_HIP(launch_emit(beams->f64, beams->i32, beams->capacity, b0, b1, rec->eps, emit, wb.box, st));
          PointsArgs pa{};
          pa.emit = emit;
          pa.nb = b1 - b0;
          pa.m = 1;
          pa.xyz = wb.xs;
          pa.n = rec->n;
          pa.eps = rec->eps;
          pa.tau = rec->tau;
          pa.partial = partial;
          pa.beams_per_block = p.bpb;
          pa.evals = ctr + 3;
          pa.tile_box = wb.box;
          pa.ntiles = (pa.nb + 63) / 64;
          pa.boxes_ready = 1;
          pa.precision = rec->precision;
          int nblk = 0;
          FGA_HIP(launch_sum_points(pa, &nblk, st));
          FGA_HIP(launch_reduce_points(partial, nblk, 1, rec->n, wb.perm, seis, p.nsamp, sample, b0 > 0 ? 1 : 0, st));
        }
      }
    }
  }
  for (int s0 = 0; s0 < (dm.kind == FGA_MEDIUM_LAYERED ? 0 : nsteps); s0 += p.chunk) {
    if (p.resort > 0 && (last_sort < 0 || s0 - last_sort >= p.resort)) {
      Arena sa(static_cast<char *>(workspace) + sort_base, sub_bytes);
      size_t need = 0;
      if ((s = sort_beams_spatial(beams, sa, st, false, &need)) != FGA_OK) return s;
      last_sort = s0;
    }
    const int64_t n = beams->count;
    const int m = s0 + p.chunk <= nsteps ? p.chunk : nsteps - s0;
    int ns = 0, sfirst = 0;
    if (rec) {
      sfirst = s0 / rec->stride;
      ns = (s0 + m) / rec->stride - sfirst;
    }
    for (int64_t b0 = 0; b0 < n; b0 += (rec && ns > 0) ? p.batch : n) {
      const int64_t b1 = (rec && ns > 0) ? (b0 + p.batch < n ? b0 + p.batch : n) : n;
      IntegrateArgs a{};
      a.f64 = beams->f64;
      a.i32 = beams->i32;
      a.cap = beams->capacity;
      a.beg = b0;
      a.end = b1;
      a.dt = dt;
      a.nsteps = m;
      a.step0 = s0;
      a.stride = (rec && ns > 0) ? rec->stride : 0;
      a.emit = emit;
      a.eps_emit = rec ? rec->eps : 1.0;
      a.cutoff_abs = cutoff;
      a.counters = ctr;
      a.s_vector = s_vector;
      FGA_HIP(launch_integrate(dm, a, st));
      if (rec && ns > 0 && rec->n > 0) {
        PointsArgs pa{};
        pa.emit = emit;
        pa.nb = b1 - b0;
        pa.m = ns;
        pa.xyz = wb.xs;
        pa.n = rec->n;
        pa.eps = rec->eps;
        pa.tau = rec->tau;
        pa.partial = partial;
        pa.beams_per_block = p.bpb;
        pa.evals = ctr + 3;
        pa.tile_box = wb.box;
        pa.ntiles = (pa.nb + 63) / 64;
        pa.precision = rec->precision;
        int nblk = 0;
        FGA_HIP(launch_sum_points(pa, &nblk, st));
        FGA_HIP(launch_reduce_points(partial, nblk, ns, rec->n, wb.perm, seis, p.nsamp, sfirst, b0 > 0 ? 1 : 0,
                                     st));
      }
    }
    if (n == 0 && rec && ns > 0 && rec->n > 0)
      FGA_HIP(launch_reduce_points(partial, 0, ns, rec->n, wb.perm, seis, p.nsamp, sfirst, 0, st));
  }
  if (opts && opts->compact && cutoff > 0 && nsteps > 0) {
    Arena a2(static_cast<char *>(workspace) + sort_base, sub_bytes);
    size_t need = 0;
    if ((s = compact_beams(beams, a2, st, false, &need)) != FGA_OK) return s;
  }
  if (stats || (cutoff > 0 && nsteps > 0)) {
    unsigned long long h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    FGA_HIP(hipMemcpyAsync(h, ctr, sizeof h, hipMemcpyDeviceToHost, st));
    FGA_HIP(hipStreamSynchronize(st));
    if (stats) {
      stats->beam_steps = (int64_t)h[0];
      stats->culled = (int64_t)h[1];
      stats->quarantined = (int64_t)h[2];
      stats->evals = (int64_t)h[3];
      stats->crossings = (int64_t)h[4];
      stats->spawned = (int64_t)h[5];
      stats->capped = (int64_t)h[6];
    }
  }
  return FGA_OK;
}

// ----------------------------------------------------------- reconstruct --

size_t fga_reconstruct_points_workspace_bytes(const fga_beams *beams, int64_t n)
{
  if (check_beams(beams) != FGA_OK || n < 0) return 0;
  const int64_t batch = beams->count < ((int64_t)1 << 22) ? (beams->count > 0 ? beams->count : 1) : ((int64_t)1 << 22);
  Arena ar(nullptr, 0);
  ar.take<unsigned long long>(1);
  ar.take<double>((size_t)12 * batch);
  const int bpb = points_beams_per_block(batch, n, 1);
  ar.take<double>((size_t)((batch + bpb - 1) / bpb) * n * 6);
  ar.take<double>((size_t)((batch + 63) / 64) * 6);
  ar.take<double>((size_t)3 * n + 1);
  ar.take<int32_t>((size_t)n + 1);
  return ar.used;
}

fga_status fga_reconstruct_points(const fga_beams *beams, double eps, double tau, int64_t n, const double *xyz,
                                  int precision, double *out, void *workspace, size_t workspace_bytes, void *stream,
                                  int64_t *evals)
{
  fga_status s;
  if ((s = check_beams(beams)) != FGA_OK) return s;
  if (n < 0 || (n > 0 && (!xyz || !out))) return fail(FGA_EINVAL, "points invalid");
  if (!(eps > 0) || !(tau > 0)) return fail(FGA_EINVAL, "eps and tau must be > 0");
  if (!point_precision_ok(precision))
    return fail(FGA_EUNSUPPORTED, "point precision %d not built (FGA_FP64, FGA_FP32, FGA_FP32_ACC32)", precision);
  hipStream_t st = (hipStream_t)stream;
  const int64_t nb = beams->count;
  const int64_t batch = nb < ((int64_t)1 << 22) ? (nb > 0 ? nb : 1) : ((int64_t)1 << 22);
  Arena ar(workspace, workspace_bytes);
  unsigned long long *ctr = ar.take<unsigned long long>(1);
  double *emit = ar.take<double>((size_t)12 * batch);
  const int bpb = points_beams_per_block(batch, n, 1);
  double *partial = ar.take<double>((size_t)((batch + bpb - 1) / bpb) * n * 6);
  double *box = ar.take<double>((size_t)((batch + 63) / 64) * 6);
  double *xs = ar.take<double>((size_t)3 * n + 1);
  int32_t *perm = ar.take<int32_t>((size_t)n + 1);
  if (!ctr || !emit || !partial || !box || !xs || !perm)
    return fail(FGA_ENOMEM, "reconstruct workspace too small (%zu bytes given, %zu needed)", workspace_bytes, ar.used);
  if (n > 0x7fffffff) return fail(FGA_EUNSUPPORTED, "more than 2^31 points");
  FGA_HIP(hipMemsetAsync(ctr, 0, sizeof(unsigned long long), st));
  if (n > 0 && (s = sort_points(xyz, n, xs, perm, st)) != FGA_OK) return s;
  if (nb == 0) FGA_HIP(launch_reduce_points(partial, 0, 1, n, nullptr, out, 1, 0, 0, st));
  for (int64_t b0 = 0; b0 < nb; b0 += batch) {
    const int64_t b1 = b0 + batch < nb ? b0 + batch : nb;
    FGA_HIP(launch_emit(beams->f64, beams->i32, beams->capacity, b0, b1, eps, emit, box, st));
    PointsArgs pa{};
    pa.emit = emit;
    pa.nb = b1 - b0;
    pa.m = 1;
    pa.xyz = xs;
    pa.n = n;
    pa.eps = eps;
    pa.tau = tau;
    pa.partial = partial;
    pa.beams_per_block = bpb;
    pa.evals = ctr;
    pa.tile_box = box;
    pa.ntiles = (pa.nb + 63) / 64;
    pa.boxes_ready = 1;
    pa.precision = precision;
    int nblk = 0;
    FGA_HIP(launch_sum_points(pa, &nblk, st));
    FGA_HIP(launch_reduce_points(partial, nblk, 1, n, perm, out, 1, 0, b0 > 0 ? 1 : 0, st));
  }
  if (evals) {
    unsigned long long h = 0;
    FGA_HIP(hipMemcpyAsync(&h, ctr, sizeof h, hipMemcpyDeviceToHost, st));
    FGA_HIP(hipStreamSynchronize(st));
    *evals = (int64_t)h;
  }
  return FGA_OK;
}

// ------------------------------------------ points without allocation --

}  // extern "C"

namespace {

// Scratch memory of fga_reconstruct_points_noalloc: one array per device,
// held by the code object until the process ends.  Host code never uses the
// array's name as a device address: the address of each device's copy comes
// from hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
__attribute__((used)) static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

fga_status scratch_of_current_device(char **out)
{
  int dev = -1;
  FGA_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(FGA_EDEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(FGA_EDEVICE, "hipGetSymbolAddress of the scratch array failed on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = static_cast<char *>(g_scratch_ptr[dev]);
  return FGA_OK;
}

__global__ void k_zero_u64(unsigned long long *p, int n)
{
  const int i = threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// Bytes of the no-allocation layout for `batch` beams and n points (the
// carving below in the same order).
size_t noalloc_bytes(int64_t batch, int64_t n)
{
  Arena ar(nullptr, 0);
  ar.take<unsigned long long>(1);
  ar.take<double>((size_t)12 * batch);
  const int bpb = points_beams_per_block(batch, n, 1);
  ar.take<double>((size_t)((batch + bpb - 1) / bpb) * n * 6);
  ar.take<double>((size_t)((batch + 63) / 64) * 6);
  return ar.used;
}

}  // namespace

extern "C" {

size_t fga_reconstruct_points_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

fga_status fga_reconstruct_points_noalloc(const fga_beams *beams, double eps, double tau, int64_t n,
                                          const double *xyz, int precision, double *out, void *stream,
                                          int64_t *evals)
{
  fga_status s;
  if ((s = check_beams(beams)) != FGA_OK) return s;
  if (n < 0 || (n > 0 && (!xyz || !out))) return fail(FGA_EINVAL, "points invalid");
  if (!(eps > 0) || !(tau > 0)) return fail(FGA_EINVAL, "eps and tau must be > 0");
  if (!point_precision_ok(precision))
    return fail(FGA_EUNSUPPORTED, "point precision %d not built (FGA_FP64, FGA_FP32, FGA_FP32_ACC32)", precision);
  if (n > 0x7fffffff) return fail(FGA_EUNSUPPORTED, "more than 2^31 points");
  // beams per batch: the largest whole number of 64-beam tiles (at most 2^22
  // and the set) whose records, boxes and partial sums fit in the scratch
  const int64_t nb = beams->count;
  int64_t batch = nb < ((int64_t)1 << 22) ? ((nb > 0 ? nb : 1) + 63) / 64 * 64 : ((int64_t)1 << 22);
  while (batch > 64 && noalloc_bytes(batch, n) > kNoAllocScratchBytes) batch = (batch / 2 + 63) / 64 * 64;
  if (noalloc_bytes(batch, n) > kNoAllocScratchBytes)
    return fail(FGA_ENOMEM, "%lld points need %zu bytes of scratch even for one 64-beam tile; the no-allocation "
                "call holds %zu (use fga_reconstruct_points)", (long long)n, noalloc_bytes(batch, n),
                kNoAllocScratchBytes);
  char *base = nullptr;
  if ((s = scratch_of_current_device(&base)) != FGA_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  Arena ar(base, kNoAllocScratchBytes);
  unsigned long long *ctr = ar.take<unsigned long long>(1);
  double *emit = ar.take<double>((size_t)12 * batch);
  const int bpb = points_beams_per_block(batch, n, 1);
  double *partial = ar.take<double>((size_t)((batch + bpb - 1) / bpb) * n * 6);
  double *box = ar.take<double>((size_t)((batch + 63) / 64) * 6);
  if (!ctr || !emit || !partial || !box) return fail(FGA_ENOMEM, "scratch layout does not fit");
  hipLaunchKernelGGL(k_zero_u64, 1, 64, 0, st, ctr, 1);
  FGA_HIP(hipGetLastError());
  if (nb == 0) FGA_HIP(launch_reduce_points(partial, 0, 1, n, nullptr, out, 1, 0, 0, st));
  for (int64_t b0 = 0; b0 < nb; b0 += batch) {
    const int64_t b1 = b0 + batch < nb ? b0 + batch : nb;
    FGA_HIP(launch_emit(beams->f64, beams->i32, beams->capacity, b0, b1, eps, emit, box, st));
    PointsArgs pa{};
    pa.emit = emit;
    pa.nb = b1 - b0;
    pa.m = 1;
    pa.xyz = xyz;
    pa.n = n;
    pa.eps = eps;
    pa.tau = tau;
    pa.partial = partial;
    pa.beams_per_block = bpb;
    pa.evals = ctr;
    pa.tile_box = box;
    pa.ntiles = (pa.nb + 63) / 64;
    pa.boxes_ready = 1;
    pa.precision = precision;
    int nblk = 0;
    FGA_HIP(launch_sum_points(pa, &nblk, st));
    FGA_HIP(launch_reduce_points(partial, nblk, 1, n, nullptr, out, 1, 0, b0 > 0 ? 1 : 0, st));
  }
  if (evals) {
    unsigned long long h = 0;
    FGA_HIP(hipMemcpyAsync(&h, ctr, sizeof h, hipMemcpyDeviceToHost, st));
    FGA_HIP(hipStreamSynchronize(st));
    *evals = (int64_t)h;
  }
  return FGA_OK;
}

size_t fga_reconstruct_grid_workspace_bytes(const fga_beams *beams, const int n[3], double eps, double tau,
                                            const double h[3])
{
  if (check_beams(beams) != FGA_OK || !n || !h) return 0;
  const double lo[3] = {0, 0, 0};
  Arena ar(nullptr, 0);
  size_t need = 0;
  grid_sum_impl(beams, eps, tau, n, lo, h, FGA_FP64, nullptr, ar, nullptr, true, &need, nullptr);
  return need;
}

static fga_status reconstruct_grid(const fga_beams *beams, double eps, double tau, const int n[3],
                                   const double lo[3], const double h[3], int precision, double *out,
                                   void *workspace, size_t workspace_bytes, void *stream, int64_t *evals, bool add)
{
  fga_status s;
  if ((s = check_beams(beams)) != FGA_OK) return s;
  if (!n || !lo || !h || !out) return fail(FGA_EINVAL, "NULL grid argument");
  for (int d = 0; d < 3; ++d) {
    if (n[d] < 1) return fail(FGA_EINVAL, "grid sizes must be >= 1");
    if (!(h[d] > 0)) return fail(FGA_EINVAL, "grid spacing must be > 0");
  }
  if (!(eps > 0) || !(tau > 0)) return fail(FGA_EINVAL, "eps and tau must be > 0");
  Arena ar(workspace, workspace_bytes);
  size_t need = 0;
  return grid_sum_impl(beams, eps, tau, n, lo, h, precision, out, ar, (hipStream_t)stream, false, &need, evals,
                       add);
}

fga_status fga_reconstruct_grid(const fga_beams *beams, double eps, double tau, const int n[3], const double lo[3],
                                const double h[3], int precision, double *out, void *workspace,
                                size_t workspace_bytes, void *stream, int64_t *evals)
{
  return reconstruct_grid(beams, eps, tau, n, lo, h, precision, out, workspace, workspace_bytes, stream, evals,
                          false);
}

fga_status fga_reconstruct_grid_add(const fga_beams *beams, double eps, double tau, const int n[3],
                                    const double lo[3], const double h[3], int precision, double *out,
                                    void *workspace, size_t workspace_bytes, void *stream, int64_t *evals)
{
  return reconstruct_grid(beams, eps, tau, n, lo, h, precision, out, workspace, workspace_bytes, stream, evals,
                          true);
}

}  // extern "C"
