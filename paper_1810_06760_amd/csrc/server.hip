// Request server for many forward solves on one GPU (tomography sweeps).
//
// Requests (initial data + receivers on a resident velocity model) queue on
// the host.  The server holds one device pool of the budget's size, taken
// once at creation; a request's buffers (beams, workspace, inputs,
// seismograms) are one block of that pool, found first-fit, so a solve never
// calls hipMalloc or hipFree (hipFree would synchronise the whole device and
// stall the other slots).  A fixed set of slots, each a host thread with its
// own HIP stream, takes the first queued request whose block fits in the pool
// next to the running ones; a slot runs its request to completion (decompose
// -> evolve with receiver sums -> seismograms to host), returns the block, and
// the next request is admitted as soon as a slot and a block are free.
// Running requests overlap on the device through their separate streams.
// Every solve is deterministic and uses only its own block, so a result is
// the same alone or in a mix.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "fga_internal.h"

namespace {

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct Sizes {
  int64_t capacity, ns;
  size_t beams, f, rec, seis, ws, total;
};

bool request_sizes(const fga_request *r, Sizes *z)
{
  if (!r || r->nsteps < 0 || r->stride < 1 || r->n_receivers < 0) return false;
  if (r->precision != FGA_FP64 && r->precision != FGA_FP32 && r->precision != FGA_FP32_ACC32) return false;
  if (r->receiver_coords != FGA_COORDS_CARTESIAN && r->receiver_coords != FGA_COORDS_SPHERICAL) return false;
  const int64_t cand = r->point_source ? fga_point_source_candidates(&r->source) : fga_decompose_candidates(&r->mesh);
  if (cand <= 0) return false;
  // layered media grow the beam set at interfaces
  z->capacity = r->medium.kind == FGA_MEDIUM_LAYERED ? 4 * cand : cand;
  z->ns = r->nsteps / r->stride;
  const int64_t ny = r->point_source ? 1 : (int64_t)r->mesh.ny[0] * r->mesh.ny[1] * r->mesh.ny[2];
  z->beams = align256((size_t)z->capacity * FGA_NF64 * sizeof(double)) +
             align256((size_t)z->capacity * FGA_NI32 * sizeof(int32_t)) + align256((size_t)z->capacity * sizeof(int64_t));
  z->f = align256((size_t)ny * 3 * 2 * sizeof(double));
  z->rec = align256((size_t)(r->n_receivers > 0 ? r->n_receivers : 1) * 3 * sizeof(double));
  z->seis = align256((size_t)(r->n_receivers > 0 ? r->n_receivers : 1) * (z->ns > 0 ? z->ns : 1) * 6 * sizeof(double));
  fga_beams b{};
  b.capacity = z->capacity;
  b.count = z->capacity;
  b.f64 = reinterpret_cast<double *>(256);  // placeholders: sizing only
  b.i32 = reinterpret_cast<int32_t *>(256);
  b.lineage = reinterpret_cast<int64_t *>(256);
  fga_receivers rc{};
  rc.n = r->n_receivers;
  rc.xyz = reinterpret_cast<const double *>(256);
  rc.stride = r->stride;
  rc.eps = r->point_source ? r->source.eps : r->mesh.eps;
  rc.tau = r->tau;
  rc.precision = r->precision;
  rc.coords = r->receiver_coords;
  const size_t wd = r->point_source ? fga_decompose_point_source_workspace_bytes(&r->source)
                                    : fga_decompose_workspace_bytes(&r->mesh, 0);
  const size_t we = fga_evolve_workspace_bytes(&b, r->nsteps, nullptr, r->n_receivers > 0 ? &rc : nullptr);
  z->ws = align256(wd > we ? wd : we);
  z->total = z->beams + z->f + z->rec + z->seis + z->ws;
  return wd > 0 && we > 0;
}

double now_s(std::chrono::steady_clock::time_point t0)
{
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

struct Job {
  uint64_t id;
  fga_request req;
  std::vector<double> f, rec;
  Sizes sz;
  double t_submit;
  size_t off = 0;  // the request's block in the pool
};

// First-fit allocator of 256-byte-aligned blocks in [0, size), free blocks
// coalesced with their neighbours on release (host bookkeeping only).
class BlockPool {
 public:
  void reset(size_t size)
  {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool take(size_t n, size_t *off)
  {
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n;
        const size_t at = it->first + n;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    return false;
  }
  void give(size_t off, size_t n)
  {
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;  // offset -> length
};

}  // namespace

struct fga_server {
  int device = 0;
  size_t budget = 0;
  char *pool = nullptr;  // device, `budget` bytes
  BlockPool blocks;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job> queue;
  std::deque<fga_completion> done;
  std::vector<std::thread> slots;
  size_t held = 0;
  int running = 0, peak = 0;
  uint64_t next_id = 1;
  bool closing = false;

  void slot_main();
  fga_completion run(Job &j, hipStream_t st);
};

fga_completion fga_server::run(Job &j, hipStream_t st)
{
  fga_completion c{};
  c.id = j.id;
  c.t_submit = j.t_submit;
  c.t_start = now_s(t0);
  c.footprint = j.sz.total;
  const fga_request &r = j.req;
  fga_status s = FGA_OK;
  char *p = pool + j.off;
  fga_beams b{};
  b.capacity = j.sz.capacity;
  b.count = 0;
  b.f64 = reinterpret_cast<double *>(p);
  p += align256((size_t)b.capacity * FGA_NF64 * sizeof(double));
  b.i32 = reinterpret_cast<int32_t *>(p);
  p += align256((size_t)b.capacity * FGA_NI32 * sizeof(int32_t));
  b.lineage = reinterpret_cast<int64_t *>(p);
  p += align256((size_t)b.capacity * sizeof(int64_t));
  double *fd = reinterpret_cast<double *>(p);
  p += j.sz.f;
  double *xd = reinterpret_cast<double *>(p);
  p += j.sz.rec;
  double *sd = reinterpret_cast<double *>(p);
  p += j.sz.seis;
  void *ws = p;
  do {
    if ((!r.point_source &&
         hipMemcpyAsync(fd, j.f.data(), j.f.size() * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess) ||
        (r.n_receivers > 0 &&
         hipMemcpyAsync(xd, j.rec.data(), j.rec.size() * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess)) {
      s = FGA_EDEVICE;
      break;
    }
    s = r.point_source ? fga_decompose_point_source(&r.medium, &r.source, &b, ws, j.sz.ws, st)
                       : fga_decompose(&r.medium, &r.mesh, fd, nullptr, &b, ws, j.sz.ws, st);
    if (s != FGA_OK) break;
    c.beams = b.count;
    fga_receivers rc{};
    rc.n = r.n_receivers;
    rc.xyz = xd;
    rc.stride = r.stride;
    rc.eps = r.point_source ? r.source.eps : r.mesh.eps;
    rc.tau = r.tau;
    rc.precision = r.precision;
    rc.coords = r.receiver_coords;
    fga_evolve_stats es{};
    if ((s = fga_evolve(&r.medium, &b, r.dt, r.nsteps, nullptr, r.n_receivers > 0 ? &rc : nullptr, sd, ws, j.sz.ws,
                        st, &es)) != FGA_OK)
      break;
    c.beam_steps = es.beam_steps;
    c.evals = es.evals;
    if (r.n_receivers > 0 && j.sz.ns > 0 &&
        hipMemcpyAsync(r.seis_out, sd, (size_t)r.n_receivers * j.sz.ns * 6 * sizeof(double), hipMemcpyDeviceToHost,
                       st) != hipSuccess) {
      s = FGA_EDEVICE;
      break;
    }
    if (hipStreamSynchronize(st) != hipSuccess) s = FGA_EDEVICE;
  } while (false);
  (void)hipStreamSynchronize(st);
  c.status = s;
  c.t_done = now_s(t0);
  return c;
}

void fga_server::slot_main()
{
  (void)hipSetDevice(device);
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
  for (;;) {
    Job j;
    {
      std::unique_lock<std::mutex> lk(mu);
      for (;;) {
        // first queued request whose block fits in the pool next to the running ones
        auto it = queue.begin();
        size_t off = 0;
        for (; it != queue.end(); ++it)
          if (blocks.take(it->sz.total, &off)) break;
        if (it != queue.end()) {
          j = std::move(*it);
          j.off = off;
          queue.erase(it);
          held += j.sz.total;
          ++running;
          if (running > peak) peak = running;
          break;
        }
        if (closing && queue.empty()) {
          if (st) (void)hipStreamDestroy(st);
          return;
        }
        cv_work.wait(lk);
      }
    }
    fga_completion c = st ? run(j, st) : fga_completion{};
    if (!st) {
      c.id = j.id;
      c.status = FGA_EDEVICE;
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      blocks.give(j.off, j.sz.total);
      held -= j.sz.total;
      --running;
      done.push_back(c);
    }
    cv_work.notify_all();
    cv_done.notify_all();
  }
}

extern "C" {

size_t fga_server_footprint(const fga_request *r)
{
  Sizes z;
  return request_sizes(r, &z) ? z.total : 0;
}

fga_status fga_server_create(size_t hbm_budget, int max_active, fga_server **out)
{
  if (!out || max_active < 1) return fga::fail(FGA_EINVAL, "server needs max_active >= 1 and an output pointer");
  fga_server *s = new fga_server();
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return fga::fail(FGA_EDEVICE, "no current HIP device");
  }
  s->budget = hbm_budget & ~size_t(255);  // footprints are multiples of 256 bytes
  if (s->budget == 0 || hipMalloc(&s->pool, s->budget) != hipSuccess) {
    (void)hipGetLastError();
    delete s;
    return fga::fail(FGA_ENOMEM, "cannot hold a device pool of %zu bytes for the server budget", hbm_budget);
  }
  s->blocks.reset(s->budget);
  s->t0 = std::chrono::steady_clock::now();
  for (int k = 0; k < max_active; ++k) s->slots.emplace_back([s] { s->slot_main(); });
  *out = s;
  return FGA_OK;
}

fga_status fga_server_submit(fga_server *s, const fga_request *r, uint64_t *id)
{
  if (!s || !r) return fga::fail(FGA_EINVAL, "server or request is NULL");
  Sizes z;
  if (!request_sizes(r, &z)) return fga::fail(FGA_EINVAL, "invalid request (mesh, steps, stride or receivers)");
  if ((!r->point_source && !r->f) || (r->n_receivers > 0 && (!r->receivers || (z.ns > 0 && !r->seis_out))))
    return fga::fail(FGA_EINVAL, "request has a NULL f, receivers or seis_out");
  if (z.total > s->budget)
    return fga::fail(FGA_ECAPACITY, "request needs %zu device bytes, above the server budget %zu", z.total, s->budget);
  Job j;
  j.req = *r;
  if (!r->point_source) {
    const int64_t ny = (int64_t)r->mesh.ny[0] * r->mesh.ny[1] * r->mesh.ny[2];
    j.f.assign(r->f, r->f + ny * 6);
  }
  if (r->n_receivers > 0) j.rec.assign(r->receivers, r->receivers + r->n_receivers * 3);
  j.sz = z;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->closing) return fga::fail(FGA_EINVAL, "server is shutting down");
    j.id = s->next_id++;
    j.t_submit = now_s(s->t0);
    if (id) *id = j.id;
    s->queue.push_back(std::move(j));
  }
  s->cv_work.notify_all();
  return FGA_OK;
}

fga_status fga_server_poll(fga_server *s, fga_completion *out, int max, int *n, int wait_ms)
{
  if (!s || !n || (max > 0 && !out)) return fga::fail(FGA_EINVAL, "poll arguments invalid");
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && wait_ms > 0)
    s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [s] { return !s->done.empty(); });
  int k = 0;
  while (k < max && !s->done.empty()) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  *n = k;
  return FGA_OK;
}

fga_status fga_server_status(fga_server *s, int *queued, int *running, size_t *held, int *peak_running)
{
  if (!s) return fga::fail(FGA_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  if (queued) *queued = (int)s->queue.size();
  if (running) *running = s->running;
  if (held) *held = s->held;
  if (peak_running) *peak_running = s->peak;
  return FGA_OK;
}

fga_status fga_server_destroy(fga_server *s)
{
  if (!s) return FGA_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->closing = true;
  }
  s->cv_work.notify_all();
  for (auto &t : s->slots) t.join();
  // every slot has synchronised its stream after its last solve
  if (s->pool) (void)hipFree(s->pool);
  delete s;
  return FGA_OK;
}

}  // extern "C"
