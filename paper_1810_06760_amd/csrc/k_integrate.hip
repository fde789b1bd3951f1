// One-thread-per-beam FP64 integrator of the FGA ODE system on gfx950.
//
// Each thread loads one beam's 47-double state from the structure-of-arrays
// planes (coalesced), advances it by `nsteps` classic RK4 steps held entirely
// in registers, optionally writes an emission record (Q, P, w e^{iS/eps} A)
// after every sample step for the receiver summation, and stores the state
// back (the right-hand side and the RK4 step are in rk4.h).  Layered media
// have a one-step kernel of their own (k_step_layered): there a beam whose
// centre leaves its layer during the step keeps its stored state and is
// flagged for the interface step.
#include "fastmath.h"
#include "rk4.h"

namespace fga {
namespace {

using namespace rk;

// Emission record of the current state: Q (3), P 128/(pi eps) (3), B = w e^{iS/eps} A (3 complex).
// SV = 1: an S beam's state holds A itself (frame-free form).
template <int SV = 0>
__device__ __forceinline__ void emit_record(double *__restrict__ out, int64_t nb, int64_t j,
                                            const double *y, const double e[3], double wr, double wi,
                                            bool isS, double ieps)
{
  double A[6];
  if (SV && isS) {
    A[0] = y[IA];
    A[1] = y[IA + 1];
    A[2] = y[IA + 2];
    A[3] = y[IA + 3];
    A[4] = y[IAZ];
    A[5] = y[IAZ + 1];
  } else if (!isS) {
    const double inp = 1.0 / sqrt(y[IP] * y[IP] + y[IP + 1] * y[IP + 1] + y[IP + 2] * y[IP + 2]);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double nh = y[IP + c] * inp;
      A[2 * c] = y[IA] * nh;
      A[2 * c + 1] = y[IA + 1] * nh;
    }
  } else {
    double nsh[3], nsv[3];
    s_frame(y + IP, e, nsh, nsv);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      A[2 * c] = y[IA] * nsv[c] + y[IA + 2] * nsh[c];
      A[2 * c + 1] = y[IA + 1] * nsv[c] + y[IA + 3] * nsh[c];
    }
  }
  double sn, cs;
  sincos(y[IS] * ieps, &sn, &cs);
  const double Wr = wr * cs - wi * sn, Wi = wr * sn + wi * cs;
  const double pscale = ieps * INV_PI_128;
  double r[12];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    r[f] = y[IQ + f];
    r[3 + f] = y[IP + f] * pscale;  // the phase (P/eps).(x - Q) in units of pi/128
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    r[6 + 2 * c] = Wr * A[2 * c] - Wi * A[2 * c + 1];
    r[7 + 2 * c] = Wr * A[2 * c + 1] + Wi * A[2 * c];
  }
  // a record with a non-finite entry is written as a dead one: it never
  // enters a window, so no sum takes a NaN from it
  bool finite = true;
#pragma unroll
  for (int f = 0; f < 12; ++f) finite = finite && isfinite(r[f]);
#pragma unroll
  for (int f = 0; f < 12; ++f) out[f * nb + j] = finite ? r[f] : (f < 3 ? -1.0e300 : 0.0);
}

__device__ __forceinline__ void emit_dead(double *__restrict__ out, int64_t nb, int64_t j)
{
  // dead beams sit at -1e300 (idle point lanes use +1e300), never in any window
#pragma unroll
  for (int f = 0; f < 3; ++f) out[f * nb + j] = -1.0e300;
#pragma unroll
  for (int f = 3; f < 12; ++f) out[f * nb + j] = 0.0;
}

// Whether the quantities a step's sample is formed from (Q, P, the
// amplitudes and S) are finite.
template <int SV = 0>
__device__ __forceinline__ bool emitted_finite(const double *y)
{
  bool ok = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) ok = ok && isfinite(y[IQ + d]) && isfinite(y[IP + d]);
#pragma unroll
  for (int t = 0; t < 4; ++t) ok = ok && isfinite(y[IA + t]);
  if (SV) ok = ok && isfinite(y[IAZ]) && isfinite(y[IAZ + 1]);
  return ok && isfinite(y[IS]);
}

// Frame-free S amplitudes: (a_SV, a_SH) in the beam's frame -> A in y, and back.
__device__ __forceinline__ void frame_to_vector(double *y, const double e[3])
{
  double nsh[3], nsv[3];
  s_frame(y + IP, e, nsh, nsv);
  const double a0r = y[IA], a0i = y[IA + 1], a1r = y[IA + 2], a1i = y[IA + 3];
  y[IA] = a0r * nsv[0] + a1r * nsh[0];
  y[IA + 1] = a0i * nsv[0] + a1i * nsh[0];
  y[IA + 2] = a0r * nsv[1] + a1r * nsh[1];
  y[IA + 3] = a0i * nsv[1] + a1i * nsh[1];
  y[IAZ] = a0r * nsv[2] + a1r * nsh[2];
  y[IAZ + 1] = a0i * nsv[2] + a1i * nsh[2];
}

// Back to the frame: the axis switched first if P has come within 10 degrees
// of it (the rule of reframe_s), then (a_SV, a_SH) = (A . N_SV, A . N_SH).
__device__ __forceinline__ void vector_to_frame(double *y, double e[3])
{
  const double np = sqrt(y[IP] * y[IP] + y[IP + 1] * y[IP + 1] + y[IP + 2] * y[IP + 2]);
  const double pe = y[IP] * e[0] + y[IP + 1] * e[1] + y[IP + 2] * e[2];
  if (fabs(pe) / np > COS10) {
    const bool was_z = e[2] != 0.0 && e[0] == 0.0 && e[1] == 0.0;
    e[0] = was_z ? 1.0 : 0.0;
    e[1] = 0.0;
    e[2] = was_z ? 0.0 : 1.0;
  }
  double nsh[3], nsv[3];
  s_frame(y + IP, e, nsh, nsv);
  const double Ar[3] = {y[IA], y[IA + 2], y[IAZ]}, Ai[3] = {y[IA + 1], y[IA + 3], y[IAZ + 1]};
  y[IA] = Ar[0] * nsv[0] + Ar[1] * nsv[1] + Ar[2] * nsv[2];
  y[IA + 1] = Ai[0] * nsv[0] + Ai[1] * nsv[1] + Ai[2] * nsv[2];
  y[IA + 2] = Ar[0] * nsh[0] + Ar[1] * nsh[1] + Ar[2] * nsh[2];
  y[IA + 3] = Ai[0] * nsh[0] + Ai[1] * nsh[1] + Ai[2] * nsh[2];
}

template <int MK, int SV = 0>
__device__ __forceinline__ void integrate_body(const DevMedium &med, const IntegrateArgs &a)
{
  const int64_t i = a.beg + (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool active = i < a.end;
  unsigned long long steps_done = 0, culled = 0, quar = 0;
  // Grid media: the workgroup's beams are neighbours in Morton order, so the
  // nodes they interpolate from for the whole launch mostly lie in one small
  // block around them; that block is staged in LDS once and the trilinear
  // gathers read it (cells outside it fall back to global memory).
  MedBlock blk{nullptr, {0, 0, 0}};
  if constexpr (MK == MK_GRID) {
    __shared__ double lds_med[MEDBLK * MEDBLK * MEDBLK * 10];
    __shared__ int bb[6];
    if (!med.two_fields) {
      if (threadIdx.x < 3) {
        bb[threadIdx.x] = 0x7fffffff;
        bb[3 + threadIdx.x] = -0x7fffffff;
      }
      __syncthreads();
      if (active && (a.i32[FGA_FLAGS * a.cap + i] & FGA_FLAG_ALIVE)) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const double u = (a.f64[(FGA_Q + d) * a.cap + i] - med.lo[d]) * med.ih[d];
          const int cell = (int)fmax(fmin(floor(u), 1.0e9), -1.0e9);
          atomicMin(&bb[d], cell);
          atomicMax(&bb[3 + d], cell);
        }
      }
      __syncthreads();
      if (bb[0] <= bb[3]) {
        int o[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const int c0 = bb[d] / 2 + bb[3 + d] / 2 - MEDBLK / 2 + 1;
          o[d] = ((c0 % med.n[d]) + med.n[d]) % med.n[d];
        }
        for (int idx = threadIdx.x; idx < MEDBLK * MEDBLK * MEDBLK; idx += 256) {
          const int lx = idx % MEDBLK, ly = (idx / MEDBLK) % MEDBLK, lz = idx / (MEDBLK * MEDBLK);
          const int nx = (o[0] + lx) % med.n[0], ny = (o[1] + ly) % med.n[1], nz = (o[2] + lz) % med.n[2];
          const double *src =
              med.table + (size_t)FGA_GRID_NODE_DOUBLES * (((size_t)nz * med.n[1] + ny) * med.n[0] + nx);
#pragma unroll
          for (int f = 0; f < 10; ++f) lds_med[10 * idx + f] = src[f];
        }
        __syncthreads();
        blk.lds = lds_med;
        blk.o[0] = o[0];
        blk.o[1] = o[1];
        blk.o[2] = o[2];
      }
    }
  }
  if constexpr (MK == MK_GRID3) {
    // the same for the cubic stencils: a MEDBLK3^3 block of spline coefficients
    // (both node fields when there are two) around the beams' cells
    constexpr int B3 = MEDBLK3 * MEDBLK3 * MEDBLK3;
    __shared__ double lds_cf[2 * B3];
    __shared__ int bb[6];
    if (threadIdx.x < 3) {
      bb[threadIdx.x] = 0x7fffffff;
      bb[3 + threadIdx.x] = -0x7fffffff;
    }
    __syncthreads();
    if (active && (a.i32[FGA_FLAGS * a.cap + i] & FGA_FLAG_ALIVE)) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double u = (a.f64[(FGA_Q + d) * a.cap + i] - med.lo[d]) * med.ih[d];
        const int cell = (int)fmax(fmin(floor(u), 1.0e9), -1.0e9);
        atomicMin(&bb[d], cell);
        atomicMax(&bb[3 + d], cell);
      }
    }
    __syncthreads();
    if (bb[0] <= bb[3]) {
      int o[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int c0 = bb[d] / 2 + bb[3 + d] / 2 - MEDBLK3 / 2 + 1;
        o[d] = ((c0 % med.n[d]) + med.n[d]) % med.n[d];
      }
      const int nf = med.two_fields ? 2 : 1;
      for (int idx = threadIdx.x; idx < nf * B3; idx += 256) {
        const int f = idx / B3, r = idx - f * B3;
        const int lx = r % MEDBLK3, ly = (r / MEDBLK3) % MEDBLK3, lz = r / (MEDBLK3 * MEDBLK3);
        const int nx = (o[0] + lx) % med.n[0], ny = (o[1] + ly) % med.n[1], nz = (o[2] + lz) % med.n[2];
        lds_cf[idx] = med.coef[f * med.coef_stride + ((int64_t)nz * med.n[1] + ny) * med.n[0] + nx];
      }
      __syncthreads();
      blk.lds = lds_cf;
      blk.o[0] = o[0];
      blk.o[1] = o[1];
      blk.o[2] = o[2];
    }
  }
  if (active) {
    const int64_t cap = a.cap;
    const int64_t nb = a.end - a.beg;
    const int64_t j = i - a.beg;
    double *__restrict__ F = a.f64;
    int32_t flags = a.i32[FGA_FLAGS * cap + i];
    const int first_emit = a.stride ? a.step0 / a.stride : 0;
    if (!(flags & FGA_FLAG_ALIVE)) {
      if (a.stride)
        for (int s = 0; s < a.nsteps; ++s)
          if ((a.step0 + s + 1) % a.stride == 0)
            emit_dead(a.emit + (int64_t)((a.step0 + s + 1) / a.stride - 1 - first_emit) * 12 * nb, nb, j);
    } else {
      const int br = a.i32[FGA_BRANCH * cap + i];
      const double sg = (double)a.i32[FGA_SIGMA * cap + i];
      const int layer = a.i32[FGA_LAYER * cap + i];
      const int sp = br == 0 ? 0 : 1;
      const bool isS = br != 0;
      double y[nstate<SV>()];
#pragma unroll
      for (int f = 0; f < NS; ++f) y[f] = F[f * cap + i];
      double e[3] = {F[(FGA_E + 0) * cap + i], F[(FGA_E + 1) * cap + i], F[(FGA_E + 2) * cap + i]};
      if (SV) {
        y[nstate<SV>() - 2] = 0.0;
        y[nstate<SV>() - 1] = 0.0;
        if (isS) frame_to_vector(y, e);
      }
      const double wr = F[FGA_W_RE * cap + i], wi = F[FGA_W_IM * cap + i];
      const double dt = a.dt;
      const double ieps = 1.0 / a.eps_emit;
      const double wabs = sqrt(wr * wr + wi * wi);
      // After every step: a beam whose sampled quantities are no longer finite
      // is quarantined, and one with |w| max|a| below the cutoff is dropped;
      // either stops stepping and emits dead records from that step's sample on.
      bool live = isfinite(wabs) && isfinite(e[0]) && isfinite(e[1]) && isfinite(e[2]);
      if (!live) {
        flags = FGA_FLAG_QUARANTINED;
        quar = 1;
      }
      for (int s = 0; s < a.nsteps; ++s) {
        if (live) {
          if constexpr (MK == MK_GRID || MK == MK_GRID3) rk4_step<MK, SV>(med, sp, layer, sg, isS, e, y, dt, &blk);
          else rk4_step_pc<MK>(med, sp, layer, sg, isS, y, dt);  // grad c = 0
          if (isS && !SV) reframe_s(y, e);
          ++steps_done;
          if (!emitted_finite<SV>(y)) {
            live = false;
            flags = FGA_FLAG_QUARANTINED;
            quar = 1;
          } else if (a.cutoff_abs > 0.0) {
            const double m0 = y[IA] * y[IA] + y[IA + 1] * y[IA + 1];
            double m1 = y[IA + 2] * y[IA + 2] + y[IA + 3] * y[IA + 3];
            // frame-free S: the magnitude of the polarisation vector
            const double mm = (SV && isS) ? m0 + m1 + y[nstate<SV>() - 2] * y[nstate<SV>() - 2] +
                                                y[nstate<SV>() - 1] * y[nstate<SV>() - 1]
                                          : (m0 > m1 ? m0 : m1);
            if (wabs * sqrt(mm) < a.cutoff_abs) {
              live = false;
              flags = 0;
              culled = 1;
            }
          }
        }
        if (a.stride && (a.step0 + s + 1) % a.stride == 0) {
          double *rec = a.emit + (int64_t)((a.step0 + s + 1) / a.stride - 1 - first_emit) * 12 * nb;
          if (live) emit_record<SV>(rec, nb, j, y, e, wr, wi, isS, ieps);
          else emit_dead(rec, nb, j);
        }
      }
      {
      if (SV && isS) vector_to_frame(y, e);
      if (live) {
        bool finite = true;
#pragma unroll
        for (int f = 0; f < NS; ++f) finite = finite && isfinite(y[f]);
        if (!finite) {
          flags = FGA_FLAG_QUARANTINED;
          quar = 1;
        }
      }
      // where grad c = 0 the step leaves P and dzP as they were: not stored
#pragma unroll
      for (int f = 0; f < NS; ++f)
        if (MK == MK_GRID || MK == MK_GRID3 || !((f >= IP && f < IP + 3) || (f >= IZPR && f < IZPR + 18)))
          F[f * cap + i] = y[f];
#pragma unroll
      for (int d = 0; d < 3; ++d) F[(FGA_E + d) * cap + i] = e[d];
      a.i32[FGA_FLAGS * cap + i] = flags;
      }
    }
  }
  // wavefront-level reduction of the counters, one atomic per wavefront
  for (int off = 32; off > 0; off >>= 1) {
    steps_done += __shfl_down(steps_done, off);
    culled += __shfl_down(culled, off);
    quar += __shfl_down(quar, off);
  }
  if ((threadIdx.x & 63) == 0 && a.counters) {
    if (steps_done) atomicAdd(a.counters + 0, steps_done);
    if (culled) atomicAdd(a.counters + 1, culled);
    if (quar) atomicAdd(a.counters + 2, quar);
  }
}

template <int MK, int SV = 0>
__global__ __launch_bounds__(256) void k_integrate(DevMedium med, IntegrateArgs a)
{
  integrate_body<MK, SV>(med, a);
}

// One step of every beam in a layered medium, the interface step's cadence
// (no emission).  The same arithmetic as the general kernel with
// rk4_step_pc, ordered so that little stays live: the ray (Q, S) advances
// first and a beam leaving its layer stops there, flagged, with its stored
// state untouched; otherwise Q, S and dzQ are stored as soon as they are
// formed, dzP enters only through Z0 = dzQ + i dzP and K = d(dzQ)/dt, and P
// and dzP are not stored (unchanged by the step).  That fits two wavefronts
// per SIMD, so one wavefront's loads overlap another's arithmetic.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_step_layered(DevMedium med,
                                                                                                 IntegrateArgs a)
{
  const int64_t i = a.beg + (int64_t)blockIdx.x * 256 + threadIdx.x;
  unsigned long long steps_done = 0, culled = 0, quar = 0;
  if (i < a.end) {
    const int64_t cap = a.cap;
    double *__restrict__ F = a.f64;
    int32_t flags = a.i32[FGA_FLAGS * cap + i];
    const int br = a.i32[FGA_BRANCH * cap + i];
    const int sgi = a.i32[FGA_SIGMA * cap + i];
    const int layer = a.i32[FGA_LAYER * cap + i];
    if (flags & FGA_FLAG_ALIVE) {
      steps_done = 1;
      const double sg = (double)sgi;
      const bool isS = br != 0;
      const double dt = a.dt, h6 = dt / 6.0;
      // all of the state, and the layer's speed and bounding interfaces, are
      // requested at once (one memory latency per beam)
      const double c = isS ? med.csl[layer] : med.cpl[layer];
      const double b_in = med.bound[layer], b_out = med.bound[layer > 0 ? layer - 1 : 0];
      double Q[3], P[3], e[3], A[4], qr[9], qi[9], pr[9], pi[9];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        Q[d] = F[(FGA_Q + d) * cap + i];
        P[d] = F[(FGA_P + d) * cap + i];
      }
      const double S = F[FGA_S * cap + i];
#pragma unroll
      for (int o = 0; o < 9; ++o) {
        qr[o] = F[(FGA_ZQ_RE + o) * cap + i];
        qi[o] = F[(FGA_ZQ_IM + o) * cap + i];
        pr[o] = F[(FGA_ZP_RE + o) * cap + i];
        pi[o] = F[(FGA_ZP_IM + o) * cap + i];
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) A[t] = F[(FGA_A0_RE + t) * cap + i];
#pragma unroll
      for (int d = 0; d < 3; ++d) e[d] = F[(FGA_E + d) * cap + i];
      double kQ[3], kS, ph[3], ci;
      pc_ray_rates(c, sg, P, kQ, kS, ph, ci);
      double Qn[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) Qn[d] = rk4_const(Q[d], kQ[d], h6);
      // the test of layer_exit: interface `layer` below (flat) or inside
      // (spherical), interface layer - 1 above or outside
      const bool in_ok = layer < med.nlayer - 1, out_ok = layer > 0;
      bool crossed;
      if (med.geometry == 1) {
        const double r = sqrt(Qn[0] * Qn[0] + Qn[1] * Qn[1] + Qn[2] * Qn[2]);
        crossed = (in_ok && r < b_in) || (out_ok && r > b_out) || (layer == 0 && med.surface > 0.0 && r > med.surface);
      } else {
        crossed = (in_ok && Qn[2] > b_in) || (out_ok && Qn[2] < b_out) ||
                  (layer == med.nlayer - 1 && med.surface > 0.0 && Qn[2] > med.surface);
      }
      if (crossed) {
        // the interface step redoes this step from the stored state
        a.i32[FGA_FLAGS * cap + i] = flags | FGA_FLAG_CROSS;
      } else {
        const double Sn = rk4_const(S, kS, h6);
        bool finite = isfinite(Sn) && isfinite(P[0]) && isfinite(P[1]) && isfinite(P[2]);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          F[(FGA_Q + d) * cap + i] = Qn[d];
          finite = finite && isfinite(Qn[d]);
        }
        F[FGA_S * cap + i] = Sn;
        double kr[9], ki[9], z0r[9], z0i[9];
        pc_jac_rates(ph, ci, pr, pi, kr, ki);
#pragma unroll
        for (int o = 0; o < 9; ++o) {
          z0r[o] = qr[o] - pi[o];
          z0i[o] = qi[o] + pr[o];
          const double nr = rk4_const(qr[o], kr[o], h6), ni = rk4_const(qi[o], ki[o], h6);
          F[(FGA_ZQ_RE + o) * cap + i] = nr;
          F[(FGA_ZQ_IM + o) * cap + i] = ni;
          finite = finite && isfinite(nr) && isfinite(ni) && isfinite(pr[o]) && isfinite(pi[o]);
        }
        pc_amplitude(z0r, z0i, kr, ki, isS, A, dt);
        if (isS) reframe_s(P, A, e);
#pragma unroll
        for (int t = 0; t < 4; ++t) finite = finite && isfinite(A[t]);
        if (!finite) {
          flags = FGA_FLAG_QUARANTINED;
          quar = 1;
        } else if (a.cutoff_abs > 0.0) {
          const double wr = F[FGA_W_RE * cap + i], wi = F[FGA_W_IM * cap + i];
          const double m0 = A[0] * A[0] + A[1] * A[1];
          const double m1 = A[2] * A[2] + A[3] * A[3];
          const double amax = sqrt(m0 > m1 ? m0 : m1);
          if (sqrt(wr * wr + wi * wi) * amax < a.cutoff_abs) {
            flags = 0;
            culled = 1;
          }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) F[(FGA_A0_RE + t) * cap + i] = A[t];
#pragma unroll
        for (int d = 0; d < 3; ++d) F[(FGA_E + d) * cap + i] = e[d];
        a.i32[FGA_FLAGS * cap + i] = flags;
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    steps_done += __shfl_down(steps_done, off);
    culled += __shfl_down(culled, off);
    quar += __shfl_down(quar, off);
  }
  if ((threadIdx.x & 63) == 0 && a.counters) {
    if (steps_done) atomicAdd(a.counters + 0, steps_done);
    if (culled) atomicAdd(a.counters + 1, culled);
    if (quar) atomicAdd(a.counters + 2, quar);
  }
}

// One step of every beam in a layered medium where some layer has a speed
// gradient: the general RK4 step (medium_eval gives c, grad c and Hess c of
// the beam's layer at each stage), and a beam whose centre has left its
// layer is flagged with its stored state untouched, as in k_step_layered.
// SV = 1: S beams take the step with the frame-free amplitude (A formed from
// the frame at the load and returned to it before the store).
template <int SV = 0>
__global__ __launch_bounds__(256) void k_step_layered_grad(DevMedium med, IntegrateArgs a)
{
  const int64_t i = a.beg + (int64_t)blockIdx.x * 256 + threadIdx.x;
  unsigned long long steps_done = 0, culled = 0, quar = 0;
  if (i < a.end) {
    const int64_t cap = a.cap;
    double *__restrict__ F = a.f64;
    int32_t flags = a.i32[FGA_FLAGS * cap + i];
    if (flags & FGA_FLAG_ALIVE) {
      steps_done = 1;
      const int br = a.i32[FGA_BRANCH * cap + i];
      const double sg = (double)a.i32[FGA_SIGMA * cap + i];
      const int layer = a.i32[FGA_LAYER * cap + i];
      const int sp = br == 0 ? 0 : 1;
      const bool isS = br != 0;
      double y[nstate<SV>()], e[3];
#pragma unroll
      for (int f = 0; f < NS; ++f) y[f] = F[f * cap + i];
#pragma unroll
      for (int d = 0; d < 3; ++d) e[d] = F[(FGA_E + d) * cap + i];
      if (SV) {
        y[nstate<SV>() - 2] = 0.0;
        y[nstate<SV>() - 1] = 0.0;
        if (isS) frame_to_vector(y, e);
      }
      rk4_step<MK_LAYERED, SV>(med, sp, layer, sg, isS, e, y, a.dt);
      int iface, nl;
      if (layer_exit(med, layer, y + IQ, iface, nl)) {
        // the interface step redoes this step from the stored state
        a.i32[FGA_FLAGS * cap + i] = flags | FGA_FLAG_CROSS;
      } else {
        if (isS && SV) vector_to_frame(y, e);
        else if (isS) reframe_s(y, e);
        bool finite = true;
#pragma unroll
        for (int f = 0; f < NS; ++f) finite = finite && isfinite(y[f]);
        if (!finite) {
          flags = FGA_FLAG_QUARANTINED;
          quar = 1;
        } else if (a.cutoff_abs > 0.0) {
          const double wr = F[FGA_W_RE * cap + i], wi = F[FGA_W_IM * cap + i];
          const double m0 = y[IA] * y[IA] + y[IA + 1] * y[IA + 1];
          const double m1 = y[IA + 2] * y[IA + 2] + y[IA + 3] * y[IA + 3];
          if (sqrt(wr * wr + wi * wi) * sqrt(m0 > m1 ? m0 : m1) < a.cutoff_abs) {
            flags = 0;
            culled = 1;
          }
        }
#pragma unroll
        for (int f = 0; f < NS; ++f) F[f * cap + i] = y[f];
#pragma unroll
        for (int d = 0; d < 3; ++d) F[(FGA_E + d) * cap + i] = e[d];
        a.i32[FGA_FLAGS * cap + i] = flags;
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    steps_done += __shfl_down(steps_done, off);
    culled += __shfl_down(culled, off);
    quar += __shfl_down(quar, off);
  }
  if ((threadIdx.x & 63) == 0 && a.counters) {
    if (steps_done) atomicAdd(a.counters + 0, steps_done);
    if (culled) atomicAdd(a.counters + 1, culled);
    if (quar) atomicAdd(a.counters + 2, quar);
  }
}

// Emission records of the current state (no stepping), e.g. for t = 0
// samples.  With box: each wavefront is one 64-beam tile of the records and
// also writes that tile's bounding box of the live centres Q (lo[3], hi[3];
// +inf / -inf when no beam of the tile is live), as k_tile_box would from
// the records.
__global__ __launch_bounds__(256) void k_emit(const double *__restrict__ F, const int32_t *__restrict__ I,
                                              int64_t cap, int64_t beg, int64_t end, double ieps,
                                              double *__restrict__ out, double *__restrict__ box)
{
  const int64_t i = beg + (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t nb = end - beg, j = i - beg;
  double q[3] = {-1.0e300, -1.0e300, -1.0e300};  // dead beams and the ragged tail
  if (i < end) {
    if (!(I[FGA_FLAGS * cap + i] & FGA_FLAG_ALIVE)) {
      emit_dead(out, nb, j);
    } else {
      double y[NS];
#pragma unroll
      for (int f = 0; f < NS; ++f) y[f] = F[f * cap + i];
      const double e[3] = {F[(FGA_E + 0) * cap + i], F[(FGA_E + 1) * cap + i], F[(FGA_E + 2) * cap + i]};
      emit_record(out, nb, j, y, e, F[FGA_W_RE * cap + i], F[FGA_W_IM * cap + i], I[FGA_BRANCH * cap + i] != 0,
                  ieps);
      q[0] = y[IQ];
      q[1] = y[IQ + 1];
      q[2] = y[IQ + 2];
    }
  }
  if (box) {
    const int lane = threadIdx.x & 63;
    double lo[3], hi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const bool dead = !(q[d] > -1.0e299);
      lo[d] = dead ? INFINITY : q[d];
      hi[d] = dead ? -INFINITY : q[d];
      for (int off = 32; off > 0; off >>= 1) {
        lo[d] = fmin(lo[d], __shfl_xor(lo[d], off));
        hi[d] = fmax(hi[d], __shfl_xor(hi[d], off));
      }
    }
    const int64_t t = (j - lane) >> 6;  // this wavefront's tile
    if (lane < 6 && t * 64 < nb) {
      double v = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        if (lane == d) v = lo[d];
        if (lane == 3 + d) v = hi[d];
      }
      box[t * 6 + lane] = v;
    }
  }
}

}  // namespace

hipError_t launch_integrate(const DevMedium &m, const IntegrateArgs &a, hipStream_t st)
{
  const int64_t n = a.end - a.beg;
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  ProfScope prof(FGA_K_INTEGRATE, st);
  switch (m.kind) {
  case FGA_MEDIUM_HOMOGENEOUS: hipLaunchKernelGGL(k_integrate<MK_HOMOG>, blocks, 256, 0, st, m, a); break;
  case FGA_MEDIUM_GRID:
    // frame-free S amplitudes: a variant of the grid-medium kernels (in a
    // homogeneous medium P is constant and the two forms are one)
    if (m.smooth && a.s_vector) hipLaunchKernelGGL((k_integrate<MK_GRID3, 1>), blocks, 256, 0, st, m, a);
    else if (m.smooth) hipLaunchKernelGGL(k_integrate<MK_GRID3>, blocks, 256, 0, st, m, a);
    else if (a.s_vector) hipLaunchKernelGGL((k_integrate<MK_GRID, 1>), blocks, 256, 0, st, m, a);
    else hipLaunchKernelGGL(k_integrate<MK_GRID>, blocks, 256, 0, st, m, a);
    break;
  default:
    // layered media advance one step per launch, the interface step between
    if (a.nsteps != 1 || a.stride != 0) return hipErrorInvalidValue;
    if (m.any_grad && a.s_vector) hipLaunchKernelGGL(k_step_layered_grad<1>, blocks, 256, 0, st, m, a);
    else if (m.any_grad) hipLaunchKernelGGL(k_step_layered_grad<0>, blocks, 256, 0, st, m, a);
    else hipLaunchKernelGGL(k_step_layered, blocks, 256, 0, st, m, a);
    break;
  }
  return hipGetLastError();
}

hipError_t launch_emit(const double *f64, const int32_t *i32, int64_t cap, int64_t beg, int64_t end,
                       double eps, double *emit, double *box, hipStream_t st)
{
  const int64_t n = end - beg;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_emit, (unsigned)((n + 255) / 256), 256, 0, st, f64, i32, cap, beg, end, 1.0 / eps, emit,
                     box);
  return hipGetLastError();
}

}  // namespace fga
