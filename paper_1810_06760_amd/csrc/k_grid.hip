// Step 3 on a uniform grid (eq:FGA) as tile GEMMs on the matrix cores.
//
// With the box window, each beam's term factorises over the axes:
//   u_c(x_i, y_j, z_l) = sum_b W_bc Ex_b(i) Ey_b(j) Ez_b(l),
//   E_d(i) = exp(i P_d (x_i - Q_d)/eps - (x_i - Q_d)^2/(2 eps)) on |x_i - Q_d| <= R, else 0,
//   W_bc = w_b exp(i S_b/eps) A_bc.
// For a 16^3 tile this is the complex product U[(j,i),(c,l)] =
// sum_b (Ey (.) Ex)[(j,i),b] (W_c Ez)[b,(c,l)] -- a Khatri-Rao row block times
// a factor block, M = 256, N = 48, K = beams near the tile.  It runs as a real
// GEMM [Re X | Im X] [[Re V, Im V], [-Im V, Re V]] on v_mfma_f64_16x16x4_f64.
//
// Mixed precision: the 1-D factors take their phases reduced modulo 2 pi
// and their Gaussian exponents in FP64, then the exponential and sine/cosine
// in FP32; W is scaled by 1 / max_b |W_b|.  The product runs with FP32
// accumulation on v_mfma_f32_16x16x4_f32 (FGA_FP32), or with each operand
// split into hi + lo halves, hi = round(x), lo = round(x - hi), and the three
// products hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_{bf16,f16}
// (FGA_BF16X3, FGA_FP16X3); FGA_FP16X2 rounds the Khatri-Rao rows to FP16
// once (2^-11 relative) and splits only the factor block, two products.
// Every tile kernel is software-pipelined: one batch of beams on the matrix
// cores while the next one's factors are built, one barrier per batch.
//
// Beams are binned by the tile-sized cell of Q (radix sort of cell keys); a
// tile's candidates are the (2r+1)^2 contiguous runs of cells within reach of
// it.  Each tile's candidate list is split into segments (work items, one
// workgroup each, launched longest first so that short items fill the end of
// the launch), whose partial tiles are then reduced in a fixed order.
#include <algorithm>
#include <hipcub/hipcub.hpp>
#include <type_traits>

#include "device_common.h"
#include "fastmath.h"

namespace fga {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int T = 16;       // tile edge (points)
constexpr int NB = 16;      // beams per LDS batch
constexpr int MAXR = 1024;  // max candidate runs per tile: (2 reach + 1)^2
constexpr int NSEG = 4096;  // work items per launch beyond one per tile (at most 8 per tile)

struct GridGeom {
  int n[3], nt[3], nc[3], reach[3];
  double lo[3], h[3];
  double R, eps;
};

__device__ __forceinline__ double axis_coord(const GridGeom &g, int d, int i)
{
  return __dadd_rn(g.lo[d], __dmul_rn(g.h[d], (double)i));
}

// Number of grid indices i in [0, n) with |lo + i h - q| <= R.
__device__ int64_t axis_count(const GridGeom &g, int d, double q)
{
  int lo_i = (int)ceil((q - g.R - g.lo[d]) / g.h[d]);
  int hi_i = (int)floor((q + g.R - g.lo[d]) / g.h[d]);
  lo_i = lo_i < 0 ? 0 : lo_i;
  hi_i = hi_i > g.n[d] - 1 ? g.n[d] - 1 : hi_i;
  while (lo_i > 0 && fabs(axis_coord(g, d, lo_i - 1) - q) <= g.R) --lo_i;
  while (lo_i <= hi_i && fabs(axis_coord(g, d, lo_i) - q) > g.R) ++lo_i;
  while (hi_i < g.n[d] - 1 && fabs(axis_coord(g, d, hi_i + 1) - q) <= g.R) ++hi_i;
  while (hi_i >= lo_i && fabs(axis_coord(g, d, hi_i) - q) > g.R) --hi_i;
  return hi_i >= lo_i ? (int64_t)(hi_i - lo_i + 1) : 0;
}

__global__ __launch_bounds__(256) void k_bin_keys(const double *__restrict__ F, const int32_t *__restrict__ I,
                                                  int64_t cap, int64_t n, GridGeom g, int32_t *__restrict__ keys,
                                                  int32_t *__restrict__ vals, unsigned long long *__restrict__ evals)
{
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  unsigned long long ev = 0;
  if (i < n) {
    int32_t key = 0x7fffffff;
    if (I[FGA_FLAGS * cap + i] & FGA_FLAG_ALIVE) {
      bool in = true;
      int c[3];
      int64_t cnt = 1;
      for (int d = 0; d < 3; ++d) {
        const double q = F[(FGA_Q + d) * cap + i];
        const double u = floor((q - g.lo[d]) / (T * g.h[d]));
        in = in && u >= -(double)g.reach[d] && u < (double)(g.nt[d] + g.reach[d]);
        c[d] = in ? (int)u + g.reach[d] : 0;
        cnt *= axis_count(g, d, q);
      }
      if (in) key = (c[2] * g.nc[1] + c[1]) * g.nc[0] + c[0];
      ev = (unsigned long long)cnt;
    }
    keys[i] = key;
    vals[i] = (int32_t)i;
  }
  for (int off = 32; off > 0; off >>= 1) ev += __shfl_down(ev, off);
  if ((threadIdx.x & 63) == 0 && ev && evals) atomicAdd(evals, ev);
}

// start[c] = first sorted position with key >= c, for c in [0, ncells].
__global__ __launch_bounds__(256) void k_cell_start(const int32_t *__restrict__ keys, int64_t n, int32_t ncells,
                                                    int64_t *__restrict__ start)
{
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c > ncells) return;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (keys[mid] < c) lo = mid + 1;
    else hi = mid;
  }
  start[c] = lo;
}

// Candidate runs of tile t: for each (cz, cy) within reach, the cells
// cx in [tx, tx + 2 reach] of the shifted cell grid.
__device__ __forceinline__ void tile_run(const GridGeom &g, const int64_t *start, int tx, int ty, int tz, int r,
                                         int64_t &b, int64_t &len)
{
  const int wy = 2 * g.reach[1] + 1;
  const int cz = tz + r / wy, cy = ty + r % wy;
  const int64_t row = ((int64_t)cz * g.nc[1] + cy) * g.nc[0];
  b = start[row + tx];
  len = start[row + tx + 2 * g.reach[0] + 1] - b;
}

__global__ __launch_bounds__(256) void k_tile_counts(GridGeom g, const int64_t *__restrict__ start,
                                                     int64_t *__restrict__ counts)
{
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int ntile = g.nt[0] * g.nt[1] * g.nt[2];
  if (t >= ntile) return;
  const int tx = t % g.nt[0], ty = (t / g.nt[0]) % g.nt[1], tz = t / (g.nt[0] * g.nt[1]);
  const int nr = (2 * g.reach[1] + 1) * (2 * g.reach[2] + 1);
  int64_t s = 0;
  for (int r = 0; r < nr; ++r) {
    int64_t b, len;
    tile_run(g, start, tx, ty, tz, r, b, len);
    s += len;
  }
  counts[t] = s;
}

struct Item {
  int32_t tile;
  int32_t pad;
  int64_t k0, k1;
};

__device__ __forceinline__ void cmul(double ar, double ai, double br, double bi, double &cr, double &ci)
{
  cr = ar * br - ai * bi;
  ci = ar * bi + ai * br;
}

// Compact per-beam record in cell order: Q (3), P/eps (3), W = w e^{iS/eps} A (3 complex).
__global__ __launch_bounds__(256) void k_grid_records(const double *__restrict__ F, const int32_t *__restrict__ I,
                                                      int64_t cap, const int32_t *__restrict__ keys,
                                                      const int32_t *__restrict__ order, int64_t n, double ieps,
                                                      double *__restrict__ rec, unsigned long long *__restrict__ wmax)
{
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= n || keys[s] == 0x7fffffff) return;
  const int64_t bi = order[s];
  const double pscale = ieps * INV_PI_128;  // the phase (P/eps).(x - Q) in units of pi/128
  double P[3], e[3];
  double *o = rec + s * 12;
  for (int d = 0; d < 3; ++d) {
    o[d] = F[(FGA_Q + d) * cap + bi];
    P[d] = F[(FGA_P + d) * cap + bi];
    o[3 + d] = P[d] * pscale;
    e[d] = F[(FGA_E + d) * cap + bi];
  }
  const double a0r = F[FGA_A0_RE * cap + bi], a0i = F[FGA_A0_IM * cap + bi];
  const double a1r = F[FGA_A1_RE * cap + bi], a1i = F[FGA_A1_IM * cap + bi];
  double Ar[3], Ai[3];
  if (I[FGA_BRANCH * cap + bi] == 0) {
    const double ip = 1.0 / sqrt(P[0] * P[0] + P[1] * P[1] + P[2] * P[2]);
    for (int c = 0; c < 3; ++c) { Ar[c] = a0r * P[c] * ip; Ai[c] = a0i * P[c] * ip; }
  } else {
    double nsh[3], nsv[3];
    s_frame(P, e, nsh, nsv);
    for (int c = 0; c < 3; ++c) {
      Ar[c] = a0r * nsv[c] + a1r * nsh[c];
      Ai[c] = a0i * nsv[c] + a1i * nsh[c];
    }
  }
  double sn, cs;
  sincos(F[FGA_S * cap + bi] * ieps, &sn, &cs);
  double wr, wi;
  cmul(F[FGA_W_RE * cap + bi], F[FGA_W_IM * cap + bi], cs, sn, wr, wi);
  double m = 0.0;
  for (int c = 0; c < 3; ++c) {
    cmul(wr, wi, Ar[c], Ai[c], o[6 + 2 * c], o[7 + 2 * c]);
    m = fmax(m, fmax(fabs(o[6 + 2 * c]), fabs(o[7 + 2 * c])));
  }
  // non-negative doubles order like their bit patterns
  if (wmax && m > 0.0 && m < INFINITY) atomicMax(wmax, (unsigned long long)__double_as_longlong(m));
}

// ------------------------------------------------------ mixed precision --
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

constexpr double LOG2E = 1.4426950408889634;
constexpr int LCAP = 1024;  // ring of accepted candidates (power of two)

// Mixed record, written over the FP64 record of the same beam once the
// largest |W| is known: Q and the phase rate in FP64, the weights in FP32
// scaled by 1 / max |W| and balanced against the x factor by an exact power
// of two (Ex scaled by 2^kb, W by 2^-kb, |W| / wmax ~ 2^(2 kb)), so that
// neither operand leaves the normal range of a 16-bit type sooner than it
// must.
struct alignas(16) MxRec {
  double q[3];
  double rev[3];  // P / (2 pi eps): the phase in revolutions per unit length
  float w[6];     // (re, im) of W_c / wmax * 2^-kb, c = 0..2
  float xs;       // 2^kb
  float pad;
};
static_assert(sizeof(MxRec) <= 12 * sizeof(double), "the mixed record fits in the FP64 record's stride");

__global__ __launch_bounds__(256) void k_mx_records(double *__restrict__ rec, const int32_t *__restrict__ keys,
                                                    int64_t n, const unsigned long long *__restrict__ wmax)
{
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= n || keys[s] == 0x7fffffff) return;
  const double ws = __longlong_as_double((long long)*wmax);
  const double iws = ws > 0.0 ? 1.0 / ws : 0.0;
  double *o = rec + s * 12;
  double W[6], wm = 0.0;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    W[f] = o[6 + f] * iws;
    wm = fmax(wm, fabs(W[f]));
  }
  const int kb = wm > 0.0 ? ilogb(wm) / 2 : 0;
  MxRec r;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    r.q[d] = o[d];
    r.rev[d] = o[3 + d] * (1.0 / 256.0);  // from units of pi/128 to revolutions
  }
#pragma unroll
  for (int f = 0; f < 6; ++f) r.w[f] = (float)ldexp(W[f], -kb);
  r.xs = ldexpf(1.0f, kb);
  r.pad = 0.0f;
  *reinterpret_cast<MxRec *>(o) = r;  // every field above depends on the loads
}

// 16-bit operands of one column block: per (column block, lane quarter, l)
// the 8 consecutive K entries a lane feeds to the matrix core (16 bytes);
// the 16 lanes of a quarter read 16 consecutive entries (no bank conflicts)
struct alignas(16) H8Raw {
  uint32_t v[4];  // pairs of 16-bit values (K order: low half first)
};

// Factors of one batch of NB beams: Ex, Ey (FP32) and the factor block
// V = W Ez, as FP32 (FGA_FP32) or split into 16-bit hi and lo in the matrix
// instruction's K order.
template <int PREC> struct MxBuf {
  float2 Ex[NB][T], Ey[NB][T];
  H8Raw Bh[6][4][T], Bl[6][4][T];
};
template <> struct MxBuf<FGA_FP32> {
  float2 Ex[NB][T], Ey[NB][T], V[NB][3][T];
};

// -1 that the compiler cannot fold, so that x - hi below stays an FMA with
// hi as a (16-bit) source: for FP16 one v_fma_mix_f32 reads hi as stored,
// with no separate conversion back to FP32.
__device__ __forceinline__ float opaque_m1()
{
  float m = -1.0f;
  asm volatile("" : "+v"(m));
  return m;
}

// x - hi, hi the 16-bit rounding of x (exact in FP32); a BF16 value widens
// by a shift, which the plain difference uses
template <class S> __device__ __forceinline__ float rem16(float x, S hi, float m1)
{
  if constexpr (std::is_same<S, _Float16>::value) return __builtin_fmaf((float)hi, m1, x);
  else return x - (float)hi;
}

// One thread's copy of the mixed record of beam jb of a batch (every thread
// of the beam's 16 reads it; the loads of one wavefront touch 4 records).
struct MxRegs {
  double2 a, b, c;  // (q0, q1), (q2, rev0), (rev1, rev2)
  float4 d, e;      // (w0, w1, w2, w3), (w4, w5, xs, pad)
};

__device__ __forceinline__ void mx_fetch(const double *__restrict__ rec, const int32_t *ring, int64_t p, int jb,
                                         int cnt, MxRegs &r)
{
  if (jb < cnt) {
    const double2 *src = reinterpret_cast<const double2 *>(rec + (int64_t)ring[(p + jb) & (LCAP - 1)] * 12);
    r.a = src[0];
    r.b = src[1];
    r.c = src[2];
    const float4 *fs = reinterpret_cast<const float4 *>(src + 3);
    r.d = fs[0];
    r.e = fs[1];
  } else {  // idle slot: outside every window, zero weight
    r.a = make_double2(-1.0e300, -1.0e300);
    r.b = make_double2(-1.0e300, 0.0);
    r.c = make_double2(0.0, 0.0);
    r.d = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    r.e = make_float4(0.0f, 0.0f, 1.0f, 0.0f);
  }
}

// Window-masked 1-D factors in FP32 from FP64 arguments, thread (jb, ii):
// the Gaussian exponent and the phase (in revolutions, reduced to
// [-1/2, 1/2]) are formed in FP64; exp2 and sin/cos of 2 pi r run on the
// FP32 transcendental unit.  For the 16-bit products (S = __bf16 / _Float16)
// the B operand's hi and lo halves are written in the K order of the matrix
// instruction: k = 2 beam + part, with column block c (Re U) taking
// (Re V, -Im V) and c + 3 (Im U) taking (Im V, Re V).
template <int PREC>
__device__ __forceinline__ void mx_make(const GridGeom &g, const double (&xq)[3], double hl2, const MxRegs &r,
                                        MxBuf<PREC> &fb, int jb, int ii)
{
  typedef typename std::conditional<PREC == FGA_BF16X3, __bf16, _Float16>::type S;
  const double q[3] = {r.a.x, r.a.y, r.b.x};
  const double rv[3] = {r.b.y, r.c.x, r.c.y};
  float2 E[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    // outside the window the offset is replaced by one whose Gaussian is
    // exactly 0 in FP32 (and whose phase is 0), so nothing branches
    const double u0 = xq[d] - q[d];
    const double u = fabs(u0) <= g.R ? u0 : 1.0e30;
    const double rev = rv[d] * u;
    const float rf = (float)(rev - rint(rev));
    const float amp = __builtin_amdgcn_exp2f((float)(u * u * hl2));
    E[d] = make_float2(amp * __builtin_amdgcn_cosf(rf), amp * __builtin_amdgcn_sinf(rf));
  }
  const float xs = r.e.z;
  fb.Ex[jb][ii] = make_float2(E[0].x * xs, E[0].y * xs);
  fb.Ey[jb][ii] = E[1];
  const float w[6] = {r.d.x, r.d.y, r.d.z, r.d.w, r.e.x, r.e.y};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float wr = w[2 * c], wi = w[2 * c + 1];
    const float vx = wr * E[2].x - wi * E[2].y, vy = wr * E[2].y + wi * E[2].x;
    if constexpr (PREC == FGA_FP32) {
      fb.V[jb][c][ii] = make_float2(vx, vy);
    } else {
      // packed conversions: hi = (round(vx), round(-vy)), lo = the rounded
      // remainders (rounding to nearest is odd-symmetric, so the Im U pairs
      // are the same values swapped and re-signed)
      typedef S s2 __attribute__((ext_vector_type(2)));
      typedef float fl2 __attribute__((ext_vector_type(2)));
      const s2 h1 = __builtin_convertvector((fl2){vx, -vy}, s2);
      const float m1 = std::is_same<S, _Float16>::value ? opaque_m1() : -1.0f;
      const float rx = rem16(vx, h1.x, m1), rny = rem16(-vy, h1.y, m1);
      const s2 l1 = __builtin_convertvector((fl2){rx, rny}, s2);
      const s2 h2 = __builtin_convertvector((fl2){vy, vx}, s2);
      const s2 l2 = __builtin_convertvector((fl2){-rny, rx}, s2);
      const int q4 = jb >> 2, t = jb & 3;  // K entries 2t, 2t + 1 of the lane's eight
      fb.Bh[c][q4][ii].v[t] = __builtin_bit_cast(uint32_t, h1);
      fb.Bl[c][q4][ii].v[t] = __builtin_bit_cast(uint32_t, l1);
      fb.Bh[c + 3][q4][ii].v[t] = __builtin_bit_cast(uint32_t, h2);
      fb.Bl[c + 3][q4][ii].v[t] = __builtin_bit_cast(uint32_t, l2);
    }
  }
}

// The K = 2 NB (re, im) slice of the tile GEMM for one batch; wavefront w
// owns tile rows j = 4 w + rb.
template <int PREC>
__device__ __forceinline__ void mx_mma(const MxBuf<PREC> &fb, f4 (&acc)[4][6], int w, int lane)
{
  const int li = lane & 15, kq = lane >> 4;
  if constexpr (PREC == FGA_FP32) {
    // K = 4 per instruction: 2 beams x (re, im); lane holds A[i = li][k = kq], B[k = kq][l = li]
    const int part = kq & 1;
#pragma unroll
    for (int ks = 0; ks < NB / 2; ++ks) {
      const int jb = 2 * ks + (kq >> 1);
      const float2 xv = fb.Ex[jb][li];
      float a[4];
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        const float2 yv = fb.Ey[jb][4 * w + rb];
        a[rb] = part ? xv.x * yv.y + xv.y * yv.x : xv.x * yv.x - xv.y * yv.y;
      }
      float b[6];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float2 v = fb.V[jb][c][li];
        b[c] = part ? -v.y : v.x;
        b[3 + c] = part ? v.x : v.y;
      }
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 6; ++cb)
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb], b[cb], acc[rb][cb], 0, 0, 0);
    }
  } else {
    // K = 32 per instruction: the 16 beams of the batch x (re, im); lane
    // holds A[i = li][k = 8 kq + t] and B[k = 8 kq + t][l = li], t < 8,
    // k = 2 beam + part
    typedef typename std::conditional<PREC == FGA_BF16X3, __bf16, _Float16>::type S;
    typedef typename std::conditional<PREC == FGA_BF16X3, bf8, h8>::type V8;
    typedef S s2 __attribute__((ext_vector_type(2)));
    typedef float fl2 __attribute__((ext_vector_type(2)));
    const float m1 = std::is_same<S, _Float16>::value ? opaque_m1() : -1.0f;
    V8 ahi[4], alo[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int jb = 4 * kq + t;
        const float2 xv = fb.Ex[jb][li], yv = fb.Ey[jb][4 * w + rb];
        const float x0 = xv.x * yv.x - xv.y * yv.y;
        const float x1 = xv.x * yv.y + xv.y * yv.x;
        const s2 h = __builtin_convertvector((fl2){x0, x1}, s2);  // one packed conversion per beam
        ahi[rb][2 * t] = h.x;
        ahi[rb][2 * t + 1] = h.y;
        if constexpr (PREC != FGA_FP16X2) {
          const s2 l = __builtin_convertvector((fl2){rem16(x0, h.x, m1), rem16(x1, h.y, m1)}, s2);
          alo[rb][2 * t] = l.x;
          alo[rb][2 * t + 1] = l.y;
        }
      }
    }
#pragma unroll
    for (int cb = 0; cb < 6; ++cb) {
      const V8 bhi = __builtin_bit_cast(V8, fb.Bh[cb][kq][li]);
      const V8 blo = __builtin_bit_cast(V8, fb.Bl[cb][kq][li]);
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        if constexpr (PREC == FGA_BF16X3) {
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[rb], bhi, acc[rb][cb], 0, 0, 0);
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[rb], blo, acc[rb][cb], 0, 0, 0);
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[rb], bhi, acc[rb][cb], 0, 0, 0);
        } else if constexpr (PREC == FGA_FP16X2) {
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ahi[rb], blo, acc[rb][cb], 0, 0, 0);
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ahi[rb], bhi, acc[rb][cb], 0, 0, 0);
        } else {
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(alo[rb], bhi, acc[rb][cb], 0, 0, 0);
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ahi[rb], blo, acc[rb][cb], 0, 0, 0);
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ahi[rb], bhi, acc[rb][cb], 0, 0, 0);
        }
      }
    }
  }
}

// Mixed policy: 16 rows of the tile per workgroup (4 per wavefront), FP32
// accumulators scaled back by max |W| at the store.
template <int PREC> struct PolMx {
  static constexpr int SPLIT = 1;
  typedef MxBuf<PREC> Buf;
  typedef MxRegs Regs;
  typedef f4 Acc[4][6];
  struct Extra {};
  static __device__ void init(Extra &) {}
  static __device__ double arg(const GridGeom &g) { return -0.5 / g.eps * LOG2E; }
  static __device__ void zero(Acc &acc)
  {
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < 6; ++cb) acc[rb][cb] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  }
  static __device__ void fetch(const double *rec, const int32_t *ring, int64_t p, int jb, int cnt, Regs &r)
  {
    mx_fetch(rec, ring, p, jb, cnt, r);
  }
  static __device__ void make(const GridGeom &g, const double (&xq)[3], double hl2, const Regs &r, Buf &fb,
                              const Extra &, int jb, int ii)
  {
    mx_make<PREC>(g, xq, hl2, r, fb, jb, ii);
  }
  static __device__ void mma(const Buf &fb, Acc &acc, int w, int lane, int) { mx_mma<PREC>(fb, acc, w, lane); }
  // result register r of lane holds D[4 (lane/16) + r][lane % 16]
  static __device__ void store(const Acc &acc, double *P, double ws, int)
  {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      const int j = 4 * w + rb;
#pragma unroll
      for (int cb = 0; cb < 6; ++cb) {
        const int u = cb / 3, c = cb % 3;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 4 * (lane >> 4) + r, l = lane & 15;
          P[((((int64_t)c * T + l) * T + j) * T + i) * 2 + u] = (double)acc[rb][cb][r] * ws;
        }
      }
    }
  }
};

// ------------------------------------------------------------------ FP64 --
// Factors of one batch in FP64 (table-driven complex exponential) and the
// factor block V = W Ez.
struct F64Buf {
  double2 Ex[NB][T], Ey[NB][T], V[NB][3][T];
};

// One thread's copy of the FP64 record of beam jb of a batch:
// (q0, q1), (q2, v0), (v1, v2), W_0, W_1, W_2 (v: phase rate in units of pi/128).
struct F64Regs {
  double2 r[6];
};

// FP64 policy: a tile's 16 rows are split over two workgroups (8 rows each,
// 2 per wavefront), which halves the accumulators so that two wavefronts fit
// per SIMD.
struct PolF64 {
  static constexpr int SPLIT = 2, RB = 2;
  typedef F64Buf Buf;
  typedef F64Regs Regs;
  typedef d4 Acc[RB][6];
  struct Extra {
    TrigTables tab;
  };
  static __device__ void init(Extra &x) { fill_tables(x.tab); }
  static __device__ double arg(const GridGeom &g) { return 0.5 / g.eps; }
  static __device__ void zero(Acc &acc)
  {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int cb = 0; cb < 6; ++cb) acc[rb][cb] = d4{0.0, 0.0, 0.0, 0.0};
  }
  static __device__ void fetch(const double *__restrict__ rec, const int32_t *ring, int64_t p, int jb, int cnt,
                               Regs &r)
  {
    if (jb < cnt) {
      const double2 *src = reinterpret_cast<const double2 *>(rec + (int64_t)ring[(p + jb) & (LCAP - 1)] * 12);
#pragma unroll
      for (int k = 0; k < 6; ++k) r.r[k] = src[k];
    } else {  // idle slot: outside every window, zero weight
      r.r[0] = make_double2(-1.0e300, -1.0e300);
      r.r[1] = make_double2(-1.0e300, 0.0);
#pragma unroll
      for (int k = 2; k < 6; ++k) r.r[k] = make_double2(0.0, 0.0);
    }
  }
  // thread (jb, ii): Ex(ii), Ey(ii), Ez(ii) of beam jb and V(ii) = W Ez(ii)
  static __device__ void make(const GridGeom &g, const double (&xq)[3], double hieps, const Regs &r, Buf &fb,
                              const Extra &x, int jb, int ii)
  {
    const double q[3] = {r.r[0].x, r.r[0].y, r.r[1].x};
    const double v[3] = {r.r[1].y, r.r[2].x, r.r[2].y};
    double2 E[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double u = xq[d] - q[d];
      cexp_neg_units(x.tab, u * u * hieps, v[d] * u, fabs(u) <= g.R, E[d].x, E[d].y);
    }
    fb.Ex[jb][ii] = E[0];
    fb.Ey[jb][ii] = E[1];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double vr, vi;
      cmul(r.r[3 + c].x, r.r[3 + c].y, E[2].x, E[2].y, vr, vi);
      fb.V[jb][c][ii] = make_double2(vr, vi);
    }
  }
  // K = 4 per instruction: 2 beams x (re, im); lane holds A[i = li][k = kk],
  // B[k = kk][l = li]; this workgroup's wavefronts own rows j = 8 half + 2 w + rb
  static __device__ void mma(const Buf &fb, Acc &acc, int w, int lane, int half)
  {
    const int li = lane & 15, kk = lane >> 4, part = kk & 1;
    const int j0 = 8 * half + RB * w;
#pragma unroll 2
    for (int ks = 0; ks < NB / 2; ++ks) {
      const int jb = 2 * ks + (kk >> 1);
      const double2 xv = fb.Ex[jb][li];
      double a[RB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const double2 yv = fb.Ey[jb][j0 + rb];
        double xr, xi;
        cmul(xv.x, xv.y, yv.x, yv.y, xr, xi);
        a[rb] = part ? xi : xr;
      }
      double b[6];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double2 v = fb.V[jb][c][li];
        b[c] = part ? -v.y : v.x;     // columns of Re U
        b[3 + c] = part ? v.x : v.y;  // columns of Im U
      }
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < 6; ++cb)
          acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb], b[cb], acc[rb][cb], 0, 0, 0);
    }
  }
  // result register r of lane holds D[lane/16 + 4r][lane % 16] (row: x index i; column: z index l)
  static __device__ void store(const Acc &acc, double *P, double, int half)
  {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int j = 8 * half + RB * w + rb;
#pragma unroll
      for (int cb = 0; cb < 6; ++cb) {
        const int u = cb / 3, c = cb % 3;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = (lane >> 4) + 4 * r, l = lane & 15;
          P[((((int64_t)c * T + l) * T + j) * T + i) * 2 + u] = acc[rb][cb][r];
        }
      }
    }
  }
};

template <class Pol> struct PipeSmem {
  int64_t run_b[MAXR], run_pre[MAXR + 1];
  int32_t ring[LCAP];
  typename Pol::Buf fb[2];
  typename Pol::Extra x;
};

// One work item (a tile's candidate segment; with SPLIT = 2, half of the
// tile's rows), software-pipelined over batches of NB accepted beams: while
// the matrix cores take batch n from one factor buffer, the same wavefronts
// fetch batch n + 1's records and build its factors into the other, with one
// barrier per batch.  Accepted candidates (window box meets the tile's point
// box) are appended to a ring 256 candidates at a time, kept at least one
// batch ahead.
template <class Pol>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_grid_tile(
    GridGeom g, const int64_t *__restrict__ start, const Item *__restrict__ items, const int32_t *__restrict__ sched,
    const double *__restrict__ rec, double *__restrict__ partial, unsigned long long *__restrict__ executed,
    const unsigned long long *__restrict__ wmax)
{
  __shared__ PipeSmem<Pol> sm;
  Pol::init(sm.x);
  const double ws = wmax ? __longlong_as_double((long long)*wmax) : 1.0;
  const int64_t item = sched[blockIdx.x / Pol::SPLIT];
  const int half = blockIdx.x % Pol::SPLIT;
  const Item it = items[item];
  const int t = it.tile;
  const int tc[3] = {t % g.nt[0], (t / g.nt[0]) % g.nt[1], t / (g.nt[0] * g.nt[1])};
  const int nr = (2 * g.reach[1] + 1) * (2 * g.reach[2] + 1);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int jb = tid >> 4, ii = tid & 15;  // NB * T == 256
  double plo[3], phi[3], xq[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int i1 = T * tc[d] + T - 1 < g.n[d] - 1 ? T * tc[d] + T - 1 : g.n[d] - 1;
    plo[d] = axis_coord(g, d, T * tc[d]);
    phi[d] = axis_coord(g, d, i1);
    xq[d] = axis_coord(g, d, T * tc[d] + ii);
  }
  const double c0 = Pol::arg(g);
  if (tid == 0) {
    int64_t s = 0;
    for (int r = 0; r < nr; ++r) {
      int64_t b, len;
      tile_run(g, start, tc[0], tc[1], tc[2], r, b, len);
      sm.run_b[r] = b;
      sm.run_pre[r] = s;
      s += len;
    }
    sm.run_pre[nr] = s;
  }
  __syncthreads();

  typename Pol::Acc acc;
  Pol::zero(acc);

  int64_t cand = it.k0, tail = 0;
  auto refill = [&]() {
    const int64_t k = cand + tid;
    bool ok = false;
    int32_t s = -1;
    if (k < it.k1) {
      int lo = 0, hi = nr - 1;  // last run with run_pre <= k
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sm.run_pre[mid] <= k) lo = mid;
        else hi = mid - 1;
      }
      s = (int32_t)(sm.run_b[lo] + (k - sm.run_pre[lo]));
      const double *q = rec + (int64_t)s * 12;
      ok = q[0] + g.R >= plo[0] && q[0] - g.R <= phi[0] && q[1] + g.R >= plo[1] && q[1] - g.R <= phi[1] &&
           q[2] + g.R >= plo[2] && q[2] - g.R <= phi[2];
    }
    int tot;
    const int rk = block_rank(ok, &tot);
    if (ok) sm.ring[(tail + rk) & (LCAP - 1)] = s;
    tail += tot;
    cand += 256;
    __syncthreads();
  };
  auto clampnb = [](int64_t v) { return (int)(v < 0 ? 0 : v > NB ? NB : v); };

  // prologue: batch 0's factors into buffer 0
  while (tail < NB && cand < it.k1) refill();
  int64_t p = 0;  // ring position of the batch on the matrix cores
  int cc = clampnb(tail);
  typename Pol::Regs ra;
  Pol::fetch(rec, sm.ring, 0, jb, cc, ra);
  Pol::make(g, xq, c0, ra, sm.fb[0], sm.x, jb, ii);
  __syncthreads();

  unsigned long long nexec = 0;
  int buf = 0;
  while (cc > 0) {
    while (tail - (p + NB) < NB && cand < it.k1) refill();
    const int cn = clampnb(tail - (p + NB));
    Pol::fetch(rec, sm.ring, p + NB, jb, cn, ra);  // in flight while the matrix cores run
    Pol::mma(sm.fb[buf], acc, w, lane, half);
    Pol::make(g, xq, c0, ra, sm.fb[buf ^ 1], sm.x, jb, ii);  // zeros after the last batch
    __syncthreads();
    nexec += cc;
    buf ^= 1;
    p += NB;
    cc = cn;
  }
  if (tid == 0 && half == 0 && executed && nexec) atomicAdd(executed, nexec);
  // partial tile [c][l][j][i] complex
  Pol::store(acc, partial + item * (3 * T * T * T * 2), ws, half);
}

// out[c][z][y][x] = sum of the tile's partials (fixed item order), added to
// the previous contents with `add`; points outside the grid of a ragged tile
// are skipped.
__global__ __launch_bounds__(256) void k_grid_reduce(GridGeom g, const int32_t *__restrict__ first,
                                                     const int32_t *__restrict__ nitems,
                                                     const double *__restrict__ partial, double *__restrict__ out,
                                                     int add)
{
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t plane = (int64_t)g.n[0] * g.n[1] * g.n[2];
  if (id >= 3 * plane) return;
  const int c = (int)(id / plane);
  const int64_t p = id % plane;
  const int x = (int)(p % g.n[0]), y = (int)((p / g.n[0]) % g.n[1]), z = (int)(p / ((int64_t)g.n[0] * g.n[1]));
  const int t = ((z / T) * g.nt[1] + (y / T)) * g.nt[0] + (x / T);
  const int i = x % T, j = y % T, l = z % T;
  double re = 0.0, im = 0.0;
  const int f = first[t];
  for (int k = 0; k < nitems[t]; ++k) {
    const double *P = partial + (int64_t)(f + k) * (3 * T * T * T * 2) + ((((int64_t)c * T + l) * T + j) * T + i) * 2;
    re += P[0];
    im += P[1];
  }
  if (add) {
    re = out[2 * id] + re;
    im = out[2 * id + 1] + im;
  }
  out[2 * id] = re;
  out[2 * id + 1] = im;
}

GridGeom make_geom(const int n[3], const double lo[3], const double h[3], double eps, double tau)
{
  GridGeom g{};
  g.R = sqrt(2.0 * tau * eps);
  g.eps = eps;
  for (int d = 0; d < 3; ++d) {
    g.n[d] = n[d];
    g.lo[d] = lo[d];
    g.h[d] = h[d];
    g.nt[d] = (n[d] + T - 1) / T;
    g.reach[d] = (int)floor(g.R / (T * h[d])) + 1;
    g.nc[d] = g.nt[d] + 2 * g.reach[d];
  }
  return g;
}

}  // namespace

fga_status grid_sum_impl(const fga_beams *b, double eps, double tau, const int n[3], const double lo[3],
                         const double h[3], int precision, double *out, Arena &ar, hipStream_t st, bool size_only,
                         size_t *need, int64_t *evals_out, bool add)
{
  if (precision != FGA_FP64 && precision != FGA_FP32 && precision != FGA_BF16X3 && precision != FGA_FP16X3 &&
      precision != FGA_FP16X2)
    return fail(FGA_EINVAL, "unknown grid summation precision %d", precision);
  const GridGeom g = make_geom(n, lo, h, eps, tau);
  if ((2 * g.reach[1] + 1) * (2 * g.reach[2] + 1) > MAXR)
    return fail(FGA_EUNSUPPORTED, "window reach %d x %d tiles exceeds the supported %d runs per tile", g.reach[1],
                g.reach[2], MAXR);
  const int64_t nb = b->count;
  const int ntile = g.nt[0] * g.nt[1] * g.nt[2];
  const int64_t ncells = (int64_t)g.nc[0] * g.nc[1] * g.nc[2];
  if (ncells >= 0x7fffffff) return fail(FGA_EUNSUPPORTED, "too many cells");
  const int nseg = NSEG < 8 * ntile ? NSEG : 8 * ntile;
  const int max_items = nseg + ntile;

  int32_t *keys = ar.take<int32_t>(nb + 1), *keys2 = ar.take<int32_t>(nb + 1);
  int32_t *vals = ar.take<int32_t>(nb + 1), *vals2 = ar.take<int32_t>(nb + 1);
  int64_t *start = ar.take<int64_t>(ncells + 1);
  int64_t *tcount = ar.take<int64_t>(ntile);
  Item *items = ar.take<Item>(max_items);
  int32_t *sched = ar.take<int32_t>(max_items);
  int32_t *first = ar.take<int32_t>(ntile), *nitems = ar.take<int32_t>(ntile);
  unsigned long long *ev = ar.take<unsigned long long>(3);  // evals, executed, max |W| bits
  double *partial = ar.take<double>((size_t)max_items * 3 * T * T * T * 2);
  double *rec = ar.take<double>((size_t)12 * (nb + 1));
  size_t sort_bytes = 0;
  if (hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, keys, keys2, vals, vals2, (int)nb, 0, 31, st) !=
      hipSuccess)
    return fail(FGA_EDEVICE, "radix sort size query failed");
  void *sort_tmp = ar.take<char>(sort_bytes);
  if (size_only) {
    *need = ar.used;
    return FGA_OK;
  }
  if (!keys || !keys2 || !vals || !vals2 || !start || !tcount || !items || !sched || !first || !nitems || !ev || !partial ||
      !sort_tmp || !rec)
    return fail(FGA_ENOMEM, "grid summation workspace too small (%zu bytes given)", ar.size);
  if (nb > 0x7fffffff) return fail(FGA_EUNSUPPORTED, "more than 2^31 beams in one grid summation");

  FGA_HIP(hipMemsetAsync(ev, 0, 3 * sizeof(unsigned long long), st));
  if (nb > 0) {
    hipLaunchKernelGGL(k_bin_keys, (unsigned)((nb + 255) / 256), 256, 0, st, b->f64, b->i32, b->capacity, nb, g,
                       keys, vals, ev);
    FGA_LAUNCH_CHECK();
    FGA_HIP(hipcub::DeviceRadixSort::SortPairs(sort_tmp, sort_bytes, keys, keys2, vals, vals2, (int)nb, 0, 31, st));
    hipLaunchKernelGGL(k_grid_records, (unsigned)((nb + 255) / 256), 256, 0, st, b->f64, b->i32, b->capacity, keys2,
                       vals2, nb, 1.0 / eps, rec, precision == FGA_FP64 ? nullptr : ev + 2);
    FGA_LAUNCH_CHECK();
    if (precision != FGA_FP64) {
      hipLaunchKernelGGL(k_mx_records, (unsigned)((nb + 255) / 256), 256, 0, st, rec, keys2, nb, ev + 2);
      FGA_LAUNCH_CHECK();
    }
  }
  hipLaunchKernelGGL(k_cell_start, (unsigned)((ncells + 1 + 255) / 256), 256, 0, st, keys2, nb, (int32_t)ncells,
                     start);
  FGA_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_tile_counts, (unsigned)((ntile + 255) / 256), 256, 0, st, g, start, tcount);
  FGA_LAUNCH_CHECK();
  std::vector<int64_t> hc(ntile);
  FGA_HIP(hipMemcpyAsync(hc.data(), tcount, ntile * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  unsigned long long hev = 0;
  FGA_HIP(hipMemcpyAsync(&hev, ev, sizeof(hev), hipMemcpyDeviceToHost, st));
  FGA_HIP(hipStreamSynchronize(st));
  if (evals_out) *evals_out = (int64_t)hev;

  int64_t total = 0;
  for (int t = 0; t < ntile; ++t) total += hc[t];
  int64_t seg = (total + nseg - 1) / nseg;
  if (seg < 64) seg = 64;
  seg = (seg + NB - 1) / NB * NB;
  std::vector<Item> hi;
  std::vector<int32_t> hf(ntile), hn(ntile);
  for (int t = 0; t < ntile; ++t) {
    hf[t] = (int32_t)hi.size();
    for (int64_t k = 0; k < hc[t]; k += seg) hi.push_back(Item{t, 0, k, k + seg < hc[t] ? k + seg : hc[t]});
    hn[t] = (int32_t)hi.size() - hf[t];
  }
  if ((int)hi.size() > max_items) return fail(FGA_EDEVICE, "internal: %zu work items > %d", hi.size(), max_items);
  // launch order: the longest items first, so that the short ones fill the
  // tail of the launch (greedy longest-processing-time scheduling)
  std::vector<int32_t> hs(hi.size());
  for (size_t k = 0; k < hi.size(); ++k) hs[k] = (int32_t)k;
  std::stable_sort(hs.begin(), hs.end(),
                   [&](int32_t a, int32_t b) { return hi[a].k1 - hi[a].k0 > hi[b].k1 - hi[b].k0; });
  if (!hi.empty()) {
    FGA_HIP(hipMemcpyAsync(items, hi.data(), hi.size() * sizeof(Item), hipMemcpyHostToDevice, st));
    FGA_HIP(hipMemcpyAsync(sched, hs.data(), hs.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
  }
  FGA_HIP(hipMemcpyAsync(first, hf.data(), ntile * sizeof(int32_t), hipMemcpyHostToDevice, st));
  FGA_HIP(hipMemcpyAsync(nitems, hn.data(), ntile * sizeof(int32_t), hipMemcpyHostToDevice, st));
  if (!hi.empty()) {
    ProfScope prof(FGA_K_GRID_TILE, st);
    const unsigned nwg = (unsigned)hi.size();
    switch (precision) {
      case FGA_FP64:
        hipLaunchKernelGGL(k_grid_tile<PolF64>, nwg * PolF64::SPLIT, 256, 0, st, g, start, items, sched, rec, partial,
                           ev + 1, nullptr);
        break;
      case FGA_FP32:
        hipLaunchKernelGGL(k_grid_tile<PolMx<FGA_FP32>>, nwg, 256, 0, st, g, start, items, sched, rec, partial,
                           ev + 1, ev + 2);
        break;
      case FGA_BF16X3:
        hipLaunchKernelGGL(k_grid_tile<PolMx<FGA_BF16X3>>, nwg, 256, 0, st, g, start, items, sched, rec, partial,
                           ev + 1, ev + 2);
        break;
      case FGA_FP16X3:
        hipLaunchKernelGGL(k_grid_tile<PolMx<FGA_FP16X3>>, nwg, 256, 0, st, g, start, items, sched, rec, partial,
                           ev + 1, ev + 2);
        break;
      default:
        hipLaunchKernelGGL(k_grid_tile<PolMx<FGA_FP16X2>>, nwg, 256, 0, st, g, start, items, sched, rec, partial,
                           ev + 1, ev + 2);
        break;
    }
    FGA_LAUNCH_CHECK();
  }
  const int64_t plane = (int64_t)n[0] * n[1] * n[2];
  hipLaunchKernelGGL(k_grid_reduce, (unsigned)((3 * plane + 255) / 256), 256, 0, st, g, first, nitems, partial, out,
                     add ? 1 : 0);
  FGA_LAUNCH_CHECK();
  // the host vectors above must outlive the copies that read them
  FGA_HIP(hipStreamSynchronize(st));
  return FGA_OK;
}

}  // namespace fga
