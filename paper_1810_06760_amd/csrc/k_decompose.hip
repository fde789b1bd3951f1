// Step 1 (Sec. 2.1, eq:psi, eq:alpha^k): FBI projection of the initial data
// onto Gaussian packets and creation of the beam set.
//
// The FBI kernel exp(-i p.(y-q)/eps - |y-q|^2/(2 eps)) is a product of three
// one-dimensional factors K_d[(q_d, p_d), y_d], so the transform of a field
// sampled on an ny^3 mesh is three mode products (batched complex GEMMs):
//   T1[c][z][y][a]  = sum_x f[c][z][y][x] Kx[a][x]
//   T2[c][z][b][a]  = sum_y Ky[b][y] T1[c][z][y][a]
//   Ft[c][g][b][a]  = sum_z Kz[g][z] T2[c][z][b][a]
// with a, b, g the (q, p) pair index of each axis (a = iq*np + ip).  Beams
// are then made per candidate lineage number, culled by |psi| and written in
// lineage order with an order-preserving compaction.
#include "device_common.h"

namespace fga {
namespace {

constexpr double COS20 = 0.93969262078590838405;  // cos(20 degrees)

// K[(iq*np + ip)][iy] = yh * exp(-i p (y - q)/eps - (y - q)^2/(2 eps))
__global__ __launch_bounds__(256) void k_fbi_table(int nq, double qlo, double qh, int np, double plo, double ph,
                                                   int ny, double ylo, double yh, double eps,
                                                   double2 *__restrict__ K)
{
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= (int64_t)nq * np * ny) return;
  const int iy = (int)(id % ny);
  const int pair = (int)(id / ny);
  const int iq = pair / np, ip = pair % np;
  const double q = qlo + iq * qh, p = plo + ip * ph, y = ylo + iy * yh;
  const double u = y - q;
  double s, c;
  sincos(-p * u / eps, &s, &c);
  const double m = yh * exp(-u * u / (2.0 * eps));
  K[id] = make_double2(m * c, m * s);
}

struct GemmDesc {
  int64_t M, N, K;
  int64_t sAi, sAk, sBk, sBj, sCi, sCj;
  int64_t bA, bB, bC;
};

// C = A B for complex matrices given by element strides, batched over blockIdx.z.
__global__ __launch_bounds__(256) void k_cgemm(const double2 *__restrict__ A, const double2 *__restrict__ B,
                                               double2 *__restrict__ C, GemmDesc d)
{
  __shared__ double2 As[16][17], Bs[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t i = (int64_t)blockIdx.y * 16 + ty, j = (int64_t)blockIdx.x * 16 + tx;
  A += d.bA * blockIdx.z;
  B += d.bB * blockIdx.z;
  C += d.bC * blockIdx.z;
  double cr = 0.0, ci = 0.0;
  for (int64_t k0 = 0; k0 < d.K; k0 += 16) {
    As[ty][tx] = (i < d.M && k0 + tx < d.K) ? A[i * d.sAi + (k0 + tx) * d.sAk] : make_double2(0.0, 0.0);
    Bs[ty][tx] = (k0 + ty < d.K && j < d.N) ? B[(k0 + ty) * d.sBk + j * d.sBj] : make_double2(0.0, 0.0);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const double2 a = As[ty][kk], b = Bs[kk][tx];
      cr += a.x * b.x - a.y * b.y;
      ci += a.x * b.y + a.y * b.x;
    }
    __syncthreads();
  }
  if (i < d.M && j < d.N) C[i * d.sCi + j * d.sCj] = make_double2(cr, ci);
}

// h_b(y) = g(y) / c_b(y) on the quadrature mesh, for b = P (out[0]) and S (out[1]).
template <int MK>
__global__ __launch_bounds__(256) void k_div_speed(DevMedium med, const double2 *__restrict__ g, int nx, int ny,
                                                   int nz, double xlo, double ylo, double zlo, double hx,
                                                   double hy, double hz, double2 *__restrict__ out)
{
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t plane = (int64_t)nx * ny * nz;
  if (id >= plane) return;
  const int i = (int)(id % nx), j = (int)((id / nx) % ny), k = (int)(id / ((int64_t)nx * ny));
  const double x[3] = {xlo + i * hx, ylo + j * hy, zlo + k * hz};
  int layer = 0;
  if (MK == MK_LAYERED) {
    if (med.geometry == 1) {
      const double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
      while (layer < med.nlayer - 1 && r < med.bound[layer]) ++layer;
    } else {
      while (layer < med.nlayer - 1 && x[2] > med.bound[layer]) ++layer;
    }
  }
  for (int sp = 0; sp < 2; ++sp) {
    double c, gr[3], H[6];
    medium_eval<MK>(med, sp, layer, x, c, gr, H);
    for (int comp = 0; comp < 3; ++comp) {
      const double2 v = g[comp * plane + id];
      out[(sp * 3 + comp) * plane + id] = make_double2(v.x / c, v.y / c);
    }
  }
}

struct BeamInit {
  int nq[3], np[3];
  double qlo[3], qh[3], plo[3], ph[3];
  int64_t Nq, Np, ncand;
  int mask, one_way;
  int merge;                // one S beam per (q, p, direction): SH candidates carry the SV term too
  double cull, eps, norm;
  const double2 *Ft, *Gt;   // [3][plane] and [2][3][plane]
  int64_t plane;
  int na[3];
  int geometry, nlayer;
  double bound[FGA_MAX_LAYERS];
};

// psi of candidate lineage L; returns false if L is not a candidate.  With
// a.merge the SV candidates are not candidates, and an SH candidate also
// returns the psi of its SV partner (s2r, s2i) for the merged beam.
__device__ __forceinline__ bool candidate_psi(const BeamInit &a, int64_t L, double q[3], double p[3],
                                              double e[3], double &psr, double &psi, double &s2r, double &s2i,
                                              int &br, int &sg)
{
  br = (int)(L / (2 * a.Np * a.Nq));
  const int dir = (int)((L / (a.Np * a.Nq)) % 2);
  const int64_t ip = (L / a.Nq) % a.Np, iq = L % a.Nq;
  if (!((a.mask >> br) & 1) || (a.one_way && dir == 1) || (a.merge && br == 2)) return false;
  sg = dir == 0 ? 1 : -1;
  int iqd[3] = {(int)(iq % a.nq[0]), (int)((iq / a.nq[0]) % a.nq[1]), (int)(iq / ((int64_t)a.nq[0] * a.nq[1]))};
  int ipd[3] = {(int)(ip % a.np[0]), (int)((ip / a.np[0]) % a.np[1]), (int)(ip / ((int64_t)a.np[0] * a.np[1]))};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    q[d] = a.qlo[d] + iqd[d] * a.qh[d];
    p[d] = a.plo[d] + ipd[d] * a.ph[d];
  }
  const int64_t ax = (int64_t)iqd[0] * a.np[0] + ipd[0];
  const int64_t ay = (int64_t)iqd[1] * a.np[1] + ipd[1];
  const int64_t az = (int64_t)iqd[2] * a.np[2] + ipd[2];
  const int64_t idx = (az * a.na[1] + ay) * a.na[0] + ax;
  const double pn = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
  // initial frame axis: e_z unless p is within 20 degrees of it, then e_x
  const bool near_z = fabs(p[2]) / pn > COS20;
  e[0] = near_z ? 1.0 : 0.0;
  e[1] = 0.0;
  e[2] = near_z ? 0.0 : 1.0;
  double n[3], n2[3] = {0.0, 0.0, 0.0};
  if (br == 0) {
    n[0] = p[0] / pn; n[1] = p[1] / pn; n[2] = p[2] / pn;
  } else {
    double nsh[3], nsv[3];
    s_frame(p, e, nsh, nsv);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      n[d] = br == 1 ? nsh[d] : nsv[d];
      n2[d] = nsv[d];
    }
  }
  // psi for the polarisation nn (eq:psi, eq:alpha^k)
  auto project = [&](const double nn[3], double &r, double &im) {
    double fr = 0.0, fi = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double2 F = a.Ft[c * a.plane + idx];
      fr += F.x * nn[c];
      fi += F.y * nn[c];
    }
    if (a.one_way) {
      r = fr;
      im = fi;
    } else {
      r = 0.5 * fr;
      im = 0.5 * fi;
      if (a.Gt) {
        const double2 *G = a.Gt + (br == 0 ? 0 : 3) * a.plane;
        double gr = 0.0, gi = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double2 v = G[c * a.plane + idx];
          gr += v.x * nn[c];
          gi += v.y * nn[c];
        }
        // + sigma * (i eps / (2|p|)) * G.n
        const double f = sg * a.eps / (2.0 * pn);
        r += -f * gi;
        im += f * gr;
      }
    }
  };
  project(n, psr, psi);
  s2r = s2i = 0.0;
  if (a.merge && br == 1) project(n2, s2r, s2i);
  return true;
}

// Whether a candidate is kept: |psi| >= cull; a merged S candidate when
// either member's is (each member's term is then kept only if its own is).
__device__ __forceinline__ bool kept(const BeamInit &a, int br, double pr, double pi, double s2r, double s2i)
{
  const bool k1 = !(sqrt(pr * pr + pi * pi) < a.cull);
  if (!(a.merge && br == 1)) return k1;
  return k1 || !(sqrt(s2r * s2r + s2i * s2i) < a.cull);
}

__global__ __launch_bounds__(256) void k_beam_count(BeamInit a, int64_t *__restrict__ counts)
{
  const int64_t L = (int64_t)blockIdx.x * 256 + threadIdx.x;
  bool keep = false;
  if (L < a.ncand) {
    double q[3], p[3], e[3], pr, pi, s2r, s2i;
    int br, sg;
    if (candidate_psi(a, L, q, p, e, pr, pi, s2r, s2i, br, sg)) keep = kept(a, br, pr, pi, s2r, s2i);
  }
  int total;
  block_rank(keep, &total);
  if (threadIdx.x == 0) counts[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void k_beam_write(BeamInit a, const int64_t *__restrict__ offs, double *__restrict__ F,
                                                    int32_t *__restrict__ I, int64_t *__restrict__ lineage, int64_t cap)
{
  const int64_t L = (int64_t)blockIdx.x * 256 + threadIdx.x;
  bool keep = false;
  double q[3], p[3], e[3], pr = 0, pi = 0, s2r = 0, s2i = 0;
  int br = 0, sg = 1;
  if (L < a.ncand) {
    if (candidate_psi(a, L, q, p, e, pr, pi, s2r, s2i, br, sg)) keep = kept(a, br, pr, pi, s2r, s2i);
  }
  int total;
  const int r = block_rank(keep, &total);
  if (!keep) return;
  const int64_t i = offs[blockIdx.x] + r;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    F[(FGA_Q + d) * cap + i] = q[d];
    F[(FGA_P + d) * cap + i] = p[d];
    F[(FGA_E + d) * cap + i] = e[d];
  }
#pragma unroll
  for (int o = 0; o < 9; ++o) {
    const bool diag = o % 4 == 0;
    F[(FGA_ZQ_RE + o) * cap + i] = diag ? 1.0 : 0.0;
    F[(FGA_ZQ_IM + o) * cap + i] = 0.0;
    F[(FGA_ZP_RE + o) * cap + i] = 0.0;
    F[(FGA_ZP_IM + o) * cap + i] = diag ? -1.0 : 0.0;
  }
  const double a0 = 2.8284271247461900976;  // 2^{3/2}
  if (a.merge && br == 1) {
    // merged S beam: weight 1, (a_SV, a_SH) = 2^{3/2} (w_SV, w_SH) of the kept members
    const bool ksh = !(sqrt(pr * pr + pi * pi) < a.cull), ksv = !(sqrt(s2r * s2r + s2i * s2i) < a.cull);
    F[FGA_A0_RE * cap + i] = ksv ? a0 * (s2r * a.norm) : 0.0;
    F[FGA_A0_IM * cap + i] = ksv ? a0 * (s2i * a.norm) : 0.0;
    F[FGA_A1_RE * cap + i] = ksh ? a0 * (pr * a.norm) : 0.0;
    F[FGA_A1_IM * cap + i] = ksh ? a0 * (pi * a.norm) : 0.0;
    F[FGA_W_RE * cap + i] = 1.0;
    F[FGA_W_IM * cap + i] = 0.0;
  } else {
    F[FGA_A0_RE * cap + i] = br == 1 ? 0.0 : a0;
    F[FGA_A0_IM * cap + i] = 0.0;
    F[FGA_A1_RE * cap + i] = br == 1 ? a0 : 0.0;
    F[FGA_A1_IM * cap + i] = 0.0;
    F[FGA_W_RE * cap + i] = pr * a.norm;
    F[FGA_W_IM * cap + i] = pi * a.norm;
  }
  F[FGA_S * cap + i] = 0.0;
  int layer = 0;
  if (a.nlayer > 1) {
    if (a.geometry == 1) {
      const double rr = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
      while (layer < a.nlayer - 1 && rr < a.bound[layer]) ++layer;
    } else {
      while (layer < a.nlayer - 1 && q[2] > a.bound[layer]) ++layer;
    }
  }
  I[FGA_BRANCH * cap + i] = br;
  I[FGA_SIGMA * cap + i] = sg;
  I[FGA_LAYER * cap + i] = layer;
  I[FGA_GEN * cap + i] = 0;
  I[FGA_FLAGS * cap + i] = FGA_FLAG_ALIVE;
  lineage[i] = L;
}

struct FbiPlan {
  int na[3];
  int64_t t1, t2, ft, tab[3];
};

FbiPlan fbi_plan(const fga_mesh *m)
{
  FbiPlan p;
  for (int d = 0; d < 3; ++d) {
    p.na[d] = m->nq[d] * m->np[d];
    p.tab[d] = (int64_t)p.na[d] * m->ny[d];
  }
  p.t1 = 3LL * m->ny[2] * m->ny[1] * p.na[0];
  p.t2 = 3LL * m->ny[2] * p.na[1] * p.na[0];
  p.ft = 3LL * p.na[2] * p.na[1] * p.na[0];
  return p;
}

hipError_t gemm(const double2 *A, const double2 *B, double2 *C, const GemmDesc &d, int64_t batch, hipStream_t st)
{
  dim3 grid((unsigned)((d.N + 15) / 16), (unsigned)((d.M + 15) / 16), (unsigned)batch);
  ProfScope prof(FGA_K_FBI_GEMM, st);
  hipLaunchKernelGGL(k_cgemm, grid, 256, 0, st, A, B, C, d);
  return hipGetLastError();
}

// FBI transform of a [3][nz][ny][nx] complex field into out [3][g][b][a].
hipError_t fbi3(const fga_mesh *m, const FbiPlan &pl, double2 *const K[3], const double2 *f, double2 *T1,
                double2 *T2, double2 *out, hipStream_t st)
{
  const int64_t nx = m->ny[0], ny = m->ny[1], nz = m->ny[2];
  const int64_t na = pl.na[0], nb = pl.na[1], ng = pl.na[2];
  hipError_t e;
  {  // T1[(c,z,y)][a] = sum_x f[(c,z,y)][x] Kx[a][x]
    GemmDesc d{3 * nz * ny, na, nx, nx, 1, 1, nx, na, 1, 0, 0, 0};
    if ((e = gemm(f, K[0], T1, d, 1, st)) != hipSuccess) return e;
  }
  {  // per (c,z): T2[b][a] = sum_y Ky[b][y] T1[y][a]
    GemmDesc d{nb, na, ny, ny, 1, na, 1, na, 1, 0, ny * na, nb * na};
    if ((e = gemm(K[1], T1, T2, d, 3 * nz, st)) != hipSuccess) return e;
  }
  {  // per c: Ft[g][(b,a)] = sum_z Kz[g][z] T2[z][(b,a)]
    GemmDesc d{ng, nb * na, nz, nz, 1, nb * na, 1, nb * na, 1, 0, nz * nb * na, ng * nb * na};
    if ((e = gemm(K[2], T2, out, d, 3, st)) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

int64_t decompose_candidates(const fga_mesh *m)
{
  const int64_t Nq = (int64_t)m->nq[0] * m->nq[1] * m->nq[2];
  const int64_t Np = (int64_t)m->np[0] * m->np[1] * m->np[2];
  return 6 * Nq * Np;
}

fga_status decompose_impl(const DevMedium &dm, const fga_mesh *m, const double *f, const double *g,
                          fga_beams *beams, Arena &ar, hipStream_t st, bool size_only, size_t *need)
{
  const FbiPlan pl = fbi_plan(m);
  const int64_t plane_y = (int64_t)m->ny[0] * m->ny[1] * m->ny[2];
  double2 *K[3];
  for (int d = 0; d < 3; ++d) K[d] = ar.take<double2>(pl.tab[d]);
  double2 *T1 = ar.take<double2>(pl.t1);
  double2 *T2 = ar.take<double2>(pl.t2);
  double2 *Ft = ar.take<double2>(pl.ft);
  double2 *Gt = nullptr, *gdiv = nullptr;
  const bool use_g = g != nullptr && !m->one_way;
  if (use_g) {
    Gt = ar.take<double2>(2 * pl.ft);
    gdiv = ar.take<double2>(6 * plane_y);
  }
  const int64_t ncand = decompose_candidates(m);
  const int64_t nblk = (ncand + 255) / 256;
  int64_t *counts = ar.take<int64_t>(nblk + 1);
  int64_t *offs = ar.take<int64_t>(nblk + 1);
  int64_t *total = ar.take<int64_t>(1);
  if (size_only) {
    *need = ar.used;
    return FGA_OK;
  }
  if (!counts || !offs || !total || !Ft || !T1 || !T2 || !K[0] || !K[1] || !K[2] || (use_g && (!Gt || !gdiv)))
    return fail(FGA_ENOMEM, "decompose workspace too small (%zu bytes given)", ar.size);

  for (int d = 0; d < 3; ++d) {
    hipLaunchKernelGGL(k_fbi_table, (unsigned)((pl.tab[d] + 255) / 256), 256, 0, st, m->nq[d], m->qlo[d], m->qh[d],
                       m->np[d], m->plo[d], m->ph[d], m->ny[d], m->ylo[d], m->yh[d], m->eps, K[d]);
    FGA_LAUNCH_CHECK();
  }
  FGA_HIP(fbi3(m, pl, K, reinterpret_cast<const double2 *>(f), T1, T2, Ft, st));
  if (use_g) {
    const unsigned blocks = (unsigned)((plane_y + 255) / 256);
    auto dv = [&](auto kern) {
      hipLaunchKernelGGL(kern, blocks, 256, 0, st, dm, reinterpret_cast<const double2 *>(g), m->ny[0], m->ny[1],
                         m->ny[2], m->ylo[0], m->ylo[1], m->ylo[2], m->yh[0], m->yh[1], m->yh[2], gdiv);
    };
    if (dm.kind == FGA_MEDIUM_HOMOGENEOUS) dv(k_div_speed<MK_HOMOG>);
    else if (dm.kind == FGA_MEDIUM_GRID && dm.smooth) dv(k_div_speed<MK_GRID3>);
    else if (dm.kind == FGA_MEDIUM_GRID) dv(k_div_speed<MK_GRID>);
    else dv(k_div_speed<MK_LAYERED>);
    FGA_LAUNCH_CHECK();
    FGA_HIP(fbi3(m, pl, K, gdiv, T1, T2, Gt, st));
    FGA_HIP(fbi3(m, pl, K, gdiv + 3 * plane_y, T1, T2, Gt + pl.ft, st));
  }

  BeamInit a{};
  for (int d = 0; d < 3; ++d) {
    a.nq[d] = m->nq[d]; a.np[d] = m->np[d];
    a.qlo[d] = m->qlo[d]; a.qh[d] = m->qh[d];
    a.plo[d] = m->plo[d]; a.ph[d] = m->ph[d];
    a.na[d] = pl.na[d];
  }
  a.Nq = (int64_t)m->nq[0] * m->nq[1] * m->nq[2];
  a.Np = (int64_t)m->np[0] * m->np[1] * m->np[2];
  a.ncand = ncand;
  a.mask = m->branch_mask;
  a.one_way = m->one_way;
  a.merge = m->merge_s && (m->branch_mask & 6) == 6;
  a.cull = m->cull_abs;
  a.eps = m->eps;
  const double dq = m->qh[0] * m->qh[1] * m->qh[2];
  const double dp = m->ph[0] * m->ph[1] * m->ph[2];
  a.norm = dq * dp * std::pow(2.0 * M_PI * m->eps, -4.5);
  a.Ft = Ft;
  a.Gt = use_g ? Gt : nullptr;
  a.plane = pl.ft / 3;
  a.geometry = dm.kind == FGA_MEDIUM_LAYERED ? dm.geometry : 0;
  a.nlayer = dm.kind == FGA_MEDIUM_LAYERED ? dm.nlayer : 1;
  for (int l = 0; l < FGA_MAX_LAYERS; ++l) a.bound[l] = dm.bound[l];

  hipLaunchKernelGGL(k_beam_count, (unsigned)nblk, 256, 0, st, a, counts);
  FGA_LAUNCH_CHECK();
  FGA_HIP(launch_scan(counts, offs, nblk, total, st));
  int64_t made = 0;
  FGA_HIP(hipMemcpyAsync(&made, total, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  FGA_HIP(hipStreamSynchronize(st));
  if (made > beams->capacity)
    return fail(FGA_ECAPACITY, "decomposition makes %lld beams but capacity is %lld", (long long)made,
                (long long)beams->capacity);
  hipLaunchKernelGGL(k_beam_write, (unsigned)nblk, 256, 0, st, a, offs, beams->f64, beams->i32, beams->lineage,
                     beams->capacity);
  FGA_LAUNCH_CHECK();
  beams->count = made;
  return FGA_OK;
}

}  // namespace fga
