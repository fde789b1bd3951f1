/*
 * fga.h -- C ABI of the MI355X (gfx950) frozen Gaussian approximation library.
 *
 * The library computes the frozen Gaussian approximation (FGA) of the 3-D
 * isotropic elastic wave equation of Hateley, Chai, Tong and Yang, "Frozen
 * Gaussian Approximation for 3-D Elastic Wave Equation and Seismic Tomography"
 * (Sec. 2, eq:ewe with F = 0 and initial data eq:ini).  Its three calls follow
 * the three steps of the method (Sec. 2.2, the algorithm and Fig. 1):
 *   fga_decompose          Step 1: FBI projection of the initial data onto
 *                          P/SH/SV Gaussian packets ("beams")          (eq:psi, eq:alpha^k)
 *   fga_evolve             Step 2: RK4 of each beam's ray, Jacobians, amplitudes
 *                          and action; optional seismogram sampling    (eq:char_plus/minus, eq:DzDt,
 *                                                                      eq:amp_P/SV/SH)
 *   fga_reconstruct_points Step 3: Gaussian summation at points        (eq:FGA)
 *   fga_reconstruct_grid   Step 3 on a uniform grid                    (eq:FGA)
 *
 * Conventions (all calls):
 *  - Every pointer marked "device" must be device memory of the current HIP
 *    device; the library never frees caller memory and keeps no pointer after
 *    a call returns.  Work is enqueued on `stream` (a hipStream_t, NULL = the
 *    default stream); a call returns once its work is enqueued unless noted.
 *  - Complex numbers are interleaved (re, im) doubles.  3-D arrays are
 *    [z][y][x] with x fastest; vector fields are [component][z][y][x].
 *  - A uniform mesh is given per axis by (n, lo, h): points lo + i*h.
 *  - k = 1/eps is the paper's large wave number.
 *  - Calls return FGA_OK or an error code; fga_last_error() then describes
 *    the failure (thread-local).  On error, outputs are unspecified, caller
 *    buffers stay valid and the beam set is unchanged unless noted.
 *  - No call allocates device memory except where a workspace query says 0
 *    and the caller passes none; every workspace-taking call states its size
 *    through the matching *_workspace_bytes query.
 */
#ifndef FGA_H
#define FGA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FGA_OK = 0,
  FGA_EINVAL = 1,       /* invalid argument (shape, size, pointer, option)         */
  FGA_ENOMEM = 2,       /* workspace too small                                      */
  FGA_EDEVICE = 3,      /* a HIP runtime call failed                                */
  FGA_ENUMERIC = 4,     /* non-finite values detected                               */
  FGA_ECAPACITY = 5,    /* beam capacity exceeded (children would not fit)          */
  FGA_EUNSUPPORTED = 6  /* option combination not implemented                       */
} fga_status;

/* Message describing the last failing call on this host thread. */
const char *fga_last_error(void);
/* Library version string. */
const char *fga_version(void);

/* ------------------------------------------------------------------------ */
/* Beam state                                                               */
/* ------------------------------------------------------------------------ */

/* Beams are held as structure-of-arrays planes in caller device memory.
 * f64 holds FGA_NF64 planes of `capacity` doubles; plane p of beam i is
 * f64[p*capacity + i].  i32 holds FGA_NI32 int32 planes likewise, lineage
 * one int64 per slot.  Live beams occupy slots [0, count).
 *
 * Meaning of the double planes (paper notation, eq:FGA and Sec. 2.2):
 *   Q[3], P[3]         packet centre and propagation vector
 *   ZQ_RE[9], ZQ_IM[9] dzQ, element (m, j) = d Q_j / d z_m at index 3m+j,
 *                      with d/dz = d/dq - i d/dp (eq:op_zZ_app)
 *   ZP_RE[9], ZP_IM[9] dzP, same layout
 *   A0, A1 (re, im)    amplitudes: P beams a_P, 0; S beams a_SV, a_SH
 *   S                  action (stays ~0: H is homogeneous of degree 1 in P)
 *   W (re, im)         psi * dq * dp * (k/2pi)^{9/2}, the beam's fixed weight
 *   E[3]               reference axis of the S polarisation frame
 *                      N_SH = (E x P)/|E x P|, N_SV = (P/|P|) x N_SH
 * int32 planes: BRANCH (0 P, 1 SH, 2 SV; beams made at interfaces are 0 or
 *   2), SIGMA (+1 "+" flow, -1 "-" flow), LAYER (layered media), GEN
 *   (interface generation), FLAGS (bit 0 alive, bit 1 quarantined: non-finite
 *   state, bit 2 internal: crossed an interface during the current step).
 * lineage: canonical number ((branch*2 + dir)*Np + ip)*Nq + iq of the mesh
 *   point a generation-0 beam came from.  A beam of generation g made at an
 *   interface as mode k (0 P reflected, 1 S reflected, 2 P transmitted,
 *   3 S transmitted) of its parent gets
 *   (g << 58) | ((parent & (2^58 - 1)) << 2) | k
 *   (FGA_LINEAGE_CHILD), so lineages stay unique and name the path. */
enum {
  FGA_Q = 0, FGA_P = 3,
  FGA_ZQ_RE = 6, FGA_ZQ_IM = 15, FGA_ZP_RE = 24, FGA_ZP_IM = 33,
  FGA_A0_RE = 42, FGA_A0_IM = 43, FGA_A1_RE = 44, FGA_A1_IM = 45,
  FGA_S = 46, FGA_W_RE = 47, FGA_W_IM = 48, FGA_E = 49,
  FGA_NF64 = 52
};
enum { FGA_BRANCH = 0, FGA_SIGMA = 1, FGA_LAYER = 2, FGA_GEN = 3, FGA_FLAGS = 4, FGA_NI32 = 5 };
enum { FGA_FLAG_ALIVE = 1, FGA_FLAG_QUARANTINED = 2, FGA_FLAG_CROSS = 4 };
#define FGA_LINEAGE_CHILD(parent, gen_parent, k)                                   \
  ((((int64_t)(gen_parent) + 1) << 58) | (((int64_t)(parent) & ((INT64_C(1) << 58) - 1)) << 2) | (int64_t)(k))

typedef struct {
  int64_t capacity;   /* slots per plane                                         */
  int64_t count;      /* live beams occupy [0, count); updated by the calls      */
  double *f64;        /* device, FGA_NF64 * capacity doubles                     */
  int32_t *i32;       /* device, FGA_NI32 * capacity int32                       */
  int64_t *lineage;   /* device, capacity int64                                  */
} fga_beams;

/* Counts over the beams [0, count) of a set (flags, branch and generation
 * planes), for monitoring a run and checking a checkpoint. */
typedef struct {
  int64_t count;          /* beams in [0, count)                                      */
  int64_t alive;          /* FGA_FLAG_ALIVE set                                       */
  int64_t quarantined;    /* FGA_FLAG_QUARANTINED set                                 */
  int64_t by_branch[3];   /* alive beams per branch (0 P, 1 SH or merged S, 2 SV)     */
  int64_t children;       /* alive beams made at an interface (generation > 0)        */
} fga_beams_stats;

#define FGA_BEAMS_INFO_WORKSPACE 64   /* bytes of device workspace fga_beams_info needs */

/* Fills *out (synchronises `stream`).  workspace: device, at least
 * FGA_BEAMS_INFO_WORKSPACE bytes, 8-byte aligned.
 * Errors: FGA_EINVAL (NULL or inconsistent set, short workspace). */
fga_status fga_beams_info(const fga_beams *beams, fga_beams_stats *out, void *workspace,
                          size_t workspace_bytes, void *stream);

/* Copies the beams [0, count) out of a set, plane by plane: f64[f * count + i]
 * (f < FGA_NF64), i32[f * count + i] (f < FGA_NI32), lineage[i].  The
 * destinations may be host or device memory (any of them NULL: that part is
 * not copied); the layout is the planes' own, so a checkpoint is the three
 * arrays and the count.  Synchronises `stream`.  Errors: FGA_EINVAL. */
fga_status fga_beams_export(const fga_beams *beams, double *f64, int32_t *i32, int64_t *lineage, void *stream);

/* Sets a set's beams [0, n) from arrays in the layout fga_beams_export writes
 * (host or device; count = n, so the rest of the planes is unused).
 * Synchronises `stream`.  Errors: FGA_EINVAL (NULL arrays), FGA_ECAPACITY
 * (n > capacity). */
fga_status fga_beams_import(fga_beams *beams, int64_t n, const double *f64, const int32_t *i32,
                            const int64_t *lineage, void *stream);

/* ------------------------------------------------------------------------ */
/* Media (Sec. 2, eq:ps_speed; Sec. 3.1 for layers)                          */
/* ------------------------------------------------------------------------ */

typedef enum {
  FGA_MEDIUM_HOMOGENEOUS = 0,  /* constant c_P, c_S                                   */
  FGA_MEDIUM_GRID = 1,         /* periodic node grid: trilinear interpolation of c and
                                  of its central-difference gradient and Hessian, or
                                  (smooth = 1) the periodic cubic B-spline through the
                                  node values with its exact derivatives               */
  FGA_MEDIUM_LAYERED = 2       /* flat layers in z or concentric spherical shells, the
                                  speeds constant or linear in the level per layer     */
} fga_medium_kind;

#define FGA_MAX_LAYERS 8
#define FGA_GRID_NODE_DOUBLES 16  /* doubles per node per speed field in a grid table */

typedef struct {
  int kind;                /* fga_medium_kind                                          */
  double cp, cs, rho;      /* homogeneous speeds and density                           */
  /* FGA_MEDIUM_GRID: nodes lo + i*h (i = 0..n-1), periodic with period n*h.          */
  int n[3];
  double lo[3], h[3];
  const double *table;     /* device, built by fga_medium_grid_build                    */
  int two_fields;          /* 1: table holds a c_P field then a c_S field;
                              0: one c_P field and c_S = cs_ratio * c_P                */
  double cs_ratio;
  /* FGA_MEDIUM_LAYERED: geometry 0: layer i is z in (bound[i-1], bound[i]) (layer 0
     below bound[0]); geometry 1: layer i is |x| in (bound[i], bound[i-1]) (layer 0
     outermost, radii descending).                                                     */
  int geometry;
  int nlayer;
  double bound[FGA_MAX_LAYERS];
  double cpl[FGA_MAX_LAYERS], csl[FGA_MAX_LAYERS], rhol[FGA_MAX_LAYERS];
  /* relative gradient per layer: c_b(x) = c_b,l (1 + gradl[l] v(x)), v = z (geometry 0)
     or |x| (geometry 1); 0 for a constant layer.  In a gradient layer rays bend and
     the crossing is found by secant iterations on RK4 sub-steps (Sec. 3.1).  The
     innermost spherical layer must be constant (|x| is not smooth at the centre);
     the speed must stay positive where beams go (not checked).                      */
  double gradl[FGA_MAX_LAYERS];
  /* Gaussian anomaly per layer (the low-velocity region of the crosswell model,
     Sec. 4 eq:true_c): in layer l the speeds are multiplied by
     1 - anom_amp[l] exp(-anom_beta[l] sum_d anom_w[l][d] (x_d - anom_x[l][d])^2);
     a weight 0 drops an axis (the model is invariant along it).  anom_amp[l] = 0:
     none.  Rays in such a layer curve: the general step and the secant crossing of
     gradient layers are used.  The factor must stay positive (not checked).          */
  double anom_amp[FGA_MAX_LAYERS], anom_beta[FGA_MAX_LAYERS];
  double anom_x[FGA_MAX_LAYERS][3], anom_w[FGA_MAX_LAYERS][3];
  /* > 0: a traction-free surface closing the outermost region, |x| = surface around
     layer 0 (geometry 1) or z = surface above the last layer (geometry 0): a beam
     reaching it is split into the reflected P and S beams of the free-surface
     problem (sigma.n = 0); 0: no surface (the outermost layer extends without end).
     Beams must start inside the surface.                                            */
  double surface;
  /* FGA_MEDIUM_GRID: 0: trilinear interpolation of the derived node fields (C^0);
     1: c is the periodic cubic B-spline through the node values (C^2), its gradient
     and Hessian the exact derivatives of the spline.  Both read the same table.     */
  int smooth;
} fga_medium;

/* Bytes of the table of a grid medium with N = n[0]*n[1]*n[2] nodes: per node
 * field (c_P, then c_S if two_fields) N records of FGA_GRID_NODE_DOUBLES
 * doubles, then per node field the N cubic B-spline coefficients. */
size_t fga_medium_grid_table_bytes(const int n[3], int two_fields);

/* Builds the table of a gridded medium (Sec. 2: the ray and variational
 * equations need c, grad c and its Hessian of a smooth medium; the paper gives
 * no discretisation of gridded media, these are the readings the library
 * uses): for each node field
 *   - per node c, grad c (3), Hessian (xx, yy, zz, xy, xz, yz) by second-order
 *     periodic central differences (slots 0..9 of the node record), read by
 *     trilinear interpolation when the medium's smooth = 0;
 *   - the coefficients a of the periodic cubic B-spline that takes the node
 *     values, (a[i-1] + 4 a[i] + a[i+1]) / 6 = c[i] along each axis in turn,
 *     by the recursive filter of the spline's two poles with periodic start
 *     values (Unser, Aldroubi and Eden, IEEE Trans. Signal Process. 41, 1993),
 *     read when smooth = 1.
 * cp_nodes, cs_nodes (NULL unless two_fields): device, [z][y][x].
 * table: device, fga_medium_grid_table_bytes(n, cs_nodes != NULL) bytes.
 * Errors: FGA_EINVAL for n < 3 or non-positive h or NULL pointers. */
fga_status fga_medium_grid_build(const int n[3], const double h[3], const double *cp_nodes,
                                 const double *cs_nodes, double *table, void *stream);

/* ------------------------------------------------------------------------ */
/* Step 1: decomposition (Sec. 2.1 eq:psi, eq:alpha^k; Sec. 2.2 Step 1)      */
/* ------------------------------------------------------------------------ */

typedef struct {
  double eps;              /* 1/k                                                     */
  int nq[3]; double qlo[3], qh[3];   /* q mesh (Gaussian centres)                      */
  int np[3]; double plo[3], ph[3];   /* p mesh (propagation vectors); |p| > 0          */
  int ny[3]; double ylo[3], yh[3];   /* quadrature mesh on which f (and g) are given    */
  int branch_mask;         /* bit b set: make branch b (0 P, 1 SH, 2 SV)               */
  int one_way;             /* 1: only "+" beams, psi = FBI[f].n (f is taken as the
                              "+"-going part); 0: "+" and "-" beams per eq:alpha^k     */
  double cull_abs;         /* beams with |psi| < cull_abs are not created             */
  /* 1 (with branch bits 1 and 2 set): one S beam per (q, p, direction) in place of
     the SH and SV pair.  Both members start from the same data and move with c_S,
     so their rays coincide, and the S amplitude equations (eq:amp_SV, eq:amp_SH) and
     the interface split are linear: the pair's field is that of one beam on the
     common ray with weight 1 and (a_SV, a_SH) = 2^{3/2} (w_SV, w_SH), a member's
     term kept only if its own |psi| passes the cull.  The beam has the SH lineage
     and branch 1; the S work per (q, p) is halved.  0: the pair as two beams.     */
  int merge_s;
} fga_mesh;

/* Workspace bytes fga_decompose needs for this mesh (with_g: g != NULL). */
size_t fga_decompose_workspace_bytes(const fga_mesh *mesh, int with_g);
/* Number of candidate beams (upper bound of the beams made). */
int64_t fga_decompose_candidates(const fga_mesh *mesh);

/* psi_{b,+-}(q,p) = (1/2) FBI[f](q,p).n_b +- (i eps/(2|p|)) FBI[g/c_b](q,p).n_b,
 * FBI[h](q,p) = sum_y yh^3 h(y) exp(-i p.(y-q)/eps - |y-q|^2/(2 eps)),
 * (eq:psi with eq:alpha^k read with prefactor 1/(2kc|p|), the normalisation
 * under which eq:FGA returns f at t = 0), then w = psi dq dp (2 pi eps)^{-9/2},
 * Q = q, P = p, dzQ = I, dzP = -iI, a = 2^{3/2} on the beam's own polarisation,
 * S = 0.  One-way mode: psi_{b,+} = FBI[f].n_b.  Beams are written in lineage
 * order (stable), replacing the previous contents; beams->count is set (this
 * call synchronises `stream` to read it back).
 * f, g: device, complex [3][ny2][ny1][ny0]; g may be NULL (g = 0).
 * Errors: FGA_EINVAL (mesh sizes, |p| = 0 on the mesh, NULL f),
 *         FGA_ENOMEM (workspace), FGA_ECAPACITY (more beams than capacity). */
fga_status fga_decompose(const fga_medium *med, const fga_mesh *mesh, const double *f,
                         const double *g, fga_beams *beams, void *workspace,
                         size_t workspace_bytes, void *stream);

/* Point moment-tensor source (the seismic examples of Sec. 3.2 and Sec. 4
 * use point sources whose decomposition the paper takes from elsewhere; the
 * reading used here): u(0) = 0, u_t(0) = g = -(1/rho0) M grad delta(x - x0),
 * whose FBI is closed-form, FBI[g/c_b](q,p) = (1/rho0) M . grad_y[K(y)/c_b(y)]
 * at y = x0 with K the FBI kernel; psi_{b,+-} = +-(i eps/(2|p|))
 * FBI[g/c_b].n_b (eq:psi, eq:alpha^k with f = 0).  Both directions and the
 * branches of branch_mask are made.  With ricker != 0 each beam's weight is
 * multiplied by R(w) = (w/w0)^2 exp(1 - (w/w0)^2) at its frequency
 * w = c_b(x0)|p|/eps, w0 = c_P(x0)/eps (zero-phase Ricker wavelet).
 * q mesh: nq^3 cell-centred points of the cube x0 +- qhalf.  p mesh per
 * branch: ndir Fibonacci directions (z_j = 1 - (2j+1)/ndir, azimuth
 * j pi (3 - sqrt 5)) times nshell Gauss-Legendre |p| shells on
 * [shell_lo, shell_hi] * c_P(x0)/c_b(x0); the p-cell measure is
 * |p|^2 w_shell 4 pi / ndir.  Lineage ((branch*2 + dir)*Np + ip)*Nq + iq with
 * ip = shell*ndir + j, iq = (iz*nq + iy)*nq + ix. */
typedef struct {
  double eps;
  double x0[3];
  double M[6];              /* symmetric moment tensor: xx, yy, zz, xy, xz, yz      */
  double rho0;              /* density at x0 (<= 0: the medium's)                    */
  int nq;
  double qhalf;
  int ndir, nshell;         /* 1 <= nshell <= 64                                     */
  double shell_lo, shell_hi;
  int ricker;
  int branch_mask;
  double cull_abs;          /* beams with |psi| < cull_abs are not made              */
  int merge_s;              /* as in fga_mesh                                         */
} fga_point_source;

int64_t fga_point_source_candidates(const fga_point_source *src);
size_t fga_decompose_point_source_workspace_bytes(const fga_point_source *src);
/* Writes the kept beams in lineage order and sets beams->count (synchronises
 * `stream`).  Errors: FGA_EINVAL, FGA_ENOMEM (workspace), FGA_ECAPACITY. */
fga_status fga_decompose_point_source(const fga_medium *med, const fga_point_source *src,
                                      fga_beams *beams, void *workspace, size_t workspace_bytes,
                                      void *stream);

/* Point force with a time function, the source of the accuracy experiment
 * of Sec. 2.3 (eq:ex_homo): rho u_tt = L u + d F(t) delta(x - x0) with
 * F(t) = cos(omega (t + t0)) exp(-(t + t0)^2 / width^2).  Reading used here
 * (the paper does not give its source treatment): by Duhamel's principle the
 * field is the superposition over source times s of free waves started with
 * u = 0, u_t = d F(s) delta(x - x0)/rho0, whose two-way weights are
 * psi_{b,+-} = +-(i eps/(2|p|)) F(s) (d.n_b)/(rho0 c_b) K(x0; q, p) (eq:psi,
 * eq:alpha^k with f = 0; K the FBI kernel).  The beam launched at time s from
 * (q, p) is represented by the beam launched at t_ref from
 * q' = q - sigma c_b(x0) (s - t_ref) p/|p| (exact for the beam centre in a
 * homogeneous medium; the amplitude's change over the source's duration is
 * left out), so each beam's weight is the integral over s of those weights,
 * a Gaussian integral done in closed form.  Evolving the beams by tau gives
 * the field at t_ref + tau.  Meshes, frames, cull (on |psi|) and lineage are
 * those of fga_point_source (q cube x0 +- qhalf; Fibonacci directions x
 * Gauss-Legendre shells on [shell_lo, shell_hi] c_P(x0)/c_b(x0)); both
 * directions and the branches of branch_mask are made.  The q cube must
 * reach as far as the wave travels during the source (about
 * 4 sqrt(eps) + 3 c_P width). */
typedef struct {
  double eps;
  double x0[3];
  double d[3];              /* force vector                                           */
  double rho0;              /* density at x0 (<= 0: the medium's)                     */
  int nq;
  double qhalf;
  int ndir, nshell;         /* 1 <= nshell <= 64                                      */
  double shell_lo, shell_hi;
  double omega, t0, width;  /* the time function F                                    */
  double t_ref;             /* the time the beams describe before any evolution      */
  int branch_mask;
  double cull_abs;
  int merge_s;              /* as in fga_mesh                                         */
} fga_point_force;

int64_t fga_point_force_candidates(const fga_point_force *src);
size_t fga_decompose_point_force_workspace_bytes(const fga_point_force *src);
/* Writes the kept beams in lineage order and sets beams->count (synchronises
 * `stream`).  Errors: FGA_EINVAL, FGA_ENOMEM (workspace), FGA_ECAPACITY. */
fga_status fga_decompose_point_force(const fga_medium *med, const fga_point_force *src, fga_beams *beams,
                                     void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Step 2: evolution (Sec. 2.2, eq:char_plus, eq:char_minus, eq:DzDt,        */
/* eq:amp_P, eq:amp_SV, eq:amp_SH; Sec. 2.3 fixed-step RK4)                  */
/* ------------------------------------------------------------------------ */

typedef enum {
  FGA_FP64 = 0, FGA_FP32 = 1, FGA_BF16X3 = 2, FGA_FP16X3 = 3, FGA_FP16X2 = 4, FGA_FP32_ACC32 = 5
} fga_precision;

enum { FGA_COORDS_CARTESIAN = 0, FGA_COORDS_SPHERICAL = 1 };

typedef struct {
  int64_t n;               /* receivers                                                */
  const double *xyz;       /* device, [n][3] positions: Cartesian (x, y, z), or with
                              coords = FGA_COORDS_SPHERICAL (r, theta, phi), theta the
                              longitude and phi the latitude, mapped by the library to
                              (r cos theta cos phi, r sin theta cos phi, r sin phi)
                              (the Earth examples' coordinates, opening of Sec. 3)    */
  int stride;              /* a sample after every `stride` steps (>= 1)               */
  double eps, tau;         /* summation: 1/k and window exp(-tau) (half-width
                              sqrt(2 tau eps) per axis)                                */
  int precision;           /* FGA_FP64: FP64 sums; FGA_FP32 (mixed): the Gaussian
                              exponent and the phase reduced modulo 2 pi in FP64, then
                              exp / sin / cos in FP32, products and sums in FP64;
                              FGA_FP32_ACC32: as FGA_FP32 with the products B e^{..}
                              and each lane's running sums in FP32 (the reductions
                              over lanes and beam ranges stay FP64)                    */
  int coords;              /* FGA_COORDS_CARTESIAN (0) or FGA_COORDS_SPHERICAL         */
} fga_receivers;

typedef struct {
  int chunk;               /* RK4 steps per integrator launch (0: library default)     */
  double cutoff_abs;       /* after every step, drop beams with |w| max(|a0|,|a1|) <
                              cutoff_abs (0: off); a dropped beam takes no further
                              step and is not summed from that step's sample on      */
  int compact;             /* 1: compact the beam set at the end of the call (stable
                              order; dead, culled and quarantined beams leave)        */
  int64_t batch;           /* beams per receiver batch (0: library default 2^22); in
                              layered media, which sum one sample per step, a batch
                              holds (chunk + stride - 1) / stride + 1 times as many  */
  int resort;              /* steps between spatial re-orderings of the beam set
                              (0: library default: with receivers in grid and
                               homogeneous media 32 for sets of 2^23 beams or more,
                               16 below, else 64; < 0: never reorder)                 */
  int gen_max;             /* layered media: interface generation cap (0: default 3)   */
  double child_cut;        /* layered media: children with |A_child| < child_cut |A_in|
                              are not made (0: default 1e-3; < 0: keep all)            */
  int s_vector;            /* 1: frame-free S amplitudes: during each integrator launch
                              an S beam carries its physical polarisation
                              A = a_SV N_SV + a_SH N_SH, advanced by
                              dA/dt = s A - (A . dPhat/dt) Phat (eq:amp_SV, eq:amp_SH
                              with the frame rotation differentiated out) and
                              projected orthogonal to P after each step; stored back
                              in the beam's frame (axis switched near P) at the end of
                              the launch.  The amplitude cutoff then uses |A|.  Agrees
                              with the framed form to RK4 truncation; identical in a
                              homogeneous medium.  Layered media: the regular steps of
                              S beams where some layer curves the rays (a gradient or
                              an anomaly); steps that reach an interface and the
                              children's partial steps stay framed.  0: framed.       */
} fga_evolve_opts;

typedef struct {
  int64_t beam_steps;      /* RK4 steps taken by live beams                            */
  int64_t evals;           /* in-window (beam, receiver, sample) terms summed          */
  int64_t culled;          /* beams dropped by the cutoff                              */
  int64_t quarantined;     /* beams dropped for non-finite state: after a step, a beam
                              whose Q, P, amplitudes or action are not finite (or whose
                              weight or frame axis is not) is flagged QUARANTINED, takes
                              no further step and is never summed                     */
  int64_t crossings;       /* interface hits (layered media)                           */
  int64_t spawned;         /* beams made at interfaces                                 */
  int64_t capped;          /* beams retired at an interface at the generation cap      */
} fga_evolve_stats;

size_t fga_evolve_workspace_bytes(const fga_beams *beams, int nsteps, const fga_evolve_opts *opts,
                                  const fga_receivers *rec);

/* Advances every live beam by nsteps classic RK4 steps of size dt, in place.
 * Unless opts->resort < 0, the beam set is first put in Morton order of the
 * beam centres Q, and again every `resort` steps: beams that share medium
 * cells then run in the same wavefronts.  Each reordering drops dead beams
 * (count shrinks); beams keep their lineage numbers, so results are matched
 * by lineage, not by slot.
 * After each step an S beam whose P has come within 10 degrees of its frame
 * axis switches axis (e_z <-> e_x) and re-expresses (a_SV, a_SH) so that the
 * physical polarisation is unchanged.  If rec != NULL, after every
 * rec->stride-th step the beams are summed at the receivers (eq:FGA with the
 * box window) into seis: device, complex [rec->n][nsteps/rec->stride][3]
 * (overwritten).  stats (host, may be NULL) receives counters; this call
 * synchronises `stream` when stats != NULL or culling is on.
 * Layered media (Sec. 3.1): the layer is beam state and the speeds are
 * constant inside a layer, so a ray is straight between interfaces.  After
 * each step a beam whose centre has left its layer is taken back to the
 * start of the step, advanced to the crossing point (theta dt, from the
 * straight ray) and put exactly on the interface; every outgoing mode that
 * propagates (eq:p:int: tangential momentum and c|P| kept) and whose
 * displacement amplitude from the elastic boundary problem (continuity of
 * displacement and traction, the physics of eq:Yilmaz) is at least
 * opts->child_cut times the incident one becomes a child with the parent's
 * weight, sigma and action, generation + 1, (dzQ, dzP) mapped by
 * eq:Inter_DzQDzP in the local tangent-normal frame, and the remaining
 * (1 - theta) dt in its own layer.  The first child takes the parent's slot,
 * the others are appended after `count` in a deterministic order; a parent at
 * the generation cap, or with no child, is retired.  The call then
 * synchronises `stream` after every step and steps one at a time.  If the
 * children would not fit in `capacity` the call stops with FGA_ECAPACITY
 * (nothing is dropped silently; the beam set is then partly advanced).
 * Errors: FGA_EINVAL, FGA_ENOMEM (workspace), FGA_ECAPACITY, FGA_EDEVICE. */
fga_status fga_evolve(const fga_medium *med, fga_beams *beams, double dt, int nsteps,
                      const fga_evolve_opts *opts, const fga_receivers *rec, double *seis,
                      void *workspace, size_t workspace_bytes, void *stream,
                      fga_evolve_stats *stats);

/* ------------------------------------------------------------------------ */
/* Step 3: reconstruction (Sec. 2.1 eq:FGA; Sec. 3 spherical coordinates)    */
/* ------------------------------------------------------------------------ */

/* u(x) = sum_b w_b exp(i S_b/eps) A_b exp(i P_b.(x-Q_b)/eps - |x-Q_b|^2/(2 eps))
 * over the beams with max_d |x_d - Q_d| <= sqrt(2 tau eps), A_b = a_P P/|P| or
 * a_SV N_SV + a_SH N_SH.  xyz: device [n][3]; out: device complex [n][3]
 * (overwritten).  precision: FGA_FP64, FGA_FP32 or FGA_FP32_ACC32 (as in
 * fga_receivers); * others give FGA_EUNSUPPORTED.  evals (host, may be NULL): number of
 * in-window terms; the call synchronises `stream` when evals != NULL. */
size_t fga_reconstruct_points_workspace_bytes(const fga_beams *beams, int64_t n);
fga_status fga_reconstruct_points(const fga_beams *beams, double eps, double tau, int64_t n,
                                  const double *xyz, int precision, double *out,
                                  void *workspace, size_t workspace_bytes, void *stream,
                                  int64_t *evals);

/* The sum of fga_reconstruct_points for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same arguments without a workspace.  Its records,
 * tile boxes, partial sums and term counter live in a fixed scratch array
 * that the library holds on each device it runs on until the process ends
 * (fga_reconstruct_points_noalloc_max_bytes() bytes, 64 MiB); the call itself
 * allocates nothing.  Beams are taken in batches of whole 64-beam tiles sized
 * so that records and partial sums fit; the points are used in the order
 * given (fga_reconstruct_points first sorts them by position, which only
 * speeds up the sum), and must be finite (not checked).  Every call on a
 * device shares that device's scratch: calls that overlap on one device (on
 * different streams or host threads) race and give wrong results.  The
 * counter is cleared by a kernel, not a memset.
 * Errors: as fga_reconstruct_points; FGA_ENOMEM when n points need more
 * scratch than the array holds even for one tile (about 1.3 million points). */
size_t fga_reconstruct_points_noalloc_max_bytes(void);
fga_status fga_reconstruct_points_noalloc(const fga_beams *beams, double eps, double tau, int64_t n,
                                          const double *xyz, int precision, double *out, void *stream,
                                          int64_t *evals);

/* The same sum on the grid points lo + i*h (i < n per axis), using the
 * separability of the window and the phase: each 16^3 tile is a complex
 * Khatri-Rao x factor product on the matrix cores.  out: device complex
 * [3][n2][n1][n0] (overwritten).  precision: FGA_FP64 (FP64 matrix cores),
 * FGA_FP32, FGA_BF16X3 or FGA_FP16X3 (split hi+lo factors, FP32 accumulation;
 * FGA_FP16X2: the Khatri-Rao rows in single FP16, the other factor split hi+lo;
 * phases reduced modulo 2 pi in FP64 before the cast).  evals (host, may be
 * NULL): algorithmic in-window (beam, point) terms. */
size_t fga_reconstruct_grid_workspace_bytes(const fga_beams *beams, const int n[3], double eps,
                                            double tau, const double h[3]);
fga_status fga_reconstruct_grid(const fga_beams *beams, double eps, double tau, const int n[3],
                                const double lo[3], const double h[3], int precision, double *out,
                                void *workspace, size_t workspace_bytes, void *stream,
                                int64_t *evals);
/* The same sum added to out (out += u) instead of overwriting it, for beam
 * sets summed in waves (Step 3 is linear in the beams, eq:FGA).  Arguments,
 * workspace and errors as fga_reconstruct_grid; out must hold the previous
 * partial sum (or zeros). */
fga_status fga_reconstruct_grid_add(const fga_beams *beams, double eps, double tau, const int n[3],
                                    const double lo[3], const double h[3], int precision, double *out,
                                    void *workspace, size_t workspace_bytes, void *stream,
                                    int64_t *evals);

/* ------------------------------------------------------------------------ */
/* Serving: forward solves for many sources on one GPU (tomography sweeps)   */
/* ------------------------------------------------------------------------ */

/* One forward solve: decompose the initial data, evolve with receivers and
 * return the seismograms (Steps 1-3 of Sec. 2 for one source). */
typedef struct {
  fga_medium medium;        /* by value; a grid table it points to is device memory,
                               built (and its build finished) before submit, that
                               the caller keeps valid until the request completes   */
  fga_mesh mesh;            /* decomposition mesh (eps = mesh.eps)                   */
  const double *f;          /* host, complex [3][ny2][ny1][ny0] initial displacement
                               ("+"-going with mesh.one_way); copied by submit      */
  int64_t n_receivers;
  const double *receivers;  /* host, [n_receivers][3]; copied by submit               */
  double tau;               /* window parameter of the receiver sums                 */
  double dt;
  int nsteps;
  int stride;               /* a sample after every stride-th step                   */
  double *seis_out;         /* host, complex [n_receivers][nsteps/stride][3]; written
                               before the completion is reported; caller-owned       */
  int precision;            /* receiver sums: FGA_FP64, FGA_FP32 or FGA_FP32_ACC32    */
  int point_source;         /* 1: the initial data is `source` (mesh and f unused)    */
  fga_point_source source;
  int receiver_coords;      /* FGA_COORDS_CARTESIAN or FGA_COORDS_SPHERICAL, as in
                               fga_receivers                                         */
} fga_request;

typedef struct {
  uint64_t id;              /* as returned by fga_server_submit                      */
  int status;               /* fga_status of the solve                               */
  double t_submit, t_start, t_done;  /* seconds on the server's monotonic clock     */
  size_t footprint;         /* device bytes the request held                         */
  int64_t beams, beam_steps, evals;
} fga_completion;

typedef struct fga_server fga_server;

/* Device bytes one request holds while it runs (beams, workspaces, inputs,
 * seismograms); admission compares this with the budget. */
size_t fga_server_footprint(const fga_request *r);

/* A request server on the current device.  It takes one device pool of
 * hbm_budget bytes at creation (its only allocation; freed by
 * fga_server_destroy); each request runs in a block of the pool of its
 * footprint, so solves allocate and free nothing on the device.  Requests
 * are admitted in arrival order, skipping ahead to the first queued one that
 * fits, whenever a slot is free (at most max_active at once) and a block of
 * the request's footprint is free in the pool (first fit).
 * Each slot runs its request on its own stream from its own host thread,
 * so admitted requests overlap on the device; a request's result does not
 * depend on what runs beside it (each solve is deterministic).
 * Errors: FGA_EINVAL (max_active < 1), FGA_ENOMEM (the pool cannot be
 * allocated), FGA_EDEVICE. */
fga_status fga_server_create(size_t hbm_budget, int max_active, fga_server **out);
/* Queues a request (non-blocking; f and receivers are copied).  Errors:
 * FGA_EINVAL (invalid request), FGA_ECAPACITY (footprint above the budget:
 * it could never run). */
fga_status fga_server_submit(fga_server *s, const fga_request *r, uint64_t *id);
/* Moves up to max finished requests into out (completion order) and sets
 * *n; waits up to wait_ms milliseconds for the first one when none is ready
 * (0: do not wait). */
fga_status fga_server_poll(fga_server *s, fga_completion *out, int max, int *n, int wait_ms);
/* Current queue length, running requests and device bytes they hold, and the
 * largest number of requests that have run at once. */
fga_status fga_server_status(fga_server *s, int *queued, int *running, size_t *held, int *peak_running);
/* Waits for every queued and running request, then frees the server;
 * completions not yet polled are discarded. */
fga_status fga_server_destroy(fga_server *s);

/* ------------------------------------------------------------------------ */
/* Kernel timing                                                             */
/* ------------------------------------------------------------------------ */

/* Kernels whose launches can be timed. */
typedef enum {
  FGA_K_INTEGRATE = 0,   /* RK4 integrator                                   */
  FGA_K_SUM_POINTS = 1,  /* receiver / point summation                       */
  FGA_K_GRID_TILE = 2,   /* grid tile GEMMs on the matrix cores              */
  FGA_K_FBI_GEMM = 3,    /* FBI mode products of the decomposition           */
  FGA_K_COUNT = 4
} fga_kernel_id;

/* While enabled (on != 0), every launch of the kernels above is bracketed by
 * a pair of hipEvents recorded on the launch's own stream.  Enabling or
 * disabling discards what was recorded.  Process-wide; not thread-safe. */
fga_status fga_profile_enable(int on);
/* Waits for the recorded events of kernel `k` and returns the number of
 * launches and their summed duration in milliseconds (GPU clock); reset != 0
 * clears the record afterwards.  Errors: FGA_EINVAL for an unknown kernel. */
fga_status fga_profile_read(int k, int64_t *launches, double *total_ms, int reset);

#ifdef __cplusplus
}
#endif
#endif /* FGA_H */
