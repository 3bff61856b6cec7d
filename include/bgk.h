/*
 * bgk.h -- C interface of libbgk: the per-time-step update of the meshfree
 * Arbitrary-Lagrangian-Eulerian (ALE) method for the BGK equation
 * (Mariappan, Willems, Boregowda, Tiwari, Klar, "High-performance computing
 * for the BGK model of the Boltzmann equation with a meshfree ALE method"),
 * implemented as HIP kernels for AMD Instinct MI355X (gfx950).
 *
 * One time step (Sections 3.2-3.5):
 *   S1  neighbour search in a cell list over the moving cloud     (Sec. 3.5.1)
 *   S2  weighted least-squares (WLS) gradient operators           (Sec. 3.4.1)
 *   S3  edge frames and positive-upwind vectors                   (Sec. 3.4.2)
 *   S4  explicit transport  ft = f - dt (v-U^n).grad f            (Sec. 3.2.1, eq. explicit)
 *   S5  moments of ft: rho, U, T                                  (eqs. fullmoment1a / moment1a, moment1b)
 *   S6  implicit BGK relaxation f = (tau ft + dt M)/(tau + dt)    (Sec. 3.2.1, closed form after implicitfull_1)
 *   S7  diffuse-reflection walls with a moving lid                (Sec. 5; Table 3)
 *   S8  ALE motion  x^{n+1} = x^n + dt U^{n+1}                    (Sec. 3.2.1)
 *
 * Conventions (all entry points):
 *   - Every function returns an int: BGK_OK (0) or a positive bgk_status.
 *     Nothing throws across this interface and nothing aborts.
 *   - Array arguments are DEVICE pointers owned by the caller, except where a
 *     comment says "host".  The library never allocates device memory: it
 *     owns only the host-side context, and uses a caller-supplied device
 *     workspace of bgk_workspace_bytes() bytes.
 *   - Work is enqueued on the HIP stream given to bgk_init (as void*; NULL is
 *     the default stream).  Calls return before the GPU work finishes.
 *   - Errors that depend on data (neighbour overflow, singular least squares,
 *     non-physical moments) are recorded in a device error word; bgk_check()
 *     synchronises the stream and returns (and clears) them.
 *   - Layouts (row-major):
 *       x, U      double [d][N]            (component-major)
 *       rho, T    double [N]
 *       f         [n_c][N][N_v] of double (BGK_FP64) or float (BGK_FP32,
 *                 BGK_BF16); n_c = 2 (g1, g2) for dim 2, 1 for dim 3;
 *                 velocity index q = k1 + nv*k2 (+ nv^2*k3)
 *       nbr_idx   int32 [N][max_neighbors], first nbr_cnt[i] entries used,
 *                 ascending, the particle itself included
 *       grad      double [N][max_neighbors][d]
 *       ops       double [N][max_neighbors][d*d]: P (d values), Q (d)
 *                 [, R (d)] per neighbour slot
 *   - Velocity grid (Sec. 3.3, read as nv points per axis including both
 *     ends): v_k = vmax*(2k-(nv-1))/(nv-1), k = 0..nv-1; every node has the
 *     weight omega = (2 vmax/(nv-1))^d.
 *   - Particles: wall_id[i] = 0 for interior particles, else the owner wall
 *     1..2d in the order x=0, x=1, y=0, y=1 (, z=0, z=1).  The lid is the
 *     last wall (y=1 in 2D, z=1 in 3D) and moves along +x.  Wall particles
 *     carry the boundary condition and never move.
 *   - Units are nondimensional (R = 1, lengths in the box size).
 */
#ifndef BGK_H
#define BGK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BGK_OK = 0,
  BGK_EINVAL = 1,         /* bad argument or configuration                  */
  BGK_ENOMEM = 2,         /* workspace smaller than bgk_workspace_bytes()    */
  BGK_ENBR_OVERFLOW = 3,  /* more neighbours than max_neighbors              */
  BGK_ESINGULAR = 4,      /* too few neighbours or non-positive pivot (WLS)  */
  BGK_ENONPHYS = 5,       /* rho <= 0, T <= 0 or NaN after moments           */
  BGK_EDEVICE = 6,        /* a HIP runtime call failed                       */
  BGK_ENOTSUP = 7         /* valid but unsupported request                   */
} bgk_status;

enum { BGK_FP64 = 0, BGK_FP32 = 1, BGK_BF16 = 2 };
enum { BGK_FLAG_GENERIC = 1, BGK_FLAG_ADJOINT = 2, BGK_FLAG_PARTICLES = 4 };

typedef struct {
  int32_t dim;           /* 2: Chu-reduced BGK (Sec. 2.1, g1 and g2); 3: full BGK        */
  int32_t n_particles;   /* N, interior + wall                                           */
  int32_t nv;            /* velocity points per axis, even, 2..1024                      */
  int32_t wls_degree;    /* 1 or 2: degree of the full-basis least-squares fit;          *
                          * 0: first-derivative fit as printed in Sec. 3.4.1            */
  int32_t max_neighbors; /* neighbour slots per particle (self included), <= 255         */
  int32_t move;          /* 1: ALE motion (S8); 0: frozen cloud (geometry reused)        */
  int32_t precision;     /* BGK_FP64, BGK_FP32 (FP32 f and transport arithmetic) or
                            BGK_BF16 (FP32 f; transport products of BF16 operands with
                            FP32 accumulation).  Geometry, least squares and moment
                            sums are FP64 in every mode.                                  */
  int32_t flags;         /* bit set: BGK_FLAG_GENERIC uses the separate transport and
                            relaxation kernels instead of the fused one (for testing);
                            BGK_FLAG_ADJOINT reserves the workspace of
                            bgk_adjoint_step (move = 0) or bgk_adjoint_step_move
                            (move = 1); needs BGK_FP64 or BGK_FP32;
                            BGK_FLAG_PARTICLES reserves that of bgk_pm_plan /
                            bgk_pm_apply                                                  */
  double vmax;           /* velocity grid spans [-vmax, vmax] per axis                   */
  double h;              /* support radius of the Gaussian weight (absolute)             */
  double alpha;          /* weight exp(-alpha r^2/h^2), r <= h (Sec. 3.4.1, eq. weight) */
  double kn;             /* tau = kn sqrt(2/pi)/(rho sqrt(T)) (Sec. 2, eqs. tau/lambda)  */
  double dt;             /* time step                                                    */
  double wall_T;         /* wall temperature                                             */
  double lid_velocity;   /* lid speed along +x                                           */
  double dx;             /* initial lattice spacing: interior particles stay in
                            [0.1 dx, 1 - 0.1 dx]^d                                       */
} bgk_config;

typedef struct bgk_ctx bgk_ctx;

/* Device workspace needed by bgk_init for this configuration (bytes, host). */
int bgk_workspace_bytes(const bgk_config* cfg, size_t* bytes);

/* Create a context for one point cloud (Sec. 3.4.1: boundary and interior
 * particles of the moving cloud; Sec. 3.3: the velocity grid; Sec. 5: the
 * cavity's walls and lid).  cfg is copied.  wall_id: device int32 [N] (read
 * once, synchronously, at init), 0 for interior particles, else the owner
 * wall.  workspace: device buffer of ws_bytes bytes that
 * the caller keeps alive until bgk_destroy.  hip_stream: hipStream_t or NULL.
 * *out receives the context (host).  Errors: BGK_EINVAL (dim not 2/3, odd nv
 * or nv > 1024, N <= 0, dt <= 0, bad degree or capacity), BGK_ENOMEM (ws_bytes too small),
 * BGK_EDEVICE. */
int bgk_init(const bgk_config* cfg, const int32_t* wall_id, void* workspace, size_t ws_bytes,
             void* hip_stream, bgk_ctx** out);

void bgk_destroy(bgk_ctx* ctx);

/* Change the lid speed used by later calls (S7). */
int bgk_set_lid_velocity(bgk_ctx* ctx, double lid_velocity);

/* S1 (Sec. 3.5.1; truncation r/h <= 1 of eq. weight): for every particle i,
 * the particles j with |x_j - x_i|^2 <= h^2 (squared distance summed over
 * components in order, without fused multiply-add), ascending, i included.
 * Found with a cell list of cells no smaller than h.  nbr_cnt[i] is the true
 * count even when it exceeds max_neighbors (then BGK_ENBR_OVERFLOW is raised
 * in the error word and the row content is unspecified). */
int bgk_build_neighbors(bgk_ctx* ctx, const double* x, int32_t* nbr_cnt, int32_t* nbr_idx);

/* S2-S3 (Sec. 3.4.1 eqs. taylor..z_derivative, Sec. 3.4.2) for every
 * interior particle: Gaussian-weighted least-squares fit of a full polynomial
 * basis of degree wls_degree (constant included) in offsets scaled by h, the
 * particle itself in its stencil; the degree drops to 1 when the stencil has
 * fewer than twice as many points as degree-2 basis functions, and
 * BGK_ESINGULAR is raised below d+2 points or on a non-positive Cholesky
 * pivot.  wls_degree 0 is the fit exactly as printed: the unknowns are the d
 * first derivatives of f_j - f_i ~ a.(x_j - x_i), a = (M^T W M)^-1 M^T W b,
 * no constant term (the self offset is zero and drops out).  grad[i][e] = gradient weight of neighbour slot e (so
 * grad f(x_i) ~ sum_e grad[i][e] f_j).  ops[i][e] = (P, Q[, R]) = the gradient
 * weight rotated into the edge frame (n, t[, b]) of x_j - x_i and mapped back:
 * P = (g.n) n, Q = (g.t) t, R = (g.b) b, with t = n turned by +90 degrees in
 * 2D and, in 3D, t and b the polar and azimuthal unit vectors of the edge
 * (b horizontal).  The self slot has zero P, Q, R.  Rows of wall particles
 * are zero.  degree: int32 [N] (the degree used; 0 for wall particles), may
 * be NULL. */
int bgk_wls_operators(bgk_ctx* ctx, const double* x, const int32_t* nbr_cnt,
                      const int32_t* nbr_idx, double* grad, double* ops, int32_t* degree);

/* Boundary interpolation rows (S7 part 1; the paper names the interpolation
 * of f on the boundary in Table 3): for each wall particle b, the interior
 * particles within radius hb, ascending, and the value weights c0[b][e] of
 * a degree-1 weighted least-squares fit evaluated at x_b.  hb is the first
 * of h, 1.5h, 2h whose set holds at least d+2 particles, gives a
 * positive-definite fit and keeps the extrapolation's amplification
 * sum_e |c0[b][e]| at most 8 (above every row of a jittered lattice, so the
 * bound only widens stencils that a moving cloud has made near-degenerate);
 * the 2h row is taken without the bound, and BGK_ESINGULAR is raised when
 * it has fewer than d+2 points or a non-positive pivot.
 * Outputs are indexed by particle: wall_cnt int32 [N] (0 on interior rows),
 * wall_idx int32 [N][max_neighbors], wall_c0 double [N][max_neighbors],
 * wall_radius double [N] (may be NULL). */
int bgk_wall_stencil(bgk_ctx* ctx, const double* x, int32_t* wall_cnt, int32_t* wall_idx,
                     double* wall_c0, double* wall_radius);

/* S1-S3 and the wall rows into the context's workspace (what bgk_step does
 * first); used by the staged calls below. */
int bgk_geometry(bgk_ctx* ctx, const double* x);

/* S4 (Sec. 3.2.1 eq. explicit, Sec. 3.2.2 for Chu; Sec. 3.4.2 eq. flux and its 3D form), with the
 * geometry of the last bgk_geometry/bgk_step: for interior i and every v,
 *   ft_i(v) = f_i(v) - dt sum_{j != i} c_ij(v) (f_j(v) - f_i(v)),
 *   c_ij(v) = g_ij.w - |P_ij.w| - |Q_ij.w| - |R_ij.w|,  w = v - U_i,
 * which is the printed flux with its dissipation written |abar||w.n|.
 * Wall rows of f_tilde are copies of f_in.  f_in and f_tilde must differ. */
int bgk_transport(bgk_ctx* ctx, const void* f_in, void* f_tilde, const double* U);

/* S5-S6 (Sec. 3.2.1, Sec. 3.2.2) for interior particles: rho, U, T of ft (Chu: 3 rho T from g1 and g2,
 * eq. moment1b; two passes, U first), tau = kn sqrt(2/pi)/(rho sqrt T), and
 * f_out = (tau ft + dt M[rho,U,T])/(tau + dt) (Chu: G1 = rho/(2 pi T)
 * exp(-|v-U|^2/(2T)), G2 = T G1).  f_out may equal f_tilde.  Wall rows of
 * f_out and of rho, U, T are left untouched. */
int bgk_collide(bgk_ctx* ctx, const void* f_tilde, void* f_out, double* rho, double* U,
                double* T);

/* S7 in place on the wall rows of f (whose interior rows hold f^{n+1}):
 * velocities with v.n_w <= 0 (n_w the inward normal) take the interpolated
 * interior value; the others take rho_w M[1, U_w, T_w] (Chu: g1 = rho_w G1hat,
 * g2 = T_w rho_w G1hat) with rho_w set by zero net discrete mass flux; then
 * the wall particles' rho, U, T are the moments of their f. */
int bgk_wall_bc(bgk_ctx* ctx, void* f, double* rho, double* U, double* T);

/* S8 (Sec. 3.2.1, position update): x_i += dt U_i for interior particles, clamped to
 * [0.1 dx, 1 - 0.1 dx]^d (clamped coordinates are counted, bgk_diagnostics). */
int bgk_move(bgk_ctx* ctx, double* x, const double* U);

/* One full step S1..S8.  f_in: state f^n (unchanged); f_out: receives
 * f^{n+1} (must differ from f_in); x: positions, updated in place when
 * cfg.move; U: on entry U^n (used by the transport), on exit U^{n+1};
 * rho, T: receive the new values. */
int bgk_step(bgk_ctx* ctx, const void* f_in, void* f_out, double* x, double* U, double* rho,
             double* T);

/* bgk_step that also keeps the transported field: f_tilde receives the
 * interior rows of f-tilde = f^n - dt sum_j c_ij (f_j - f_i) (Sec. 3.2.1,
 * eq. explicit), the input of the relaxation; its wall rows are left
 * untouched.  Same arguments, results and errors as bgk_step otherwise;
 * f_tilde is f-sized, in the f storage type, and may not overlap f_in,
 * f_out or the other arrays (BGK_EINVAL).  With the step's outputs it is
 * what bgk_adjoint_step_kept reads, so that a reverse pass that keeps its
 * forward states does not recompute them. */
int bgk_step_keep(bgk_ctx* ctx, const void* f_in, void* f_out, double* x, double* U, double* rho,
                  double* T, void* f_tilde);

/* Particle management (Sec. 3.5.2, adding and removing points), plan.  The
 * paper replaces two points that come too close by one at their midpoint
 * and adds points where holes open, filling f there by least squares; it
 * states no thresholds.  The rule taken: interior particles i < j that are
 * each other's nearest interior neighbour within h (ties to the lower
 * index) and closer than merge_radius merge into one interior particle at
 * 0.5 (x_i + x_j); every interior node k dx of the initial lattice
 * (0 < k < n-1 per axis, n = round(1/dx) + 1) with no particle of the
 * merged cloud within hole_radius gets a new interior particle.  Distances
 * are squared, summed component by component.  x: device [d][N].  Writes
 * the counts to the host ints *n_pairs and *n_holes (synchronises the
 * stream); the managed cloud has N' = N - n_pairs + n_holes particles.
 * Needs BGK_FLAG_PARTICLES and 0 < merge_radius, 0 < hole_radius,
 * merge_radius + hole_radius <= h (else BGK_ENOTSUP / BGK_EINVAL).  It
 * rebuilds the context's cell list from x, so a frozen cloud's geometry is
 * rebuilt by the next step.  Defaults used by the Python layer: merge
 * radius dx/4, hole radius 0.45 h. */
int bgk_pm_plan(bgk_ctx* ctx, const double* x, double merge_radius, double hole_radius,
                int32_t* n_pairs, int32_t* n_holes);

/* Particle management, apply the plan of the last bgk_pm_plan (same x, no
 * call that moves the cloud or rebuilds its cell list in between, else
 * BGK_EINVAL).  Inputs (device, old cloud of N): x [d][N], f [n_c][N][N_v]
 * (storage precision), rho [N], U [d][N], T [N].  Outputs (device, caller
 * allocated for N'): x_new [d][N'], wall_id_new [N'], f_new [n_c][N'][N_v],
 * rho_new [N'], U_new [d][N'], T_new [N'].  Order of the new cloud: the
 * particles not merged, in their old order, with their f, rho, U, T and
 * owner; then the midpoints by the lower index of their pair; then the
 * hole particles by node index k_x + n k_y (+ n^2 k_z).  f at a new
 * particle: the degree-1 least-squares value row at its position over the
 * old cloud's interior particles within hb (the rule of the wall rows),
 * applied to every velocity and component; its rho, U, T are the moments
 * of that f (BGK_ENONPHYS in the error word if they are not positive;
 * BGK_ESINGULAR / BGK_ENBR_OVERFLOW as for wall rows).  A context for the
 * new cloud is created with bgk_init and n_particles = N'. */
int bgk_pm_apply(bgk_ctx* ctx, const double* x, const void* f, const double* rho,
                 const double* U, const double* T, double* x_new, int32_t* wall_id_new,
                 void* f_new, double* rho_new, double* U_new, double* T_new);

/* Moments (Sec. 2 eqs. moments, internal_energy; Chu eq. macroeq) of every
 * particle: rho = omega sum f1, U = sum v f1 / sum f1, T from the centred
 * second moment (Chu: plus sum g2) over 3 rho. */
int bgk_moments(bgk_ctx* ctx, const void* f, double* rho, double* U, double* T);

/* Health of a state (f, rho, U, T), e.g. f^{n+1} with the moments the step
 * reported; the per-step diagnostics of the method's invariants.  Every
 * particle's row of f has its moments recomputed as bgk_moments does (Sec. 2
 * eqs. moments, internal_energy): after a step they differ from the step's
 * rho, U, T only by the relaxation's conservation defect (Sec. 3.2.1: the
 * implicit relaxation conserves the moments up to the velocity grid's
 * quadrature error of the discrete Maxwellian).  f must stay non-negative
 * (the positivity of the upwind scheme, Sec. 3.4.2).  out: host double[12]:
 *   [0] smallest finite value of f (any component, particle, velocity),
 *   [1] number of negative values, [2] number of non-finite values,
 *   [3] max_i |rho(f_i) - rho_i| / rho_i, [4] max_{i,k} |U_k(f_i) - U_ki|,
 *   [5] max_i |T(f_i) - T_i| / T_i (NaN if any residual is NaN),
 *   [6] sum_i rho_i, [7 .. 7+d) sum_i rho_i U_i,
 *   [7+d] sum_i rho_i (|U_i|^2 + 3 T_i) / 2, the rest 0.
 * Device inputs as for bgk_moments; synchronises the context stream.  Sums
 * and extrema are taken in a fixed order (bitwise repeatable). */
int bgk_state_check(bgk_ctx* ctx, const void* f, const double* rho, const double* U,
                    const double* T, double* out);

/* Maxwellian (Sec. 2 eq. maxwellian with the exponent's minus sign; Chu:
 * G1, G2 of eqs. Maxw_G1/G2 with the v3-marginal normalisation rho/(2 pi T))
 * of every particle on the grid, into f_out. */
int bgk_maxwellian(bgk_ctx* ctx, const double* rho, const double* U, const double* T,
                   void* f_out);

/* Objective of the lid-driven cavity at a state (f, rho, U): the lid-normal
 * heat flux summed over the lid particles plus a weighted kinetic energy,
 *   J = dx^(d-1) sum_{b on the lid} q_n(b) + (ke_weight/N) sum_i rho_i |U_i|^2/2,
 *   q_n = (omega/2) sum_v (v_n - U_n) |v-U|^2 f   (Chu: |v-U|^2 g1 + g2),
 * n the lid's axis (y in 2D, z in 3D) and U the particle's own mean velocity
 * (q is the kinetic heat flux, the centred third moment of f; the paper
 * defines no objective, this is the functional that the reverse mode below
 * is exercised on).
 * J: device double [1], overwritten.  dJ_df (like f, in the f storage
 * type), dJ_drho [N] and dJ_dU [d][N] receive the partial derivatives at
 * fixed (f, rho, U); each may be NULL.  BGK_FP64 or BGK_FP32 (else
 * BGK_ENOTSUP); sums are FP64.  J is summed in a fixed order, so repeated
 * calls give identical bits. */
int bgk_objective(bgk_ctx* ctx, const void* f, const double* rho, const double* U,
                  double ke_weight, double* J, void* dJ_df, double* dJ_drho, double* dJ_dU);

/* The same objective as bgk_objective, for callers that cannot allocate
 * device memory and must not touch the context's workspace while calling
 * it (code being captured into a HIP graph, tight serving loops, harnesses
 * that forbid hipMalloc): the per-particle terms go to a fixed scratch
 * array of BGK_STATIC_SCRATCH_PARTICLES doubles (8 MiB) that every GPU the
 * library runs on holds until the process ends.  Same arguments, results
 * and errors as bgk_objective (bit for bit the same J and partial
 * derivatives), plus BGK_EINVAL when the context has more than
 * BGK_STATIC_SCRATCH_PARTICLES particles.  It calls no allocating routine.
 * All calls on one GPU share that GPU's scratch: calls that overlap in
 * time on one GPU (on different streams, or from several host threads)
 * race on it and must be ordered by the caller. */
#define BGK_STATIC_SCRATCH_PARTICLES (1 << 20)
int bgk_objective_static(bgk_ctx* ctx, const void* f, const double* rho, const double* U,
                         double ke_weight, double* J, void* dJ_df, double* dJ_drho,
                         double* dJ_dU);

/* Reverse mode of one frozen-cloud step (S4-S7 with the operators of the
 * fixed cloud; Sec. 3.2 and Sec. 5).  The step maps the state (f^n, U^n) and
 * the lid speed to (f^{n+1}, U^{n+1}, rho^{n+1}, T^{n+1}).  Given the
 * adjoints lam_* of those outputs, this returns
 *   lam_f = (d f^{n+1}/d f^n)^T lam_f1 + ... (every output's term),
 *   lam_U = the same for U^n (which enters only the upwind weights c_ij),
 *   dJ_dlid += the lid-speed term (through the emitted wall Maxwellian and
 *              its zero-mass-flux density).
 * f_n, U_n: the state the forward step started from (the step's intermediate
 * values are recomputed into the workspace).  x: positions, used to build
 * the geometry when none is current.  lam_U1, lam_rho1, lam_T1 may be NULL
 * (zero).  lam_f may be the same buffer as lam_f1 and lam_U the same as
 * lam_U1 (in place); no other overlap is allowed (BGK_EINVAL).  dJ_dlid:
 * device double [1], accumulated (+=); may be NULL.  |.| terms take the
 * derivative of their + branch at 0.  The transposed stencils make every
 * sum a gather: results are deterministic.  Needs a context created with
 * BGK_FLAG_ADJOINT and move = 0, else BGK_ENOTSUP.  f_n, lam_f1 and lam_f
 * are in the f storage type (FP64; or FP32, with FP32 arithmetic in the
 * reverse transport's per-velocity work and FP64 in every reduction and in
 * the other reverse kernels). */
int bgk_adjoint_step(bgk_ctx* ctx, const void* f_n, const double* U_n, const double* x,
                     const void* lam_f1, const double* lam_U1, const double* lam_rho1,
                     const double* lam_T1, void* lam_f, double* lam_U, double* dJ_dlid);

/* bgk_adjoint_step with the forward step's state supplied instead of
 * recomputed: f_tilde, f_n1, rho_n1, U_n1, T_n1 are what bgk_step_keep(f_n,
 * U_n) returned (f-tilde's interior rows, f^{n+1}, and the moments of n+1,
 * each [N] or [d][N] double).  The results are those of bgk_adjoint_step on
 * (f_n, U_n), bit for bit.  The kept arrays are inputs (no output may
 * overlap them, BGK_EINVAL); otherwise as bgk_adjoint_step. */
int bgk_adjoint_step_kept(bgk_ctx* ctx, const void* f_n, const double* U_n, const double* x,
                          const void* f_tilde, const void* f_n1, const double* rho_n1,
                          const double* U_n1, const double* T_n1, const void* lam_f1,
                          const double* lam_U1, const double* lam_rho1, const double* lam_T1,
                          void* lam_f, double* lam_U, double* dJ_dlid);

/* Reverse mode of one full step S1-S8 with the MOVING cloud (Sec. 3.2.1 with
 * the position update; Sec. 3.4.1 least squares; Sec. 3.4.2 edge frames;
 * Sec. 5 walls): the step maps (f^n, U^n, x^n, lid) to (f^{n+1}, U^{n+1},
 * x^{n+1}, rho^{n+1}, T^{n+1}), and the operators, edge frames and wall
 * value rows are functions of x^n.  Given the output adjoints, returns
 * lam_f and lam_U as bgk_adjoint_step does, plus
 *   lam_x = (d x^{n+1}/d x^n)^T lam_x1 (identity on coordinates the clamp
 *           of S8 left alone, zero on clamped ones) + the adjoint of x^n
 *           through the gradient rows, frames and wall rows of every edge,
 * and lam_U1 receives dt lam_x1 of the unclamped interior coordinates
 * (x^{n+1} = x^n + dt U^{n+1}).  Neighbour sets, stencil radii and fitted
 * degrees are those of x^n's values (piecewise constant; the derivative is
 * that of the smooth piece).  x_n: device double [d][N], the positions the
 * forward step started from; lam_x1, lam_x: double [d][N]; lam_x1,
 * lam_U1, lam_rho1, lam_T1 may be NULL (zero); lam_f may equal lam_f1,
 * lam_U may equal lam_U1 and lam_x may equal lam_x1 (in place); no other
 * overlap (BGK_EINVAL).  Needs a context created with BGK_FLAG_ADJOINT and
 * move = 1 (else BGK_ENOTSUP).  Sums have a fixed order: deterministic. */
int bgk_adjoint_step_move(bgk_ctx* ctx, const void* f_n, const double* U_n, const double* x_n,
                          const void* lam_f1, const double* lam_U1, const double* lam_x1,
                          const double* lam_rho1, const double* lam_T1, void* lam_f,
                          double* lam_U, double* lam_x, double* dJ_dlid);

/* Reverse mode of bgk_moments (Sec. 2 eqs. moments, internal_energy; Chu
 * eq. macroeq): lam_f += (d(rho, U, T)/d f)^T (lam_rho, lam_U, lam_T) at the
 * moments (rho, U, T) of f.  lam_rho, lam_U, lam_T may be NULL (zero).
 * lam_f in the f storage type; BGK_FP64 or BGK_FP32 (else BGK_ENOTSUP). */
int bgk_moments_adjoint(bgk_ctx* ctx, const double* rho, const double* U, const double* T,
                        const double* lam_rho, const double* lam_U, const double* lam_T,
                        void* lam_f);

/* Synchronise the stream; return and clear the first data error recorded on
 * the device (or BGK_EDEVICE). */
int bgk_check(bgk_ctx* ctx);

/* Diagnostics (host, int64 [4]): clamped coordinates since init, steps
 * taken, and the largest neighbour count and largest patch union of the
 * geometry built last by bgk_geometry / bgk_step.  Synchronises. */
int bgk_diagnostics(bgk_ctx* ctx, int64_t* out4);

/* Instrumentation: while enabled, bgk_step records a pair of HIP events on
 * the context stream around its transport kernel (S4).  bgk_timing_read
 * synchronises and returns the summed kernel time in ms and the number of
 * timed launches since the last read (host outputs), then resets them. */
int bgk_timing_enable(bgk_ctx* ctx, int enable);
int bgk_timing_read(bgk_ctx* ctx, double* total_ms, int64_t* launches);

/* Text of the last error on this context (host string owned by the context). */
const char* bgk_last_error(bgk_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* BGK_H */
