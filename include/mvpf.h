/*
 * mvpf -- Newton-step solver for the finite-strain multivariant martensite
 * phase-field model on one AMD Instinct MI355X (gfx950).
 *
 * Model: Tuma, Rezaee-Hajidehi, Hron, Farrell, Stupkiewicz, "Phase-field
 * modeling of multivariant martensitic transformation at finite-strain:
 * computational aspects and large-scale finite-element simulations",
 * CMAME 2021 (cited below by section / equation / table).
 *
 * Unknowns: 3 + N per node, node-interleaved [u_x, u_y, u_z, eta_1 .. eta_N]:
 * displacement u = phi - X and the condensed order parameters eta_hat with
 * eta_0 = 1 - sum eta_i (Sec. 3.1).  N, the number of martensite variants,
 * is a compile-time constant of a library build (mvpf_nvar()): 6 for
 * libmvpf.so (CuAlNi, Sec. 4.1; 9 unknowns per node), 12 for
 * libmvpf_n12.so (15 unknowns per node).  "9" below stands for 3 + N and
 * "6" (order parameters) for N.  Nodes are numbered lexicographically,
 * x fastest: node(i,j,k) = i + (nx+1)*(j + (ny+1)*k).  The mesh is a uniform
 * grid of nx*ny*nz cubes of side h (trilinear Q1 elements, 2x2x2 Gauss).
 *
 * Conventions for every call:
 *  - return 0 on success; negative on error (MVPF_EINVAL, MVPF_ENOMEM,
 *    MVPF_EDEVICE, MVPF_ESINGULAR, MVPF_ESTATE); MVPF_ENOTCONV (> 0) when a
 *    solve or Newton loop stopped without converging -- outputs and stats are
 *    still valid.  mvpf_last_error() gives a message.
 *  - every "device" array argument is a device pointer (e.g. a torch CUDA
 *    tensor's data_ptr) to FP64 data, node-interleaved, length 9*n_nodes of
 *    the addressed level unless stated otherwise; the caller owns it; the
 *    library reads/writes it in stream order on the problem's stream and does
 *    not retain it after the call returns.
 *  - the library owns all of its internal device memory (operators, Krylov
 *    bases, work vectors); it is allocated in mvpf_create / on first use and
 *    released by mvpf_destroy.
 *  - one HIP stream per problem (given at creation; NULL = the default
 *    stream).  Calls on one handle are not thread-safe; separate handles are
 *    independent.
 */
#ifndef MVPF_H
#define MVPF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MVPF_OK = 0,
  MVPF_ENOTCONV = 1,
  MVPF_EINVAL = -1,
  MVPF_ENOMEM = -2,
  MVPF_EDEVICE = -3,
  MVPF_ESINGULAR = -4,
  MVPF_ESTATE = -5
};

enum { MVPF_FP64 = 0, MVPF_MIXED = 1 };          /* mvpf_opts.precision */
enum { MVPF_MIX_LINEAR = 0, MVPF_MIX_LOG = 1 };  /* mixing rule of the transformation stretch */
enum { MVPF_LOAD_PATCH = 0, MVPF_LOAD_CAP = 1, MVPF_LOAD_SPHERE = 2 };  /* mvpf_loading.kind */
enum { MVPF_COARSE_REDISCRETISE = 0, MVPF_COARSE_GALERKIN = 1 };  /* mvpf_opts.coarse */

typedef struct mvpf_problem mvpf_problem;
typedef struct mvpf_batch mvpf_batch;

/* Structured mesh of nx*ny*nz cubes of side h, and the number of geometric
 * multigrid levels.  Level l has nx/2^l x ny/2^l x nz/2^l elements, so nx, ny,
 * nz must be divisible by 2^(n_levels-1); n_levels >= 2 (the coarsest level is
 * solved directly and must have at most MVPF_MAX_COARSE_DOF unknowns). */
typedef struct {
  int nx, ny, nz;
  double h;
  int n_levels;
} mvpf_mesh;

#define MVPF_MAX_COARSE_DOF 8192
#define MVPF_MAX_BATCH 256

/* Material card (Sec. 2.2, 2.3, 3.1, 4.1; Table 1).  Stresses and energy
 * densities in GPa, lengths in units of the mesh coordinates.
 *  cubic   austenite c11, c12, c44 in the cubic crystal axes
 *  ortho   martensite c11, c22, c33, c44, c55, c66, c12, c13, c23 in the
 *          orthorhombic axes; variant k's axes 1,2,3 are the principal axes of
 *          its stretch tensor U_k for the eigenvalues alpha, beta, gamma
 *  alpha, beta, gamma   transformation stretch parameters (Sec. 4.1)
 *  Q       rotation, row-major; rows are the sample axes in crystal axes
 *  F0      chemical energy densities of phases 0..6 (austenite first)
 *  w_am, w_mm  double-obstacle coefficients 4 gamma_ij / (pi l_ij) of the
 *          austenite-martensite and martensite-martensite pairs (Eq. IntEnergy)
 *  ell     interface thickness parameter l_ij (all pairs)
 *  rho     viscous coefficient 1/(m tau) (all phases, Sec. 2.3)
 *  eps_eta penalty parameter of eta_i >= 0 (Eq. PenPot)
 *  pade    Pade order of the Hencky strain: 11, 22 or 33 for the (1,1), (2,2) or
 *          (3,3) approximant (Eqs. pade11, pade22, pade33); other values are
 *          rejected with MVPF_EINVAL
 *  mixing  MVPF_MIX_LINEAR: F^t = sum_i eta_i U_i (Eq. LinMix, the paper's
 *          choice); MVPF_MIX_LOG: F^t = exp(sum_i eta_i log U_i), the
 *          logarithmic rule of Sec. 2.1 (its exponential is evaluated by its
 *          power series, exact to rounding while ||sum eta_i log U_i||_F <= 1,
 *          i.e. far beyond the order parameters' range [0, 1] here)
 * This card has six variants: it needs a library built for N = 6
 * (mvpf_nvar()); otherwise mvpf_create returns MVPF_EINVAL. */
typedef struct {
  double cubic[3];
  double ortho[9];
  double alpha, beta, gamma;
  double Q[9];
  double F0[7];
  double w_am, w_mm;
  double ell;
  double rho;
  double eps_eta;
  int pade;
  int mixing;
} mvpf_material;

/* Material card with N variants generated from one stretch tensor (Sec. 2.1:
 * the variants are crystallographically equivalent; the paper's footnote in
 * Sec. 4.4 mentions NiTi with 12 variants, 15 unknowns per node).  The
 * variants are the distinct images R U1 R^T of U1 under the 24 rotations R
 * of the cube, taken in a fixed order (signed permutation matrices
 * R[i][perm[i]] = sign[i] of determinant +1: permutations of (0,1,2) in
 * lexicographic order, then sign patterns with row 0's sign varying
 * slowest, + before -; images within 1e-12 of an earlier one are the same
 * variant); variant k's stiffness is L1 rotated by the R that produced it.
 * All in the cubic axes, then rotated by Q into the sample frame.
 *  U1      row-major symmetric 3x3 stretch tensor of variant 1
 *  L1      6x6 Voigt stiffness of variant 1 (order 11,22,33,23,13,12,
 *          engineering shear strains), row-major, GPa
 *  cubic, Q, w_am, w_mm, ell, rho, eps_eta, pade, mixing: as mvpf_material
 *  F0_a, F0_m  chemical energy densities of the austenite and of every variant
 * The orbit must have exactly mvpf_nvar() variants (else MVPF_EINVAL). */
typedef struct {
  double U1[9];
  double L1[36];
  double cubic[3];
  double Q[9];
  double F0_a, F0_m;
  double w_am, w_mm;
  double ell;
  double rho;
  double eps_eta;
  int pade;
  int mixing;
} mvpf_orbit_material;

/* Indentation loading (Sec. 4.1).  Bottom face z = 0: u = 0.  Top face
 * z = nz*h, with d = the indenter depth (mvpf_set_state, mvpf_time_step):
 *  MVPF_LOAD_PATCH  nodes of the centred patch x patch element square have
 *                   u_z = -d (patch, nx and ny even);
 *  MVPF_LOAD_CAP    nodes with r^2 < 2 R d - d^2 (r from the top-face centre,
 *                   R = radius) have u_z = -(d - (R - sqrt(R^2-r^2)));
 *  MVPF_LOAD_SPHERE no prescribed top displacements: a rigid sphere of radius
 *                   R centred at (nx h/2, ny h/2, nz h + R - d) acts by
 *                   frictionless penalty contact on the whole top face
 *                   (Sec. 2.4, Eqs. Ngap and PenPot): gap g = |x - c| - R
 *                   at the current position x = X + u, energy
 *                   int 1/2 eps_n <g>_-^2 dS by 2x2 Gauss points per face
 *                   (eps_n > 0, energy per area per squared length).
 * All other dofs are free; order parameters have natural conditions. */
typedef struct {
  int kind;
  int patch;
  double radius;
  double eps_n;
} mvpf_loading;

/* Solver options.  precision MVPF_FP64: every multigrid level in FP64;
 * MVPF_MIXED: multigrid operators, smoother and transfers in FP32 inside the
 * FP64 outer FGMRES (finest operator kept in FP64 for the outer product; the
 * coarsest level always solved in FP64).  rtol: FGMRES stops when the true
 * FP64 residual satisfies ||b - A x|| <= rtol ||b||.  restart: Krylov space
 * size m (<= 64).  max_it: total FGMRES iterations.  nu_pre, nu_post, omega:
 * damped point-block Jacobi sweeps and damping.  newton_max, newton_rtol:
 * Newton iterations of a time step (Sec. 3.4: 12) and its tolerance on the
 * free-dof residual relative to the first right-hand side.  coarse: how the
 * multigrid levels below the finest get their operators --
 * MVPF_COARSE_REDISCRETISE (the paper's choice, Sec. 3.4): the tangent
 * reassembled on each level's own mesh at the injected state (contact
 * included); MVPF_COARSE_GALERKIN: A_(l+1) = P~^T A_l P~ from the finest
 * tangent down, P~ the trilinear prolongation with the rows of constrained
 * level-l unknowns zeroed, then the constrained level-(l+1) unknowns
 * eliminated.  The two agree where the state is uniform over each coarse
 * element; where the order parameters' penalty (Eq. PenPot) is active on a
 * pattern finer than the coarse mesh, the Galerkin levels keep the coarse
 * correction consistent with the fine operator.  It needs device memory for
 * the element matrices of every coarse level (the first level below the
 * finest: 36 * 81 doubles per element of that level, ~1/8 of the finest
 * element count), allocated on first use; batches (mvpf_create_batch) use
 * MVPF_COARSE_REDISCRETISE only. */
typedef struct {
  int precision;
  double rtol;
  int restart;
  int max_it;
  int nu_pre, nu_post;
  double omega;
  int newton_max;
  double newton_rtol;
  int coarse;
} mvpf_opts;

typedef struct {
  int iterations;        /* FGMRES iterations (preconditioner applications) */
  int restarts;
  int converged;
  double rel_residual;   /* true FP64 ||b - A x|| / ||b|| at exit */
  double solve_ms;       /* wall time of the FGMRES solve (stream-synchronised) */
} mvpf_solve_stats;

typedef struct {
  int newton_iterations;
  int linear_iterations; /* summed over the Newton iterations */
  int halvings;          /* depth-increment halvings after Newton failures */
  int converged;
  double residual0;      /* ||b|| of the first Newton system */
  double residual;       /* final free-dof residual norm */
  double assemble_ms;    /* residual + tangent assembly on all levels, block inverses */
  double setup_ms;       /* rest of the coarse factorisation (it overlaps the assembly) */
  double solve_ms;       /* all FGMRES solves */
} mvpf_step_stats;

typedef struct {
  int n_levels;
  int nx[8], ny[8], nz[8];
  int64_t n_nodes[8];
  int64_t bytes_device;  /* device memory held by the problem */
} mvpf_info;

/* Fill opts with the defaults (FP64, rtol 1e-8, restart 30, max_it 500,
 * V(2,2), omega 0.55, newton_max 12, newton_rtol 1e-9, rediscretised coarse
 * levels). */
void mvpf_default_opts(mvpf_opts* opts);

/* Create a problem (the setup of the paper's problem statement, Sec. 2 and
 * Sec. 4.1): validates the inputs, builds the material card in the sample
 * frame (stretch tensors of Sec. 4.1 and Table 1 stiffnesses, each variant's
 * orthorhombic axes being the principal axes of its stretch tensor, rotated
 * by Q), allocates every level's operators and vectors, zeroes the state
 * (u = 0, eta_hat = eta_hat_n = 0, depth 0).  stream: hipStream_t or
 * NULL.  On error *out is NULL and mvpf_last_error(NULL) explains. */
int mvpf_create(const mvpf_mesh* mesh, const mvpf_material* mat, const mvpf_loading* load,
                const mvpf_opts* opts, void* stream, mvpf_problem** out);
/* mvpf_create with a card generated from one stretch tensor (see
 * mvpf_orbit_material); the only way to create problems in a library built
 * for N != 6. */
int mvpf_create_orbit(const mvpf_mesh* mesh, const mvpf_orbit_material* mat, const mvpf_loading* load,
                      const mvpf_opts* opts, void* stream, mvpf_problem** out);
/* Number of variants N the library was built for (the order parameters per
 * node; 3 + N unknowns per node). */
int mvpf_nvar(void);
void mvpf_destroy(mvpf_problem* p);
/* Last error message of p, or of the last failed mvpf_create if p is NULL. */
const char* mvpf_last_error(const mvpf_problem* p);
int mvpf_get_info(const mvpf_problem* p, mvpf_info* info);
/* Change options that do not change memory layout (rtol, max_it, restart <=
 * the value at creation, sweeps, omega, Newton limits); precision is fixed. */
int mvpf_set_opts(mvpf_problem* p, const mvpf_opts* opts);

/* State transfer.  u: device n_nodes x 3, eta, eta_prev: device n_nodes x 6
 * (node-major); NULL leaves that field unchanged / unread.  depth: the
 * indenter depth the state corresponds to. */
int mvpf_set_state(mvpf_problem* p, const double* u, const double* eta, const double* eta_prev,
                   double depth);
int mvpf_get_state(mvpf_problem* p, double* u, double* eta, double* eta_prev, double* depth);
/* Seeded initial state (the paper starts from a perturbed austenite; the
 * perturbation here is a reading: a uniform random eta_hat in [0, 0.05)
 * from a counter-based generator, so that CPU and GPU draw identical bits):
 * u = 0, depth 0, eta_hat = eta_hat_n with eta_hat(a, i) =
 * 0.05 * (splitmix64(seed ^ (9a + 3 + i)) >> 11) * 2^-53, i = 0..5
 * (splitmix64: Steele, Lea and Flood, OOPSLA 2014). */
int mvpf_init_random(mvpf_problem* p, uint64_t seed);

/* Residual R = dPi/dU of the discrete penalised incremental potential at the
 * current state (Eqs. PenPot, FinalRes; Sec. 3.4), contact term excluded,
 * Dirichlet rows NOT zeroed.  R: device (nullable).  norm_free: host
 * (nullable), Euclidean norm of R over the free dofs of the loading at the
 * current depth. */
int mvpf_residual(mvpf_problem* p, double* R, double* norm_free);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * residual of mvpf_residual (same arguments, same results bitwise) computed
 * with a fixed scratch region compiled into the library -- 64 MiB of device
 * memory per GPU, held from the first call on that GPU until the process
 * ends -- instead of the problem's assembly scratch; neither the call nor the
 * library allocates device memory for it.  The Gauss-point gradients go
 * through the scratch in slabs of whole element layers, so a layer may hold
 * at most mvpf_residual_noalloc_max_layer() elements (nx * ny; 34 880, e.g.
 * 128 x 256); larger layers are rejected with MVPF_EINVAL.  Every call on a
 * GPU shares that GPU's scratch: calls that overlap on one GPU (different
 * host threads, or different streams in flight) race and must be serialised
 * by the caller.  Each call writes every scratch value it reads, so nothing
 * carries over between calls. */
int mvpf_residual_noalloc(mvpf_problem* p, double* R, double* norm_free);
int mvpf_residual_noalloc_max_layer(void);

/* Build the Newton system of Eq. linAlgEq at the current state for the
 * loading at total depth `depth`: tangent K = d^2 Pi / dU^2 on the finest
 * level, and on every coarser level either reassembled at the injected state
 * (Sec. 3.4) or the Galerkin product of the level above (opts.coarse),
 * Dirichlet rows/columns
 * replaced by the identity, right-hand side b_free = -R_free - (K g)_free,
 * b_con = g with g = target - current on constrained dofs (lifting); inverts
 * the 9x9 diagonal blocks (LU, partial pivoting) and factors the coarsest
 * level.  Returns MVPF_ESINGULAR if a block or the coarse matrix is singular. */
int mvpf_newton_system(mvpf_problem* p, double depth);
/* Copy the right-hand side b of the last mvpf_newton_system (device). */
int mvpf_get_rhs(mvpf_problem* p, double* b);

/* y = A_level x with the eliminated operator of the last mvpf_newton_system
 * (Dirichlet rows/columns = identity).  level 0 = finest.  precision
 * MVPF_FP64 uses the FP64 copy (finest level, or every level in FP64 mode),
 * MVPF_MIXED the FP32 copy (mixed mode, levels above the coarsest); on a
 * matrix-free finest level the FP64 / FP32 Gauss-point Hessians.  x, y:
 * device, length 9*n_nodes(level). */
int mvpf_jacobian_apply(mvpf_problem* p, int level, int precision, const double* x, double* y);

/* z = M^-1 v: one application of the preconditioner (V-cycle; identity on the
 * constrained dofs of the finest level).  v, z: device, finest level. */
int mvpf_precondition(mvpf_problem* p, const double* v, double* z);

/* FGMRES(m) with the V-cycle as right preconditioner, x0 = 0 (Sec. 3.4).
 * b: device right-hand side or NULL for the one built by mvpf_newton_system;
 * x: device solution or NULL to keep it internally for mvpf_newton_update.
 * Returns MVPF_ENOTCONV if max_it was reached. */
int mvpf_solve(mvpf_problem* p, const double* b, double* x, mvpf_solve_stats* stats);

/* U <- U + Delta with the internally kept solution of the last mvpf_solve;
 * constrained dofs are set to their targets. */
int mvpf_newton_update(mvpf_problem* p);

/* One Newton iteration of the monolithic scheme (Sec. 3.4, Eq. linAlgEq) at
 * indenter depth `depth`: mvpf_newton_system(depth), mvpf_solve with the
 * system's own right-hand side (stats: nullable), mvpf_newton_update.  The
 * Newton loop of a time step is mvpf_time_step; this is one of its
 * iterations without the convergence test.  Returns MVPF_ESINGULAR (state
 * unchanged) for a singular block or coarse operator; MVPF_ENOTCONV if the
 * solve stopped at max_it (the update is still applied). */
int mvpf_newton_step(mvpf_problem* p, double depth, mvpf_solve_stats* stats);

/* One implicit time step to total depth `depth` (Sec. 3.4): Newton
 * iterations (newton_system, solve, update) until the free-dof residual is
 * <= newton_rtol * ||b_0|| (a linear solve stopped at max_it still gives its
 * update: an inexact Newton step); if not within newton_max iterations, or if
 * a 9x9 diagonal block or the coarsest operator is singular, or the residual
 * is not finite, the attempt fails: the state and depth are restored to their
 * values before the attempt and the depth increment is halved (at most 8
 * times, then MVPF_ENOTCONV).  The
 * material's rho = 1/(m tau) belongs to the whole increment (depth minus the
 * current depth); an attempt over a fraction f of it runs with rho / f (the
 * time step tau is proportional to the increment), and the material's rho is
 * in place again when the call returns.  Any error returned (negative) also
 * leaves the state and depth as they were before the failing attempt.  On
 * success eta_hat_n <- eta_hat and the depth is advanced. */
int mvpf_time_step(mvpf_problem* p, double depth, mvpf_step_stats* stats);

/* Set the viscous coefficient rho = 1/(m tau) of the material (Sec. 2.3: the
 * time-discrete dissipation (rho / 2) |eta_hat - eta_hat_n|^2; it depends on
 * the time step tau, so a caller that chooses its own steps sets it per
 * step).  rho finite and >= 0, else MVPF_EINVAL.  Takes effect with the next
 * residual or system. */
int mvpf_set_viscosity(mvpf_problem* p, double rho);

/* Indentation load of the sphere-contact loading at the current state and
 * depth: P = d/dd of the contact energy at fixed displacements,
 * int eps_n <g>_- n_z dS (n = the sphere's outward normal at the closest
 * point; P >= 0 while the indenter presses).  FP64, deterministic.
 * MVPF_EINVAL for other loadings. */
int mvpf_contact_load(mvpf_problem* p, double* load);

/* Quasi-static indentation run with adaptive time steps (Sec. 3.4, Sec. 4.1):
 * the indenter moves from the current depth to depth_max, then (unload != 0)
 * back to 0, at constant speed v.  The time step enters through the viscous
 * coefficient rho = 1/(m tau), tau = dd / v, so every attempted step sets
 * rho = visc_depth / |dd| (visc_depth = v / m); the material's rho is
 * restored at exit.  Step control: after an accepted step with n Newton
 * iterations the next increment is multiplied by grow if n < newton_desired
 * (7 in the paper) and by shrink if n > newton_desired, within
 * [dd_min, dd_max]; a step not converged within newton_max iterations
 * (mvpf_opts, 12 in the paper) is rejected, the state restored and the step
 * retried with half the increment.  When at most dd + dd_min is left in a
 * phase, the step goes exactly to its end. */
typedef struct {
  double depth_max;
  int unload;
  double dd_init, dd_min, dd_max;
  double grow, shrink;
  int newton_desired;
  double visc_depth;
  int max_steps;
} mvpf_indent_opts;

/* One accepted step: depth after it, indentation load there (as
 * mvpf_contact_load), its depth increment, Newton and FGMRES iterations,
 * rejected attempts before it, and its device times (ms). */
typedef struct {
  double depth, load, dd;
  int newton_iterations, linear_iterations, rejected;
  double assemble_ms, setup_ms, solve_ms;
} mvpf_indent_record;

/* depth_max 0.05, unload 1, dd 0.0025 in [1e-5, 0.01], grow 1.25, shrink 0.8,
 * newton_desired 7, visc_depth 2.857e-4, max_steps 1000. */
void mvpf_default_indent_opts(mvpf_indent_opts* o);

/* Called after every accepted step with its record and index (progress
 * reporting); runs on the calling thread. */
typedef void (*mvpf_indent_callback)(const mvpf_indent_record* rec, int index, void* user);

/* Runs the indentation; rec: caller-owned host array of max_rec >= max_steps
 * records, *n_rec = accepted steps; on_step (nullable) with `user` after each
 * accepted step.  MVPF_EINVAL for another loading kind or bad options
 * (depth_max must exceed the current depth); MVPF_ENOTCONV if a step falls
 * below dd_min or max_steps is reached (the records so far and the last
 * accepted state are kept). */
int mvpf_indent(mvpf_problem* p, const mvpf_indent_opts* o, mvpf_indent_callback on_step, void* user,
                mvpf_indent_record* rec, int max_rec, int* n_rec);

/* Launch-shape tuning (results are bitwise independent of it).  key
 * "row_blocks": number of 256-thread workgroups of the smoother and defect
 * kernels on `level` (0 = one workgroup per 256 rows; fewer makes each
 * workgroup loop over rows in rounds, which keeps the rows in flight within
 * cache reach of each other); "outer_blocks": the same for the outer FP64
 * operator product (level ignored); "small_grid_nodes": levels with at most
 * this many nodes use the latency-oriented small-grid smoother and defect
 * kernels (27 threads per row; default 10000; level ignored).  The two kernel
 * families sum the 27 block products in different orders, so this key alone
 * changes results at rounding level; the others never do.  "coarse_overlap":
 * 1 = the coarsest level's dense inversion runs on a second (default
 * priority) stream, overlapping the assembly of the finer levels; 0 = in
 * order on the problem's stream before them (default 1; level ignored;
 * results unchanged).
 * "assembly_slab_elements": elements per assembly slab (0 = the capacity
 * allocated by mvpf_create: the whole finest level if its Gauss-point and
 * element-matrix buffers take at most 96 GiB, else slabs of 40 GiB).  Levels
 * with more elements are assembled in slabs of whole element layers, one
 * halo layer recomputed per slab; at least 2 nx ny + 64, at most the
 * capacity; level ignored; results bitwise unchanged.
 * "matrix_free": 1 (default for problems with two or more levels) = the
 * finest-level tangent is never assembled: its Gauss-point Hessians (Sec.
 * 3.4; 8 x 120 per element, FP64 and, in mixed mode, FP32) are stored and
 * applied directly in the smoother, the defect and the outer product, and
 * only the diagonal blocks the smoother inverts are assembled; 0 = the
 * finest level is assembled into half-stencil blocks like the others (the
 * blocks are allocated on first use).  Both give the same operator up to
 * rounding (summation order); takes effect at the next mvpf_newton_system;
 * level ignored.  row_blocks on level 0 and outer_blocks apply to the
 * assembled finest level only.  "mf_elements_per_block": elements per
 * workgroup of the matrix-free element kernel, 8, 16 or 32 (64, 128 or 256
 * threads; default 32; level ignored; results bitwise unchanged).
 * "autotune_cache": 1 (default) = mvpf_autotune reuses the results of earlier
 * tuning runs for the same GPU architecture, multigrid precision,
 * finest-level mode (matrix-free or assembled) and level shape (elements per
 * direction) instead of timing again; 0 = always time (and record).  The
 * results are kept for the process; if the environment variable
 * MVPF_TUNE_CACHE names a file, they are also read from it at the first
 * lookup and every new result is appended to it as a "key value" line
 * (level ignored). */
int mvpf_set_tuning(mvpf_problem* p, const char* key, int level, int value);
int mvpf_get_tuning(const mvpf_problem* p, const char* key, int level, int* value);
/* Time candidate launch shapes of the smoother (every level but the coarsest;
 * on a matrix-free finest level its elements per workgroup) and of the outer
 * product (assembled finest level only) on the operators of the last
 * mvpf_newton_system, and keep the fastest; shapes already tuned for the same
 * architecture, precision, finest-level mode and level shape are taken from
 * the tuning cache (tuning key "autotune_cache").  row_blocks_out (nullable,
 * n_levels ints): chosen values per level (on a matrix-free finest level:
 * elements per workgroup), the last entry being the outer product's. */
int mvpf_autotune(mvpf_problem* p, int* row_blocks_out);

/* Per-kernel device timing with HIP events on the problem's stream.  name:
 * "pbj_sweep" (finest-level smoother sweep), "spmv_outer" (finest FP64
 * operator product), "residual" (finest defect), "qp_hessian" (finest-level
 * Gauss-point gradient and Hessian of the density, Sec. 3.2; bytes = its
 * output).  enable != 0 starts
 * recording (and clears totals); stats: launches, summed ms, algorithmic
 * bytes moved per launch. */
int mvpf_kernel_timing(mvpf_problem* p, int enable);
int mvpf_kernel_stats(mvpf_problem* p, const char* name, int* launches, double* total_ms,
                      double* bytes_per_launch);

/* ---- Batches of independent problems --------------------------------------
 * Many independent indentation problems of uneven size (each with its own
 * mesh, material card -- e.g. its own crystal orientation -- and loading)
 * solved together: the problems advance in lockstep, one Arnoldi step of
 * every problem per host synchronisation, and the multigrid V-cycles of all
 * problems run as one captured HIP graph (one graph launch per step) in
 * which every V-cycle operator (sweep, defect, transfer, coarse solve) is
 * one launch covering all problems, whatever their sizes: each problem is a
 * job of the launch, owning a range of its workgroups.  Each problem's
 * numbers are bitwise those of solving it alone with mvpf_solve (under the
 * same tuning: the problems of a batch start with small_grid_nodes = 0, the
 * small-grid kernels pay only in narrow single-problem launches).  Every problem is a full handle (mvpf_batch_problem)
 * on which the single-problem calls work; the batch owns them. */

/* Create n (1..MVPF_MAX_BATCH) problems: meshes[i], mats[i], loads[i] as for
 * mvpf_create; opts (one for all) and stream shared.  On error nothing is
 * left allocated and mvpf_batch_last_error(NULL) describes it. */
int mvpf_create_batch(int n, const mvpf_mesh* meshes, const mvpf_material* mats, const mvpf_loading* loads,
                      const mvpf_opts* opts, void* hip_stream, mvpf_batch** out);
void mvpf_destroy_batch(mvpf_batch* b);
const char* mvpf_batch_last_error(const mvpf_batch* b);
/* Problem i of the batch (owned by the batch; NULL if out of range). */
mvpf_problem* mvpf_batch_problem(mvpf_batch* b, int i);
/* mvpf_newton_system on every problem; depths: n host doubles. */
int mvpf_batch_newton_system(mvpf_batch* b, const double* depths);
/* Solve every problem's Newton system (right-hand side and increment kept
 * inside each problem, as mvpf_solve with b = x = NULL); stats: n entries,
 * solve_ms = the whole batch's time.  The V-cycle graph is captured on the
 * first call and again whenever a problem's options or tuning changed.
 * Returns MVPF_ENOTCONV if any problem did not converge. */
int mvpf_batch_solve(mvpf_batch* b, mvpf_solve_stats* stats);
/* mvpf_newton_update on every problem. */
int mvpf_batch_newton_update(mvpf_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* MVPF_H */
