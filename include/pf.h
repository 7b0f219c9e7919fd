/*
 * pf.h -- C ABI of the MI355X (gfx950) library for one explicit time step of
 * the 3D time-dependent Ginzburg-Landau (TDGL) equation of a ferroelectric
 * film, after Ashraf & Salahuddin, "A Massively Parallel Time Domain Phase
 * Field Model for Multi-domain Ferroelectric Device Simulation",
 * arXiv:1202.6116.
 *
 * The step (Sec. II and III of the paper) combines
 *   - the Landau bulk force (Eq. 1),
 *   - the gradient (domain-wall) force, a 7-point Laplacian (Eq. 2-3),
 *   - the electrostatic field E = -grad phi with eps Lap phi = div P (Eq. 4-5,
 *     17-18), solved by preconditioned conjugate gradients,
 *   - the elastic force of the electrostrictive eigenstrain (Eq. 6, 15),
 *     with the displacement from a trilinear-hex FEM solve K u = f (Eq. 8-16),
 *     also by preconditioned conjugate gradients,
 *   - the predictor-corrector of Eq. 19 (rate carried as state) or forward
 *     Euler.
 * Both solves take the same preconditioner (pf_config.precond): Jacobi, or
 * one geometric multigrid V-cycle per CG iteration.
 *
 * Conventions.
 *   Grid: nodes (i, j, k), 0 <= i < nx, 0 <= j < ny, 0 <= k < nz, spacing h,
 *   linear index n = i + nx (j + ny k) (the paper's natural numbering, x
 *   fastest).  Periodic in x and y.  k = 0 is the substrate side (mechanically
 *   clamped), k = nz - 1 the free top surface.
 *   Vector fields (P, V, u, forces) are structure-of-arrays: component c of
 *   node n at element c*N + n, N = nx ny nz.  The potential phi lives on the
 *   potential grid of Np = nx ny nzp nodes, same ordering: nzp = nz with the
 *   metal top, nz + n_air with the open top (the air planes follow the film
 *   planes).
 *   Potential boundary values: k = -1 is a ghost plane holding phi_bottom.
 *   Metal top (PF_TOP_METAL): k = nz is a ghost plane holding phi_top except
 *   where an electrode covers it (Sec. III.C, Dirichlet electrodes).  Open
 *   top (PF_TOP_OPEN, the open-circuit film of Sec. IV): planes nz .. nzp-1
 *   are air (permittivity eps_air; z-faces across the film/air interface take
 *   the harmonic mean), the top of the air has a zero normal field, and the
 *   electrode nodes of plane nz are Dirichlet nodes holding the electrode
 *   voltage (phi_top is unused).
 *   Voigt order (xx, yy, zz, xy, yz, zx) with engineering shear (Eq. 12).
 *
 * Precision.  PF_FP64: every array is double.  PF_FP32_REFINE: P, V and
 *   forces are float, phi and u are double (the refined masters); the sweeps
 *   run in float, dot products and the outer residuals in double.
 *   PF_FP32_SOLVES: the solves of PF_FP32_REFINE (float CG and multigrid
 *   sweeps on the correction, double dot products, outer residuals and
 *   masters), everything else as PF_FP64 (double state, force and update),
 *   so the state keeps double precision while the solves move half the
 *   bytes.
 *
 * Memory.  The caller owns all device memory: the state arrays it passes in
 *   and one workspace of pf_workspace_size() bytes (256-byte aligned).  The
 *   library never allocates or frees device memory.  It allocates a small
 *   pinned host block per context (status read-back).
 *
 * Streams.  Every call enqueues on the stream given to pf_init and returns
 *   without waiting, except calls that return host values (pf_step and the
 *   solves, which read back iteration counts; pf_energy), which synchronise
 *   that stream.  Each context also owns one more stream (default priority)
 *   and one host worker thread, created by pf_init and released by
 *   pf_destroy: when a step (or an adjoint step) solves both fields, the FEM
 *   solve runs there, forked from and joined back into the caller's stream
 *   by events, concurrently with the Poisson solve; results are bitwise
 *   those of the sequential order.  With per-launch timing on (pf_timing)
 *   the solves run one after the other on the caller's stream.
 *
 * Errors.  Every call returns a pf_status; nothing is thrown across the ABI.
 *   pf_last_error() describes the last failure of a context.  A context is
 *   not thread-safe: use one per host thread.
 */
#ifndef PF_H
#define PF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PF_OK = 0,
  PF_EINVAL = -1,      /* invalid argument or configuration */
  PF_ENOMEM = -2,      /* workspace too small */
  PF_EHIP = -3,        /* HIP runtime error */
  PF_ENOCONV = -4,     /* a CG solve hit maxit; results are the last iterate */
  PF_ENONFINITE = -5,  /* NaN/Inf found in a reduction; results are undefined */
  PF_ESTATE = -6       /* call out of order (e.g. pf_step before pf_set_state) */
} pf_status;

/* terms: which contributions enter the force (tests switch terms off) */
enum { PF_TERM_LANDAU = 1, PF_TERM_GRAD = 2, PF_TERM_ELEC = 4, PF_TERM_ELAS = 8, PF_TERM_ALL = 15 };
/* precond: preconditioner of both conjugate-gradient solves (Poisson and FEM) */
enum { PF_PRECOND_JACOBI = 0, PF_PRECOND_MG = 1 };
/* top_bc: electrostatic condition above the film */
enum { PF_TOP_METAL = 0, PF_TOP_OPEN = 1 };
/* integrator */
enum { PF_INT_PC = 0, PF_INT_EULER = 1 };
/* precision */
enum { PF_FP64 = 0, PF_FP32_REFINE = 1, PF_FP32_SOLVES = 2 };

/* An electrode: the half-open node rectangle [x0, x1) x [y0, y1) of the top
 * ghost plane held at `volts` (Sec. III.C).  Electrodes must not overlap. */
typedef struct {
  int32_t x0, x1, y0, y1;
  double volts;
} pf_electrode;

typedef struct {
  int32_t nx, ny, nz;           /* nx, ny >= 3, nz >= 3 */
  double h;                     /* grid spacing (> 0) */
  double a1, a11, a12;          /* Landau coefficients, Eq. 1 */
  double G;                     /* gradient coefficient G11, Eq. 2-3 */
  double L;                     /* mobility: dP/dt = -L dF/dP, Eq. 7 */
  double dt;                    /* time step (> 0), Eq. 19 */
  double eps_b;                 /* permittivity in Eq. 18 (> 0) */
  double phi_bottom, phi_top;   /* ghost-plane potentials */
  int32_t n_electrodes;         /* 0..64 */
  const pf_electrode *electrodes;  /* host array, copied by pf_init */
  double C11, C12, C44;         /* cubic elastic stiffness (Eq. 13 generalised) */
  double Q11, Q12, Q44;         /* electrostriction, Eq. 15 */
  int32_t integrator;           /* PF_INT_PC (default) or PF_INT_EULER */
  int32_t precision;            /* PF_FP64, PF_FP32_REFINE or PF_FP32_SOLVES */
  double tol_phi, tol_u;        /* CG stop: ||b - A x||_2 <= tol ||b||_2 */
  int32_t maxit;                /* CG iteration cap per solve (> 0) */
  int32_t warm_start;           /* 0: solves start from zero; 1: from the previous
                                   solution (the paper's warm start); 2: from the
                                   polynomial extrapolation to the next step of the
                                   last solutions (see extrap_order); 3: as 2, the
                                   order of each refresh (0..extrap_order) chosen
                                   as the one whose extrapolation from the solutions
                                   before the newest came closest to the newest
                                   (squared second differences along x of the error
                                   on a fixed 1/64 sample of the field); the adjoint
                                   solves extrapolate as with 2 */
  uint32_t terms;               /* PF_TERM_* mask */
  int32_t nonlocal_every;       /* refresh phi and u every k steps (<= 1: every
                                   step), the paper's Fig. 3d option */
  int32_t extrap_order;         /* warm_start 2 and 3: the guess is the polynomial through
                                   the last solution and up to extrap_order (0..8)
                                   earlier ones, x_next = sum_t (-1)^t C(m+1,t+1)
                                   x_{n-t}; the order grows with the history kept
                                   since pf_set_state/pf_restore_state/pf_set_params */
  double noise_sigma;           /* thermal noise (the random force zeta of Eq. 7),
                                   >= 0: the force of step s gains
                                   zeta = (noise_sigma / sqrt(dt)) xi_s, so one Euler
                                   step adds noise_sigma sqrt(dt) xi_s; V0 has none */
  uint64_t noise_seed;          /* key of the noise generator (see pf_noise) */
  int32_t top_bc;               /* PF_TOP_METAL (ghost plane) or PF_TOP_OPEN (air) */
  int32_t n_air;                /* PF_TOP_OPEN: air planes, 1 .. 4 nz */
  double eps_air;               /* PF_TOP_OPEN: permittivity of the air (> 0) */
  double misfit[3];             /* in-plane strain the substrate imposes on the film
                                   (xx, yy, engineering xy; grid axes): the clamped
                                   plane holds the affine displacement of that strain
                                   and u is the displacement relative to it (Sec. III.B) */
  double rotation[9];           /* crystal-to-grid rotation R, row-major (v_grid =
                                   R v_crystal; all zeros: identity).  a1, a11, a12,
                                   C and Q are crystal-axis coefficients; P, E, u and
                                   the stresses live on the grid axes (Sec. II) */
  int32_t precond;              /* Poisson and FEM solves alike:
                                   PF_PRECOND_JACOBI (the paper's
                                   Jacobi-preconditioned CG) or PF_PRECOND_MG (CG
                                   preconditioned by one multigrid V-cycle: Galerkin
                                   coarse operators of the trilinear prolongation,
                                   one damped Jacobi sweep before and after, dense
                                   coarsest solve; same solution, same stopping
                                   test, far fewer iterations).  Grids too small to
                                   coarsen fall back to Jacobi. */
} pf_config;

typedef struct {
  int32_t iters;      /* CG iterations (FP32_REFINE: inner iterations, summed) */
  int32_t outer;      /* refinement sweeps (FP32_REFINE), 1 in FP64 */
  double relres;      /* final ||b - A x|| / ||b|| (recursive residual) */
} pf_solve_stats;

typedef struct {
  int32_t steps;                 /* steps taken by the call */
  int64_t iters_phi, iters_u;    /* CG iterations summed over the call */
  int32_t last_iters_phi, last_iters_u;
  int32_t solves_phi, solves_u;  /* solves performed (nonlocal_every skips some) */
  double relres_phi, relres_u;   /* largest final relative residual */
} pf_step_stats;

typedef struct pf_ctx pf_ctx;

/* Bytes of device workspace a context for `cfg` needs (for all calls,
 * including pf_energy and the adjoint).  Validates cfg. */
pf_status pf_workspace_size(const pf_config *cfg, size_t *bytes);

/* Binds a context to cfg, a device workspace of at least
 * pf_workspace_size() bytes (256-byte aligned, owned by the caller, must
 * outlive the context) and a HIP stream (NULL: the null stream).  Builds the
 * FEM operator tables and the ghost planes, then waits for the stream.  The
 * potential of the boundary values alone (for pf_energy) and the electrode
 * basis potentials (for the adjoint) are solved on first use, to
 * min(tol_phi, 1e-12).  *out is set on success. */
pf_status pf_init(const pf_config *cfg, void *dev_workspace, size_t bytes, void *hip_stream, pf_ctx **out);

/* pf_init for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the
 * context's workspace is the library's static device array of 64 MiB
 * (one per GPU, held from the first use on that GPU until the process
 * ends; enough for a 64 x 64 x 16 film in FP64 with the multigrid), not
 * caller memory.  Binds to the current device and to hip_stream (NULL: the
 * null stream).  The call allocates no device memory and no pinned host
 * memory and creates no stream, event or thread; the context's two solves
 * of a step therefore run one after the other on hip_stream (results are
 * bitwise those of a pf_init context).  Rejects a configuration whose
 * pf_workspace_size exceeds 64 MiB with PF_EINVAL (message on stderr).  One
 * context per GPU at a time: while one made by this call lives, a second on
 * the same device returns PF_ESTATE; pf_destroy (which waits for the
 * stream) frees the array for the next.  The array keeps the last
 * context's contents: initialisation clears what must start at zero, as
 * pf_init does for the caller's uninitialised workspace.  Calls that
 * overlap on one context race (contexts are not thread-safe). */
pf_status pf_init_static(const pf_config *cfg, void *hip_stream, pf_ctx **out);

/* Loads the polarisation P (device, 3N) as the current state, with optional
 * initial guesses phi0 (Np doubles) and u0 (3N doubles) for the first solves
 * (NULL: zero).  For the predictor-corrector it solves phi and u at P and
 * sets the carried rate V0 = F(P) (the paper does not state V0; this is the
 * reading taken).  Synchronises.  Resets the step counter to 0. */
pf_status pf_set_state(pf_ctx *ctx, const void *P, const void *phi0, const void *u0);

/* Restores a full state saved by pf_get_state (P, V: state precision; phi,
 * u: double; none may be NULL) and the step counter.  Asynchronous. */
pf_status pf_restore_state(pf_ctx *ctx, const void *P, const void *V, const void *phi, const void *u, int64_t step);

/* Copies the current state into caller arrays (any may be NULL): P and V
 * (3N, state precision), phi (Np doubles), u (3N doubles), and the step
 * counter into *step (host; may be NULL).  The counter is an addition to the
 * four state arrays: checkpoints need it to resume the thermal noise of
 * Eq. 7, whose variates are keyed by the step.  Asynchronous. */
pf_status pf_get_state(const pf_ctx *ctx, void *P, void *V, void *phi, void *u, int64_t *step);

/* Advances the state by nsteps (Eq. 19 or forward Euler): per step one
 * Poisson solve and one FEM solve (both warm-started when configured; every
 * nonlocal_every steps only), and one fused force + update sweep.
 * Synchronises at least once per solve to read convergence.  stats may be
 * NULL.  Returns PF_ENOCONV if some solve hit maxit (the step still
 * completes), PF_ENONFINITE on NaN/Inf (the state is then undefined). */
pf_status pf_step(pf_ctx *ctx, int32_t nsteps, pf_step_stats *stats);

/* Poisson solve for a given polarisation P (device, 3N, state precision),
 * Eq. 4-5 discretised as Eq. 17-18 (Sec. III.C): div_h(eps grad_h phi) = div_h P (eps = eps_b in the film, eps_air in the
 * air of the open top) with the boundary values.  phi (device, Np doubles)
 * is the initial guess when warm_start is set and receives the solution
 * (electrode nodes of the open top: their voltage).  Synchronises. */
pf_status pf_solve_phi(pf_ctx *ctx, const void *P, void *phi, pf_solve_stats *stats);

/* FEM solve K u = f(P) for a given polarisation (Eq. 15-16): clamped k = 0
 * (u = 0 there), free top, periodic x and y.  u (device, 3N doubles) is the
 * initial guess when warm_start is set and receives the solution.
 * Synchronises. */
pf_status pf_solve_u(pf_ctx *ctx, const void *P, void *u, pf_solve_stats *stats);

/* Force F = -L dF/dP at P (Eq. 7 without noise) for given phi (Np doubles)
 * and u (3N doubles), written to F (3N, state precision).  No solves.  In
 * PF_FP32_REFINE the force is evaluated in float from rounded phi and u.
 * Asynchronous. */
pf_status pf_force(pf_ctx *ctx, const void *P, const void *phi, const void *u, void *F);

/* The standard normal variates xi_s of step s of the thermal noise, written
 * to xi (device, 3N doubles, component-major like P), whatever noise_sigma
 * is.  Node n = i + nx (j + ny k) of step s takes one Philox4x32-10 block
 * (Salmon et al., SC 2011) with counter words (n mod 2^32, n / 2^32,
 * s mod 2^32, s / 2^32) and key words (seed mod 2^32, seed / 2^32); with u_w
 * = (w + 1) 2^-32 and a_w = 2 pi w 2^-32, Box-Muller gives xi_x =
 * sqrt(-2 ln u_w0) cos a_w1, xi_y = sqrt(-2 ln u_w0) sin a_w1 and xi_z =
 * sqrt(-2 ln u_w2) cos a_w3.  pf_step draws step s = the step counter before
 * the step (pf_get_state).  Asynchronous. */
pf_status pf_noise(pf_ctx *ctx, int64_t step, double *xi);

/* Free energy of the current P (Eq. 1-6 on the grid of Sec. III.A):
 * out[0..4] = bulk (Eq. 1), gradient (Eq. 2), electrostatic (Eq. 4-5),
 * elastic (Eq. 6), total (host doubles), evaluated in FP64.  Solves phi and u at P
 * in FP64 (warm-started from the state's solutions, configured
 * tolerances); the electrostatic energy is split into the polarisation
 * part, (h^3/2) rho^T A^-1 rho, and the applied part -h^3 P . E_app (linear
 * superposition with the potential of the boundary values).  The
 * polarisation and elastic parts are evaluated as the stationary values of
 * their quadratic forms, so their error is second order in the solve
 * error.  Synchronises. */
pf_status pf_energy(pf_ctx *ctx, double out[5]);

/* Changes electrode voltages (n_electrodes host doubles, NULL: keep) and
 * the Landau coefficient a1 (used by the differentiable layer).  A
 * non-finite value returns PF_EINVAL and changes nothing. */
pf_status pf_set_params(pf_ctx *ctx, const double *volts, double a1);

/* One reverse step of the discrete adjoint of pf_step (needs
 * nonlocal_every <= 1; the linearised solves run in FP64 in both
 * precisions, warm-started from the previous adjoint step's solutions, with
 * warm_start 2 extrapolated from the last extrap_order + 1 of them).  In: the state
 * (P_n, V_n) before forward step n (device, 3N each, state precision; V_n is
 * ignored for Euler) and the adjoints (lamP, lamV) of the state after it;
 * out: lamP, lamV overwritten by the adjoints of the state before it, and
 * dtheta (host, n_electrodes + 1 doubles: dJ/dV_1..dJ/dV_ne, dJ/da1)
 * accumulated.  Re-solves u at the linearisation point (warm-started), then
 * one adjoint Poisson and one adjoint FEM solve.  Synchronises. */
pf_status pf_adjoint_step(pf_ctx *ctx, const void *P_n, const void *V_n, void *lamP, void *lamV, double *dtheta);

/* pf_adjoint_step with the displacement at the linearisation point given:
 * u_n (device, 3N doubles) is what forward step n solved for (the u that
 * pf_get_state returns after that step), so only the adjoint Poisson and
 * FEM systems are solved.  u_n = NULL: the same as pf_adjoint_step.
 * Synchronises. */
pf_status pf_adjoint_step_u(pf_ctx *ctx, const void *P_n, const void *V_n, const void *u_n, void *lamP, void *lamV,
                            double *dtheta);

/* Folds the initial rate V0 = F(P0) of the predictor-corrector into the
 * adjoints: lamP += (dF/dP)(P0) lamV, dtheta += lamV . dF/dtheta(P0),
 * lamV = 0 (no-op for Euler).  Ends the reverse sweep in both cases: the
 * next adjoint step starts its solves from zero instead of from this sweep's
 * adjoint solutions.  Synchronises. */
pf_status pf_adjoint_initial_rate(pf_ctx *ctx, const void *P0, void *lamP, void *lamV, double *dtheta);

/* Kernel classes for pf_timing. */
enum {
  PF_KC_POISSON_SETUP = 0, /* Poisson rhs + initial residual */
  PF_KC_POISSON_A,         /* Poisson direction update + operator + p.q */
  PF_KC_POISSON_B,         /* Poisson residual update + r.z */
  PF_KC_FEM_SETUP,         /* FEM body force + initial residual */
  PF_KC_FEM_A,             /* FEM direction update + operator + p.q */
  PF_KC_FEM_B,             /* FEM residual update + r.z */
  PF_KC_FORCE,             /* force + time update */
  PF_KC_FINISH,            /* deferred solution update of a solve */
  PF_KC_REDUCE,            /* single-block reductions of the CG scalars */
  PF_KC_OTHER,             /* fills, copies, energy and adjoint sweeps */
  PF_KC_MG,                /* multigrid V-cycles: coarse levels, transfers, first sweeps */
  PF_KC_MG_U0,             /* FEM multigrid: residual and last sweep on the solver grid */
  PF_KC_MG_PHI0,           /* Poisson multigrid: residual and last sweep on the solver grid */
  PF_KC_COUNT
};

/* Modes of pf_timing. */
enum {
  PF_TIMING_OFF = 0,
  PF_TIMING_EVENTS = 1, /* HIP events around every launch, byte and launch counts;
                           the two solves of a step run one after the other */
  PF_TIMING_BYTES = 2   /* launch and byte counts only (no events); the solves
                           stay concurrent */
};

/* Per-kernel-class accounting of launches on the context's streams.
 * Returns what was accumulated since the last call (arrays of PF_KC_COUNT,
 * each may be NULL): milliseconds between the events around each launch
 * (PF_TIMING_EVENTS only), launch counts, and algorithmic bytes: the HBM
 * traffic each launch must move at least, its compulsory reads and writes
 * with every stencil neighbour counted once (e.g. a FEM CG direction
 * update + operator launch: r or z, the old direction and x read, the new
 * direction and x written, 5 x 3 values per node above the clamped plane).
 * Launches that return at entry after a solve has converged are not
 * counted.  Resets the accumulators and sets the mode (PF_TIMING_*; other
 * values: PF_EINVAL).  Synchronises. */
pf_status pf_timing(pf_ctx *ctx, int mode, double *ms, int64_t *launches, double *bytes);

/* Diagnostic (host only, no GPU needed): the constant 27-point operator
 * tables the kernels use for cfg, as doubles in this order:
 *   K[2][3][3][27]   stiffness rows, interior planes then the top plane:
 *                    (K u)_c = sum_e sum_o K[z][c][e][o] u_e(n + o)
 *   Bf[2][3][6][27]  body force of a nodal Voigt stress sigma0 = C eps0
 *   Su[3][6][3][27]  int N_n eps_v(u) for bottom, interior, top planes
 *   Ms[3][27]        consistent mass for bottom, interior, top planes
 * with offset o = (dx+1) + 3 (dy+1) + 9 (dz+1).  `count` is the capacity of
 * out in doubles; needs at least pf_fem_table_size() of them. */
size_t pf_fem_table_size(void);
pf_status pf_fem_tables(const pf_config *cfg, double *out, size_t count);

/* Diagnostic (host only): the multigrid hierarchy used with PF_PRECOND_MG,
 * field 0 for the Poisson operator, 1 for the FEM operator.  *nlevels
 * receives the number of levels; for the first max_levels of them
 * dims[3l..3l+2] = (nx, ny, nz) and omega[l] = the Jacobi smoother's damping
 * (either array may be NULL).  The Poisson levels count the ghost planes: the
 * bottom one (plane 0) and, with the metal top, the top one, both fixed. */
pf_status pf_mg_levels(const pf_config *cfg, int32_t field, int32_t *nlevels, int32_t *dims, double *omega,
                       int32_t max_levels);

/* Diagnostic (host only): the operator of level `level` as nz x nc x nc x 27
 * doubles (nc = 1 for field 0, 3 for field 1), T[k][c][e][o]: row component
 * c of plane k against component e of the neighbour at offset o (same
 * numbering as the FEM tables); level 0 is the solver's operator, levels
 * >= 1 the Galerkin products P^T A P.  `count` is the capacity of out. */
pf_status pf_mg_table(const pf_config *cfg, int32_t field, int32_t level, double *out, size_t count);

const char *pf_status_str(pf_status s);
const char *pf_last_error(const pf_ctx *ctx);

/* Releases the context's host state (not the caller's device memory). */
void pf_destroy(pf_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* PF_H */
