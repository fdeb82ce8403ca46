/*
 * stokes.h -- C-ABI of the MI355X (gfx950) variable-coefficient Stokes solver.
 *
 * The operation is one implicit solve of the conservative momentum and
 * continuity equations on a staggered MAC grid (Nangia, Patankar & Bhalla,
 * arXiv:1901.07892, Sec. 4.2.2, eqs. eq_c_discrete_momentum and
 * eq_c_discrete_continuity, layout of Sec. 3.1):
 *
 *     (rho_face/dt) u - theta * div_h[ mu (grad_h u + grad_h u^T) ] + grad_h p = f
 *                                                          -div_h u = g
 *
 * rho is given on faces (the face density the momentum equation uses), mu at
 * cell centres; shear viscosities on cell edges (2D: nodes) are the harmonic
 * mean of the surrounding cells (Sec. 4.2, footnote on harmonic averaging).
 * theta scales the implicit viscous operator: 1 gives the full operator, 1/2
 * the Crank-Nicolson half of Sec. 4.2.2.  By default every boundary is a
 * no-slip wall: wall-normal velocity is zero and is not an unknown, tangential
 * ghosts are minus the interior value, and the pressure is defined up to a
 * constant (returned with zero mean).  An axis may be periodic instead
 * (stokes_grid.periodic), and the top of the vertical axis may be the wave
 * tank's open boundary of Sec. 7.1 (stokes_options.open_top: zero pressure
 * there, so the pressure has no free constant).
 *
 * The solver is restarted flexible GMRES on the coupled (u, p) system
 * (Sec. 4.2.4), right-preconditioned by a projection step with a
 * local-viscosity pressure update whose velocity and pressure subsolves are
 * geometric-multigrid cycles with red-black Gauss-Seidel smoothing (the
 * pressure smoother over-relaxed, red-black SOR, see p_omega).
 *
 * Conventions for every entry point
 *   - Arrays are C order with x fastest.  u is (Nz, Ny, Nx+1), v is
 *     (Nz, Ny+1, Nx), w is (Nz+1, Ny, Nx), p and mu are (Nz, Ny, Nx).  In 2D
 *     Nz = 1 and every w / rho_z pointer is NULL.
 *   - Every array pointer (coefficients, right-hand sides, solutions and the
 *     workspace) is a DEVICE pointer owned by the caller.  The library never
 *     allocates device memory: everything it keeps lives in the workspace.
 *   - Wall-normal face entries are ignored on input and written as 0 on output
 *     (the faces of an open top, see stokes_options.open_top, are not walls).
 *   - Work is queued on the caller's HIP stream (passed as void*; NULL is the
 *     default stream).  A context belongs to one stream and is not thread-safe.
 *   - Negative status codes mean nothing was written to the outputs.  No C++
 *     exception crosses this interface.
 */
#ifndef PAPER_1901_07892_STOKES_H
#define PAPER_1901_07892_STOKES_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    STOKES_OK = 0,
    STOKES_NOT_CONVERGED = 1,   /* max_iters reached or stagnation; best iterate returned */
    STOKES_BREAKDOWN = 2,       /* Arnoldi breakdown without convergence */
    STOKES_EINVAL = -1,         /* bad argument: grid, options, rho <= 0, mu < 0, NULL pointer */
    STOKES_ESHAPE = -2,         /* grid unsupported (e.g. fewer than 2 cells along an axis) */
    STOKES_ENOMEM = -3,         /* workspace smaller than stokes_workspace_size() */
    STOKES_EHIP = -4,           /* a HIP runtime call failed */
    STOKES_ENAN = -5            /* NaN or Inf in the right-hand side, the guess or the residual */
} stokes_status;

typedef struct {
    int dim;          /* 2 or 3 */
    int n[3];         /* cells Nx, Ny, Nz (Nz ignored and taken as 1 in 2D) */
    double h[3];      /* spacings hx, hy, hz */
    int periodic[3];  /* per axis: 0 no-slip walls at both ends, 1 periodic (an even
                         number of cells; cells and faces 0 .. N-1 wrap).  Arrays keep
                         the wall layouts below: on a periodic axis the last face
                         (index N) repeats face 0, is ignored on input and receives
                         face 0's value on output.  Only the solve (setup, apply,
                         solve, pressure_op and the learned hooks) takes periodic axes;
                         the steps around it (coefficients, explicit right-hand side,
                         rigid projection, density transport, wave inflow and its
                         lift) need walls and return STOKES_EINVAL. */
} stokes_grid;

typedef struct {
    int precision;       /* 0: all FP64; 1: multigrid in FP32 inside FP64 FGMRES */
    double visc_scale;   /* theta; 1.0 full viscous operator, 0.5 Crank-Nicolson half */
    double cont_scale;   /* weight sigma of the continuity rows in the residual norm,
                            ||(r_u, r_p)||^2 = ||r_u||^2 + sigma^2 ||r_p||^2;
                            0 = automatic balance (see stokes_solve), 1 = plain 2-norm */
    int restart;         /* FGMRES restart length m (>= 1) */
    int max_iters;       /* total FGMRES iterations allowed */
    int nu1, nu2;        /* pre- and post-smoothing sweeps per V-cycle level */
    int vel_cycles;      /* velocity V-cycles per preconditioner application (>= 0) */
    int p_cycles;        /* pressure cycles in the first preconditioner application of each
                            FGMRES restart cycle (>= 1), 0 = automatic: 4 for 3D FP64, else 3 */
    int coarse_sweeps;   /* smoothing sweeps on the coarsest velocity level (and on the
                            coarsest pressure level when it is too big for a dense solve) */
    int vel_levels;      /* velocity multigrid levels.  0 = automatic: a single level (the
                            smoother alone) when the viscous part of every momentum diagonal
                            is below 1% of its mass term rho/dt -- the coarse-grid correction
                            can then improve the subsolve by at most that fraction -- and the
                            full hierarchy otherwise.  n > 0: min(n, pressure levels). */
    int vel_sweeps;      /* red-black sweeps of the velocity smoother when the velocity
                            hierarchy is a single level (>= 1) */
    int p_prolong;       /* pressure prolongation: 0 piecewise constant, 1 bi/trilinear */
    int vel_smoother;    /* 0: red-black Gauss-Seidel.  1: when the velocity hierarchy is a
                            single level with one sweep and one cycle, that sweep is a point
                            Jacobi (diagonal) step folded into the projection kernels;
                            otherwise red-black Gauss-Seidel is used */
    int orth;            /* Arnoldi orthogonalisation: 1 classical Gram-Schmidt (default; the
                            residual is always recomputed before returning, so a loss of
                            orthogonality can only cost iterations), 2 twice */
    int matvec_z;        /* 3D matvec kernel: 1 z-marching (register reuse along z), 0 one
                            thread per point; same result to rounding */
    int p_gamma;         /* pressure cycle: 1 V-cycle, 2 W-cycle (two coarse cycles per level) */
    int p_small;         /* 3D: 1 runs the pressure cycle from the finest level (below the
                            finest, at most 64^3 cells) whose cycle fits in the LDS of one
                            workgroup down to the coarsest as one single-workgroup launch per
                            visit (same passes and arithmetic as 0); 0 one launch per pass */
    int p_wdepth;        /* levels that use p_gamma coarse cycles: the p_wdepth finest (0 =
                            all); coarser levels take one (a V-cycle below them) */
    int p_cycles_next;   /* pressure cycles in the later applications (>= 1), 0 = automatic:
                            for 3D FP64 when p_cycles is automatic 5 with the automatic p_omega
                            and 6 with any other, else p_cycles (FGMRES is flexible, so the
                            preconditioner may change between iterations) */
    int p_nu_second;     /* pre- and post-smoothing sweeps on the second-finest pressure level
                            (>= 0; the coarser levels keep nu1 / nu2).  0 = automatic: with FP64
                            multigrid and W-cycles (the second level is cycled twice per visit of
                            the finest, the third and fourth four times) at most one sweep on
                            each side of the second (min(nu1, 1), min(nu2, 1)) and one
                            pre-smoothing sweep on the third and fourth (min(nu1, 1)), and, with
                            the automatic p_omega on a 3D grid, one post-smoothing sweep
                            (min(nu2, 1)) on the levels of at most 16^3 cells; otherwise
                            nu1 / nu2 */
    int open_top;        /* 1: the upper end of the vertical axis (y = Ly in 2D, z = Lz in 3D) is
                            the wave tank's open top (Sec. 7.1): zero pressure and zero tangential
                            velocity there, and the vertical velocity on its faces (index Ny in 2D,
                            Nz in 3D of v / w) is an unknown, read from the right-hand side and the
                            guess and written in the solution.  The pressure ghost above the top
                            is minus the cell below (p = 0 on the face) and so is the normal
                            viscous stress (d w / d z = 0 on the face, from continuity with zero
                            tangential velocity); the pressure has no free constant, so neither
                            rhs_p nor p is made mean-free.  Needs the single-level diagonal
                            velocity step (a mass-dominated operator, as at every workload here;
                            EINVAL otherwise).  0 (default): walls everywhere. */
    double p_omega;      /* over-relaxation factor of the red-black pressure smoother on every
                            level (red-black SOR): each point's Gauss-Seidel value g replaces its
                            old value e by e + p_omega (g - e); 1 is plain Gauss-Seidel.  0 =
                            automatic: 1.1 on 3D grids, 1 in 2D; otherwise in (0, 2) */
} stokes_options;

typedef struct {
    int iters;            /* FGMRES iterations (= preconditioner applications) */
    int restarts;
    int vcycles;          /* velocity + pressure V-cycles */
    int levels;           /* multigrid levels built */
    double rel_res_est;   /* Givens estimate at exit, weighted norm */
    double rel_res_true;  /* recomputed ||b - K x|| / ||b|| in FP64, weighted norm */
    double rel_res_plain; /* the same in the plain 2-norm */
    double rel_res_mom;   /* ||r_u|| / ||b|| (plain) */
    double rel_res_cont;  /* ||r_p|| / ||b|| (plain) */
    double sigma;         /* continuity weight used */
    double g_mean;        /* mean removed from rhs_p before solving */
    double ms_total;      /* wall time of the call on the host, milliseconds */
    int fell_back;        /* 1 if the learned stage was switched off for stagnation */
    int small_level;      /* first pressure level cycled in one workgroup (p_small), -1 none */
} stokes_stats;

typedef struct stokes_ctx stokes_ctx;

/* Fill *opts with the defaults (FP64, theta 1, automatic sigma, restart 30,
 * max_iters 200, (2,2) smoothing, one velocity cycle and an automatic number of
 * pressure cycles (4 then 5 for 3D FP64, otherwise 3) that are W-cycles on
 * the two finest levels and V-cycles below, red-black SOR smoothing with an
 * automatic relaxation factor (1.1 in 3D, 1 in 2D), 40 coarse sweeps,
 * automatic velocity levels, 1 single-level velocity sweep, piecewise-constant
 * pressure prolongation, diagonal velocity step, one-pass Gram-Schmidt, z-marching
 * matvec, small levels cycled in one workgroup, in FP64 one sweep on each side on
 * the second-finest pressure level and one pre-smoothing sweep on the third and
 * fourth). */
void stokes_default_options(stokes_options *opts);

/* Bytes of device workspace that stokes_setup needs for this grid and these
 * options (opts may be NULL for the defaults).  Returns 0 for an invalid grid.
 * Host-only; makes no HIP call. */
size_t stokes_workspace_size(const stokes_grid *grid, const stokes_options *opts);

/* Build a solver context for one coefficient set (once per time step).
 *   rho_face[3]  face densities (rho_face[2] NULL in 2D); interior values must be > 0
 *   mu_cell      cell viscosities, >= 0
 *   dt           time step (> 0); the mass term is rho_face/dt
 *   workspace    device buffer of ws_bytes >= stokes_workspace_size(grid, opts),
 *                owned by the caller and kept alive until stokes_destroy; any
 *                alignment (the library starts at its first 256-byte boundary)
 *   stream       hipStream_t (as void*)
 * Validates shapes and options on the host (ESHAPE for fewer than 2 cells along
 * an axis or a grid whose solution vector would exceed 2^30 entries; EINVAL
 * for any other bad argument), copies the coefficients into the workspace (the
 * caller may free its arrays afterwards), builds the multigrid hierarchy and
 * factors the coarsest pressure problem.  Checks rho > 0 and
 * mu >= 0 on the device (EINVAL).  Blocks until setup has finished.  On success
 * *out owns a host-side context to release with stokes_destroy. */
stokes_status stokes_setup(const double *const rho_face[3], const double *mu_cell, double dt,
                           const stokes_grid *grid, const stokes_options *opts,
                           void *workspace, size_t ws_bytes, void *stream, stokes_ctx **out);

/* y = K x: y_u = A x_u + G x_p on interior faces, y_p = -D x_u on cells.
 * Asynchronous on the context's stream; wall-normal outputs are 0.  In-place
 * (y aliasing x) is not allowed. */
stokes_status stokes_apply(stokes_ctx *ctx, const double *const x_u[3], const double *x_p,
                           double *const y_u[3], double *y_p);

/* Solve K x = (rhs_u, rhs_p) to ||b - K x|| <= tol ||b|| in the weighted norm
 * ||(a, c)||^2 = ||a||^2 + sigma^2 ||c||^2 over interior unknowns, with sigma =
 * opts.cont_scale, or, when that is 0, sigma = a_ref * l / pi: l is the
 * longest side of the domain and a_ref = sqrt(min rho * max rho)/dt +
 * theta * max(mu) * (pi/l)^2.  This balances the momentum rows (scale rho/dt)
 * against the continuity rows (scale 1/h) at the slowest pressure mode; in the
 * plain 2-norm the system's condition number is near 1e14 and the pressure is
 * barely determined.  With rhs_p = 0 and sigma >= 1 (every workload here has
 * sigma > 1e4), convergence in this norm implies convergence in the plain
 * 2-norm (stats->rel_res_plain reports it either way); with sigma < 1 the
 * continuity rows are under-weighted and the plain residual can exceed tol.
 * The mean of rhs_p (incompatible with walls everywhere) is removed first and
 * reported in stats->g_mean.  x holds the initial guess on entry (its wall
 * entries ignored) and the solution on exit (p with zero mean); the residual is
 * recomputed in FP64 before returning.  Blocks until done.  stats may be NULL.
 * Returns OK, NOT_CONVERGED (best iterate in x), BREAKDOWN, ENAN, EINVAL or EHIP.
 * ENAN: a NaN or Inf among the values read (the right-hand side, or the initial
 * guess; x is then left untouched), or a non-finite residual during the solve. */
stokes_status stokes_solve(stokes_ctx *ctx, const double *const rhs_u[3], const double *rhs_p,
                           double tol, double *const x_u[3], double *x_p, stokes_stats *stats);

/* Measurement hook.  Kernel classes that can be timed: */
enum {
    STOKES_PROF_MATVEC = 0,    /* fine-level K x and b - K x (k_apply3_z / k_apply) */
    STOKES_PROF_P_SWEEP = 1,   /* fused 3D red-black pressure sweep on the finest level: 6 fields
                                  (5 from a zero guess) + 1/8 field with a folded prolongation */
    STOKES_PROF_MULTIDOT = 2,  /* Arnoldi inner products, up to 8 vectors per launch */
    STOKES_PROF_MAXPY = 3      /* Arnoldi vector updates, up to 8 vectors per launch */
};

/* Time every launch of one kernel class (kernel = -1 stops) with a pair of HIP
 * events on the context's stream during the following stokes_solve calls, and
 * add up the algorithmic bytes each launch must move (unique inputs and
 * outputs of that launch, documented with each class).  The events are created
 * here on first use (at most 8192; later launches go untimed).  Resets the
 * accumulators.  Returns EINVAL for an unknown class, EHIP if event creation fails. */
stokes_status stokes_profile_kernel(stokes_ctx *ctx, int kernel);

/* Read and reset the accumulators: summed event time (ms), launches timed and
 * their summed algorithmic bytes. */
stokes_status stokes_profile_read(stokes_ctx *ctx, double *ms_total, long long *launches, double *bytes);

/* Streaming reference for the measurements: dst[i] = src[i] for i < n, device
 * pointers that do not overlap, asynchronously on `stream` (a hipStream_t; NULL
 * = default stream), one read and one write of every element with the
 * library's own copy kernel (16-byte accesses when both pointers are 16-byte
 * aligned).  Timing it gives the practical HBM bandwidth next to the nominal
 * 8 TB/s.  Returns EINVAL for n < 0 or a null pointer with n > 0, EHIP if the
 * launch fails. */
stokes_status stokes_stream_copy(const double *src, double *dst, long long n, void *stream);

/* ---------------------------------------------------------------------------
 * Coefficient step (Sec. 4.1, eqs. eq_heaviside, eq_ls_flow, eq_ls_solid;
 * Sec. 4.2.2 for the face density): the rho_face and mu_cell that
 * stokes_setup takes, computed on the device from signed-distance level sets.
 *
 *   H(x) = 0 for x < -eps, 1 for x > eps, (1 + x/eps + sin(pi x/eps)/pi)/2
 *          between, with eps = n_cells * hx (the grid is taken as isotropic);
 *   flowing phase  z = z_liquid + (z_gas - z_liquid) H(phi)   (liquid: phi < 0);
 *   each solid q   z = z_s[q] + (z - z_s[q]) H(psi_q)        (solid: psi_q < 0),
 *                  applied in the order given.
 *
 * mu_cell uses the cell level sets.  A face uses the level sets averaged onto
 * it: the mean of its two cells, or the one cell of a boundary face (every
 * face of the output arrays is written, wall faces included).
 * rho_flow_face, if not NULL, receives the flowing-phase density alone (no
 * solid) on the same faces, as the well-balanced gravity force needs (Sec. 5).
 * --------------------------------------------------------------------------- */
#define STOKES_MAX_SOLIDS 8

typedef struct {
    double rho_liquid, rho_gas;   /* > 0 */
    double mu_liquid, mu_gas;     /* >= 0 */
    double n_cells;               /* Heaviside half-width in cells of hx, > 0 */
} stokes_fluids;

/* phi          device, cell layout (Nz, Ny, Nx): liquid/gas level set
 * n_solids     0..STOKES_MAX_SOLIDS
 * psi          HOST array of n_solids DEVICE pointers, each a cell-layout level set
 * rho_solid, mu_solid   HOST arrays of n_solids values (> 0, >= 0)
 * rho_face[3]  device outputs in the face layouts (rho_face[2] ignored in 2D)
 * mu_cell      device output, cell layout
 * rho_flow_face  NULL, or device outputs like rho_face
 * stream       hipStream_t (as void*); asynchronous, no workspace, no allocation.
 * Grids need >= 1 cell per axis and fewer than 2^31 points (Nx+1)(Ny+1)(Nz+1)
 * (ESHAPE otherwise).  EINVAL for a NULL required pointer, a non-positive or
 * non-finite density, spacing or n_cells, a negative viscosity or n_solids out
 * of range; EHIP if the launch fails.  Outputs must not overlap the inputs. */
stokes_status stokes_coefficients(const stokes_grid *grid, const stokes_fluids *fluids,
                                  const double *phi, int n_solids, const double *const *psi,
                                  const double *rho_solid, const double *mu_solid,
                                  double *const rho_face[3], double *mu_cell,
                                  double *const rho_flow_face[3], void *stream);

/* ---------------------------------------------------------------------------
 * Face-density transport of the conservative scheme (Sec. 4.2.2, eqs. eq_rk1,
 * eq_rk2 and eq_rk3): the face densities that stokes_setup takes, advanced
 * from rho_n by three-stage SSP-RK3,
 *     rho1 = rho_n - dt R(u1, rho_n)
 *     rho2 = 3/4 rho_n + 1/4 rho1 - 1/4 dt R(u2, rho1)
 *     rho  = 1/3 rho_n + 2/3 rho2 - 2/3 dt R(u3, rho2),
 * with R(u, rho) the divergence of u_adv rho_lim over each face's control
 * volume (one cell long in every direction, centred on the face): u_adv on a
 * control-volume face is the mean of the two nearest velocities normal to it,
 * rho_lim the cubic upwind value limited by CUI (Waterson and Deconinck 2007),
 * densities beyond a wall mirror the interior, and nothing crosses a wall
 * (wall-normal velocities are zero).  Wall-normal faces are not transported:
 * they hold rho_n.  The stage velocities are the caller's (the paper takes u^n,
 * then extrapolations of u^n, u^{n-1} and the latest iterate).
 *   rho_n[3]     device face densities in the solver's layouts (rho_n[2] NULL in 2D)
 *   u_stage[9]   device face velocities of the three stages: stage s, component c
 *                at u_stage[3 s + c] (the c = 2 entries NULL in 2D); wall-normal
 *                entries must be 0
 *   rho_out[3]   device outputs in the same layouts; must not overlap the inputs
 *   workspace    device buffer of ws_bytes >= stokes_density_workspace_size(grid)
 *                (the second stage's densities)
 * Asynchronous on stream (three launches).  EINVAL for a NULL pointer, dt <= 0 or
 * a bad spacing; ESHAPE for fewer than 2 cells along an axis or a face array of
 * 2^31 entries or more; ENOMEM for a small workspace; EHIP if a launch fails.
 * --------------------------------------------------------------------------- */
size_t stokes_density_workspace_size(const stokes_grid *grid);   /* 0 for a grid the update rejects */

stokes_status stokes_density_rk3(const stokes_grid *grid, double dt, const double *const rho_n[3],
                                 const double *const u_stage[9], double *const rho_out[3],
                                 void *workspace, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Wave-tank boundaries (Sec. 7.1, "Stokes wave theory and numerics"): the
 * inflow on the x = 0 side and, with stokes_options.open_top, the open top.
 * The vertical axis is y in 2D and z in 3D; the tank bottom is at 0, the still
 * level at the depth d, and the wave travels along +x.
 *
 * stokes_wave_inflow evaluates the second-order Stokes wave (eqs.
 * eq_stokes_eta, eq_stokes_u, eq_stokes_v; height H, wavelength lambda,
 * k = 2 pi / lambda, angular frequency omega, gravity g) on x = 0 at time t,
 * restricted to the liquid by 1 - H~(phi), phi = -eta(0, t) + (height above the
 * still level), with H~ the smoothed Heaviside of eq. eq_heaviside_normal_bdry
 * of half-width n_cells sqrt(h_x h_vertical):
 *   u_n  device (Nz, Ny) (2D: Ny): the normal velocity of the x-faces at x = 0
 *        (at the faces' heights, cell centres);
 *   u_t  device (Nz+1, Ny) (2D: Ny+1): the vertical velocity on the wall at the
 *        vertical faces' heights (nodes).
 * The lateral velocity of the wave (3D) is 0.  Asynchronous on stream.  EINVAL
 * for a NULL pointer or a parameter that is not positive and finite (H may be
 * 0); ESHAPE for fewer than 2 cells along an axis.
 *
 * stokes_inflow_lift moves Dirichlet inflow data on x = 0 (u_n, u_t in the
 * layouts above) to the right-hand side: in place, rhs_u and rhs_p (device,
 * the caller's layouts) lose the contribution of the boundary values to the
 * rows next to the wall -- the continuity of the cells (0, j, k) (-u_n / h_x),
 * the normal viscous stress of the x-faces i = 1, and the wall-edge shear
 * stress of the tangential faces i = 0 (with the tangential ghost 2 u_t minus
 * the interior, and the variation of u_n along the wall) -- with the context's
 * viscosities and theta.  Solve with the lifted right-hand side, then put u_n
 * into the solution's x-faces at x = 0 (the solver writes wall faces as 0).
 * Asynchronous on the context's stream.  EINVAL for a NULL pointer, EHIP if the
 * launch fails.
 * --------------------------------------------------------------------------- */
typedef struct {
    double height;       /* H, peak to peak (>= 0) */
    double depth;        /* d: still level above the bottom (> 0) */
    double wavelength;   /* lambda (> 0) */
    double omega;        /* angular frequency (> 0), e.g. from omega^2 = g k tanh(k d) */
    double gravity;      /* g (> 0) */
    double n_cells;      /* half-width of the boundary Heaviside in cells (> 0) */
} stokes_wave;

stokes_status stokes_wave_inflow(const stokes_grid *grid, const stokes_wave *wave, double t,
                                 double *u_n, double *u_t, void *stream);

stokes_status stokes_inflow_lift(stokes_ctx *ctx, const double *u_n, const double *u_t,
                                 double *const rhs_u[3], double *rhs_p);

/* ---------------------------------------------------------------------------
 * Explicit momentum right-hand side of one time step (Sec. 4.2.2,
 * eq_nc_discrete_momentum, and eq_c_discrete_momentum with the old density;
 * Sec. 5 for the gravity force):
 *
 *     f = (rho/dt) u^n + (1 - theta) L_mu u^n + rho_force g   on interior faces,
 *
 * L_mu the strain-rate operator of the solve (same edge viscosities and wall
 * rules), theta the implicit fraction of the following stokes_solve (1/2: the
 * paper's Crank-Nicolson split, which the solver takes as visc_scale).  With
 * rho = the level-set density this is the non-conservative scheme's
 * right-hand side, with the old density the conservative one's; rho_force = the
 * flow-only density gives the well-balanced gravity force.  The convective term
 * is the caller's (add it to f).
 *   rho_face[3], mu_cell, u_n[3]  device inputs in the solver's layouts
 *                                 (wall-normal entries of u_n are read as 0)
 *   rho_force[3], gravity[3]      NULL for no gravity term; gravity is a host array
 *   f[3]                          device output (wall-normal entries written as 0)
 * Asynchronous on stream; no workspace.  EINVAL for NULL pointers, dt <= 0,
 * theta outside [0, 1] or a non-finite gravity; ESHAPE for fewer than 2 cells
 * along an axis or 2^31 - 256 points (Nx+1)(Ny+1)(Nz+1) or more; EHIP if the
 * launch fails.  f must not overlap the inputs.
 * --------------------------------------------------------------------------- */
stokes_status stokes_explicit_rhs(const stokes_grid *grid, const double *const rho_face[3],
                                  const double *mu_cell, double dt, double theta,
                                  const double *const u_n[3], const double *const rho_force[3],
                                  const double gravity[3], double *const f[3], void *stream);

/* ---------------------------------------------------------------------------
 * Rigid-body constraint projection after the solve (Sec. 4.2.5, eqs.
 * eq_velocity_correction, eq_prescribed_velocity, eq_linear_conservation and
 * eq_angular_conservation; interpolation and spreading of Sec. 3.3):
 *
 *     u <- u + S (U_b - J u),   U_b = U_r + W_r x (X - x_com)  at each marker X,
 *
 * J interpolates the face velocities onto the body's Lagrangian markers with
 * the four-point regularised delta function of Peskin (2002), delta_h(x) =
 * prod_d phi(x_d / h_d) / h_d, times the cell volume; S spreads marker values
 * back with the same kernel times the marker volume dV.  Near a no-slip wall
 * stencil points beyond the wall take the odd mirror image of the interior and
 * wall-normal points on the wall hold zero, with S the exact adjoint of J.
 * free_body = 0: (U_r, W_r) are the caller's (prescribed motion).  free_body = 1:
 * they are computed from the momentum of J u over the markers,
 *     M U_r = sum (J u) dV,  I W_r = sum R x (J u) dV,  R = X - x_com,
 *     M = n dV,  I = sum (|R|^2 Id - R (x) R) dV,
 * and returned in *body.  In 2D, W_r is the rotation rate about z (w_r[0]) and
 * I = sum |R|^2 dV.
 * --------------------------------------------------------------------------- */
typedef struct {
    double x_com[3];   /* centre of mass (rotation centre) */
    double u_r[3];     /* linear velocity: input (prescribed) or output (free body) */
    double w_r[3];     /* angular velocity: input or output; 2D uses w_r[0] only */
} stokes_body;

/* Workspace bytes for n_markers markers in dim dimensions; 0 if invalid.  Host-only. */
size_t stokes_rigid_workspace_size(int dim, long long n_markers);

/* u[3]       device face velocities in the solver's layouts (u[2] ignored in 2D),
 *            corrected in place; plain device memory (hipMalloc), as the
 *            correction is added with device atomics
 * X          device marker positions, n_markers x dim, each inside [0, n h]
 * dV         marker volume (> 0)
 * workspace  device buffer of ws_bytes >= stokes_rigid_workspace_size(dim, n_markers)
 * Blocks until the momentum sums are on the host (it synchronises the stream
 * once); the correction itself is queued after them.  EINVAL for NULL pointers,
 * bad dV or body values, a marker outside the domain (then u is untouched), a
 * free body without markers or whose markers are collinear (singular inertia);
 * ESHAPE for fewer than 2 cells along an axis; ENOMEM for a small workspace;
 * EHIP if a HIP call fails.  Several bodies: one call per body. */
stokes_status stokes_rigid_projection(const stokes_grid *grid, double *const u[3], long long n_markers,
                                      const double *X, double dV, int free_body, stokes_body *body,
                                      void *workspace, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * projection as stokes_rigid_projection, same arguments and results, without a
 * workspace.  Its scratch (the interpolated marker velocities and the block
 * partials of the momentum sums) is a fixed array inside the library, one per
 * GPU, held until the process ends: 8 * (3 * STOKES_RIGID_NOALLOC_MAX_MARKERS +
 * 13 * 1024) bytes, about 12.7 MB.  The call allocates nothing (no hipMalloc,
 * hipFree or host heap); it reads the array's device address once per GPU with
 * hipGetSymbolAddress, on the current device, which must be the device of u, X
 * and stream.  Every entry of the scratch is written before it is read, so
 * nothing carries over between calls; but calls that overlap on one GPU (other
 * host threads, other streams) share the array and race: serialise them.
 * ENOMEM (with stokes_last_error(NULL) naming the limit) for more than
 * STOKES_RIGID_NOALLOC_MAX_MARKERS markers, before any GPU work; the other
 * errors as for stokes_rigid_projection, EHIP also if the symbol address cannot
 * be read. */
#define STOKES_RIGID_NOALLOC_MAX_MARKERS 524288
stokes_status stokes_rigid_projection_noalloc(const stokes_grid *grid, double *const u[3], long long n_markers,
                                              const double *X, double dV, int free_body, stokes_body *body,
                                              void *stream);

/* ---------------------------------------------------------------------------
 * Learned form: a 4-level 3D U-Net (channels 16/32/48/64, 3x3x3 convolutions,
 * ReLU, 2x2x2 average pooling, nearest upsampling, additive skips) in BF16 with
 * FP32 accumulation on the matrix cores (v_mfma_f32_16x16x16_bf16), with its
 * backward pass and an Adam optimiser.  It maps three planar FP32 features
 * (normalised log rho, log mu, and the pressure right-hand side scaled to unit
 * RMS) on an n^3 grid to a predicted pressure shape.  Its weights are the
 * caller's (stokes_unet_set_params); all memory is the caller's workspace.
 * --------------------------------------------------------------------------- */
typedef struct stokes_unet stokes_unet;

/* Number of FP32 parameters (all weights as [c_out][27][c_in] layer by layer, then all biases). */
long long stokes_unet_param_count(void);

/* Floating-point operations of the convolutions of one forward pass at n^3
 * (two per multiply-add, input channels padded to 16 as computed); 0 for an
 * invalid n.  Host-only. */
double stokes_unet_forward_flops(int n);

/* Workspace bytes for an n^3 network (n >= 8, n % 8 == 0), 0 otherwise.  Host-only. */
size_t stokes_unet_workspace_size(int n);

/* Create a network on the caller's device workspace and HIP stream (void*). */
stokes_status stokes_unet_create(int n, void *workspace, size_t ws_bytes, void *stream, stokes_unet **out);

/* He-uniform weights from a counter-based generator, zero biases and Adam state. */
stokes_status stokes_unet_init(stokes_unet *net, unsigned long long seed);

/* Copy the FP32 parameters from / to host memory (count = stokes_unet_param_count()). */
stokes_status stokes_unet_get_params(stokes_unet *net, float *host, long long count);
stokes_status stokes_unet_set_params(stokes_unet *net, const float *host, long long count);

/* Forward pass: out = prediction for the planar device features f0, f1, f2 (n^3 FP32 each). */
stokes_status stokes_unet_forward(stokes_unet *net, const float *f0, const float *f1, const float *f2, float *out);

/* One Adam step (lr, beta 0.9/0.999) on the mean-square error between the
 * prediction and `target` (device, n^3 FP32); *loss (host) receives the loss
 * before the step.  Blocks until done. */
stokes_status stokes_unet_train_step(stokes_unet *net, const float *f0, const float *f1, const float *f2,
                                     const float *target, float lr, float *loss);

/* Gradient of the last training step's loss (host, count = stokes_unet_param_count()). */
stokes_status stokes_unet_get_grads(stokes_unet *net, float *host, long long count);

/* Grid size n of a network; 0 for NULL. */
int stokes_unet_size(const stokes_unet *net);

/* Release the host-side network object (the workspace stays the caller's). */
void stokes_unet_destroy(stokes_unet *net);

/* Use `net` as the learned stage of this context's preconditioner (NULL
 * detaches).  The network runs on the multigrid level with net's n^3 cells
 * (3D, n <= 64; EINVAL if there is none) and must share the context's stream.
 * Before the pressure cycles of each preconditioner application the pressure
 * right-hand side is restricted to that level, scaled to unit RMS and fed to
 * the network with the level's static features; the prediction's amplitude is
 * fitted by least squares against that level's Poisson operator and the
 * result, prolonged trilinearly to the finest level, is the initial guess of
 * the pressure cycles.  Fallback on stagnation: as soon as an FGMRES iteration
 * reduces the residual estimate by less than the factor stall_ratio (0.9 in
 * production), the rest of the solve runs plain multigrid and
 * stokes_stats.fell_back is set.  The FP64 residual check is unchanged. */
stokes_status stokes_attach_learned(stokes_ctx *ctx, stokes_unet *net, double stall_ratio);

/* Training tuple on the level with n^3 cells (device FP32 planar outputs,
 * x fastest): static features f0 = log10(rho)/3 - 1/2 (rho from the level's
 * face coefficients) and f1 = log10(mu)/2 + 2, the pressure right-hand side of
 * the first preconditioner application for the right-hand side (rhs_u, rhs_p)
 * restricted to that level and scaled to unit RMS (s_c), and the pressure
 * solution of that right-hand side after `cycles` pressure cycles, restricted
 * and scaled to zero mean and unit RMS (phi_c).  Blocks until done. */
stokes_status stokes_learned_tuple(stokes_ctx *ctx, const double *const rhs_u[3], const double *rhs_p, int n,
                                   int cycles, float *f0, float *f1, float *s_c, float *phi_c);

/* Measurement hook for the learned stage: what an initial guess is worth to
 * the pressure cycles of the first preconditioner application on the packed
 * right-hand side (rhs_u, rhs_p as in stokes_solve; 3D only).  The reference
 * solution phi* of that pressure subsolve is `ref_cycles` (>= 1) cycles from
 * zero.  res (host, STOKES_STUDY_ROWS x (max_cycles + 1), row-major; 0 <=
 * max_cycles <= 64) receives the relative residual ||s - (-L_rho) phi_k|| /
 * ||s|| after k = 0 .. max_cycles cycles started from:
 *   row 0      zero (the plain solve);
 *   row 1      the attached network's guess (NaN without a network);
 *   row 1 + l  (l = 1 .. STOKES_STUDY_ROWS - 2) the ideal guess of a perfect
 *              predictor on multigrid level l (2^l times coarser): phi*
 *              averaged to that level, then the amplitude fit and trilinear
 *              prolongation the network's output takes (NaN if the hierarchy
 *              has no level l).
 * The solve is not changed; the Krylov scratch it uses is cleared again by the
 * next solve.  Blocks until done. */
#define STOKES_STUDY_ROWS 6
stokes_status stokes_learned_study(stokes_ctx *ctx, const double *const rhs_u[3], const double *rhs_p, int ref_cycles,
                                   int max_cycles, double *res);

/* ---------------------------------------------------------------------------
 * Test hook: one kernel of the pressure multigrid on the finest level, run on
 * caller data exactly as the cycle launches it.  The operator is the pressure
 * Poisson operator of the projection step, -L_rho = -D beta G with beta =
 * 1/rho on interior faces and Neumann walls (Sec. 4.2.4 names the projection
 * preconditioner; the multigrid is this library's subsolve for it).
 *   STOKES_POP_SWEEP          one red-black Gauss-Seidel sweep of -L_rho e = r
 *                             (cells with i+j+k even first, then odd; relaxed
 *                             by the context's p_omega as in the cycle), in the
 *                             form the cycle uses on this level: the fused
 *                             z-marching kernel on 3D levels of more than 2^18
 *                             cells, two colour passes otherwise;
 *   STOKES_POP_SWEEP_FLAT     the same sweep as two one-thread-per-point passes;
 *   STOKES_POP_RESTRICT       out (cells of the next-coarser level) = the mean
 *                             over the 2^d children of r - (-L_rho) e, in the
 *                             cycle's form (z-marching on 3D levels of at least
 *                             2^21 cells);
 *   STOKES_POP_RESTRICT_FLAT  the same with the one-thread-per-coarse-cell kernel.
 * e_in, r   device cell arrays (Nz, Ny, Nx) of the grid; e_in NULL starts a
 *           sweep from zero
 * ec        NULL, or (sweeps with e_in only) a device cell array of the
 *           next-coarser level whose prolongation (piecewise constant, or
 *           trilinear with p_prolong = 1) is added to e_in before the sweep, as
 *           the cycle does after its coarse-grid correction
 * out       device cell array of the fine level (sweeps) or the next-coarser
 *           level (restriction)
 * With FP32 multigrid the inputs are rounded to float on the way in and the
 * result widened on the way out.  Uses the context's level buffers (not
 * concurrently with a solve on the same context); blocks until done.  EINVAL for
 * an unknown op, a missing pointer, ec without e_in, or a coarse operand on a
 * grid that has no coarser level; EHIP if a HIP call fails.
 * --------------------------------------------------------------------------- */
enum {
    STOKES_POP_SWEEP = 0,
    STOKES_POP_SWEEP_FLAT = 1,
    STOKES_POP_RESTRICT = 2,
    STOKES_POP_RESTRICT_FLAT = 3
};
stokes_status stokes_pressure_op(stokes_ctx *ctx, int op, const double *e_in, const double *r, const double *ec,
                                 double *out);

/* Release the host-side context (the workspace stays the caller's). NULL is a no-op. */
void stokes_destroy(stokes_ctx *ctx);

/* Message describing the last failure on this context ("" if none).  With
 * ctx == NULL, the message of the last failed stokes_setup (or
 * stokes_rigid_projection_noalloc) in this thread. */
const char *stokes_last_error(const stokes_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif
