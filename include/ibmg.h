/*
 * ibmg.h -- C interface of the MI355X (gfx950) immersed-boundary biofilm
 * library: multigrid projection step on a staggered MAC grid, delta-function
 * spread and interpolation with the delta width set to the bacterial radius,
 * Hookean springs with breakage.
 *
 * The method is that of Hammond, Stewart, Younger, Solomon and Bortz,
 * "Spatially heterogeneous biofilm simulations using an immersed boundary
 * method with Lagrangian nodes defined by bacterial locations".  Each entry
 * point below names the passage that defines what it computes.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  Every array argument is a DEVICE pointer unless stated otherwise.
 *   The caller owns all memory, including the workspace handed to
 *   ibb_create; the library never allocates device memory.  The workspace
 *   must stay valid until ibb_destroy.  Input arrays are read in stream order
 *   during the call and are not retained.
 * Streams.  All work is enqueued on the stream given to ibb_create
 *   (a hipStream_t passed as void*; NULL is the default stream).  Calls that
 *   return statistics or convergence results synchronise that stream.  A
 *   context is not thread-safe.
 * Errors.  Every call returns an ibb_status; nothing is thrown across the
 *   interface.  Arguments are validated before any work is enqueued.
 *   IBB_ENOCONV is not fatal: the iterate is kept and statistics are filled.
 *   ibb_last_error() gives a message for the last failure on a context;
 *   with a null context, that of the last failed ibb_create on the thread.
 * Units.  Nondimensional, as in the paper's scaling (sigma = Strouhal number,
 *   eps = Euler number, Re = Reynolds number).
 *
 * Grid and layouts
 * ----------------
 * The domain is n[0] x n[1] (x n[2]) cells of width h.  Pressure and the cell
 * viscosity live at cell centres; velocity component a, density and the
 * force component a live on the faces normal to axis a; the cross viscosity
 * lives on cell edges (in 2D on cell corners).  Each axis is PERIODIC,
 * WALLS (no-slip walls on both sides) or INOUT (prescribed inflow on the low
 * side, zero normal derivative on the high side, where the pressure is 0).
 *
 * Arrays are exchanged in the "compact" layout: one lattice lists its
 * closed-domain positions with x fastest, then y, then z.  Along an axis a
 * lattice is cell-centred (n positions) or vertex-centred (n + 1 positions,
 * n on a periodic axis).  Velocity, force and density arrays concatenate the
 * D face lattices (faces normal to x, then y, then z).  Edge arrays
 * concatenate the edge lattices parallel to x, y, z (2D: the corner lattice).
 * ibb_lattice_count gives each size.  Node arrays are structure-of-arrays
 * [dim][n] in FP64.  Spring endpoints are int32 [2][m].
 */
#ifndef IBMG_H
#define IBMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    IBB_OK = 0,
    IBB_EINVAL = 1,   /* bad descriptor, shape, size or pointer */
    IBB_ENOMEM = 2,   /* workspace smaller than ibb_footprint_bytes */
    IBB_ENOCONV = 3,  /* a solve hit max_cycles before reaching rtol */
    IBB_ENUMERIC = 4, /* NaN or Inf in a residual norm */
    IBB_EDEVICE = 5,  /* a HIP runtime call failed */
    IBB_ESTATE = 6    /* call out of order (e.g. a step before coefficients) */
} ibb_status;

typedef enum { IBB_AXIS_PERIODIC = 0, IBB_AXIS_WALLS = 1, IBB_AXIS_INOUT = 2 } ibb_axis_bc;

/* regularised delta: cosine phi_2 (eq:PhiCosAlternative, the paper's choice)
 * or Peskin's four-point phi_1 (eq:PhiPeskin) */
typedef enum { IBB_PHI_COS = 0, IBB_PHI_PESKIN4 = 1 } ibb_kernel;

/* IBB_FP64: V-cycles in FP64.  IBB_FP32_REFINED: V-cycles in FP32 inside an
 * FP64 defect-correction loop (FP64 residual of the full operator, FP64
 * update, FP64 coarsest-level inverse). */
typedef enum { IBB_FP64 = 0, IBB_FP32_REFINED = 1 } ibb_precision;

typedef struct {
    int dim;            /* 2 or 3 */
    int n[3];           /* cells per axis, each even; n[2] ignored in 2D; the product of
                           (n + 3) over the axes below 2^31 */
    int axis_bc[3];     /* ibb_axis_bc per axis */
    double h;           /* mesh width (isotropic) */
    double sigma;       /* Strouhal number */
    double eps;         /* Euler number */
    double inv_re;      /* 1 / Reynolds number */
    double force_coef;  /* L f0 / (rho0 u0^2), eq:N-SnondimFull */
    double dt;          /* time step */
    double body_force[3]; /* constant body force added to the momentum equation */
    double rho0;        /* fluid density, eq:discrDensCouple */
    double rho_b;       /* extra biofilm density */
    double d0_pow_d;    /* average node volume (area in 2D) */
    double mu_out;      /* fluid viscosity, eq:ViscExp */
    double mu_max;      /* viscosity at a node */
    double omega;       /* spread width (bacterial radius) */
    int kernel;         /* ibb_kernel */
    double break_ratio; /* springs break beyond break_ratio x rest length */
    int nu1, nu2;       /* pre- and post-smoothing sweeps per V-cycle */
    int max_levels;     /* 0: coarsen while every axis stays even and >= 2 */
    int max_cycles;     /* cap on V-cycles (FP64) or outer iterations (refined) */
    double rtol;        /* relative residual target ||b - A x|| / ||b|| */
    double gamma[16];   /* coarse viscosity scaling per level, eq:ViscCoarseGrid (<= 0 means 1) */
    int precision;      /* ibb_precision */
    int inner_cycles;   /* FP32 V-cycles per outer FP64 iteration (refined) */
    int wg_coarse_max;  /* levels whose largest colour class has at most this many points
                           run the rest of the V-cycle in one workgroup; 0: 512 (one point
                           per thread of the workgroup), < 0: never */
    /* detached fragments (see ibb_fragments): a node is anchored when, at the
     * positions given to ibb_set_nodes, its coordinate along attach_axis is
     * below attach_dist (the attachment wall is that axis's low wall) */
    int track_fragments;   /* nonzero: ibb_lagrangian_update counts fragments */
    int attach_axis;
    double attach_dist;
    /* 0: plain V-cycles (the paper's method).  m in 1..64: GCR(m) with one
     * V-cycle (refined: inner_cycles FP32 V-cycles) from zero as the right
     * preconditioner, modified Gram-Schmidt against the stored directions,
     * restarted after m directions; the FP64 residual b - A x and the
     * stopping test are those of the plain solver, and max_cycles caps the
     * iterations.  In a group, such a member's solves run on their own
     * rather than in the shared launches. */
    int krylov_restart;
    /* launches per red-black sweep of a component on levels swept with
     * launched passes: 0 or 2, one per colour; 1, one launch for both
     * colours (LDS tiles with a redundant red ring, a second iterate
     * buffer; needs nu1 + nu2 even, otherwise two); 3, one launch for both
     * colours of a velocity component on 3D levels, each workgroup marching
     * along z through a run of planes with a window of the component in
     * LDS (a second iterate buffer; needs nu1 + nu2 even and periodic axes
     * long enough for the window, otherwise two; the pressure keeps two).
     * All give the same bits. */
    int smoother_passes;
    /* 0: the coupled viscous system of eq:NSdis1-1.  1: constant viscosity,
     * eq:NSdis1: (sigma rho / dt) u_a - Re^-1 mu L_h u_a for each component
     * on its own (mu = mu_out, times the product of gamma down to a coarse
     * level); needs mu_max == mu_out, otherwise IBB_EINVAL.  The components'
     * smoothing passes of one colour share a launch. */
    int decoupled;
    /* 0: the levels below the start of the one-workgroup cycle (see
     * wg_coarse_max) are applied as their linear map, a matrix rebuilt with
     * every coefficient update by running those levels' passes on each unit
     * right-hand side (when the level below the start has at most 512
     * unknowns and all levels from there fit one workgroup's LDS); it gives
     * the same result as the recursion up to rounding.  < 0: always recurse. */
    int coarse_tail;
    /* 1: colour passes of launched 3D levels walk z in blocks of planes (one
     * workgroup per band of rows and run of 16 planes) instead of one point
     * per thread across the whole level; same bits, slower on the grids
     * measured here.  0 (default) or < 0: one point per thread. */
    int smoother_zblock;
    /* 1: the viscous system's coarse operators satisfy the Galerkin
     * condition, A_{l+1} = R_l A_l P_l with the V-cycle's own restriction and
     * prolongation (Sec. "Numerical Concerns", second remedy for slow
     * convergence at large mu_max), rebuilt with the coefficients; such a
     * level is smoothed red-black with every (component, colour) set updated
     * from its values before the pass, since R A P couples points of one
     * colour.  The velocity V-cycles then run launched passes to the
     * coarsest level (no one-workgroup cycle or tail); the pressure system
     * is unchanged.  Not with decoupled = 1, nor in an ibb_group.  0: the
     * coarse operators are rediscretised on restricted coefficients. */
    int galerkin;
} ibb_desc;

typedef struct {
    int status_u, status_p;    /* ibb_status of each solve */
    int cycles_u, cycles_p;    /* V-cycles (FP64) or outer iterations (refined) */
    int vcycles_u, vcycles_p;  /* V-cycles actually run (refined: outer x inner) */
    double relres_u, relres_p; /* final FP64 relative residuals */
    double t_u_ms, t_p_ms;     /* device time of each solve, RHS ready to converged */
    long long dof_u, dof_p;    /* unknowns of each system */
} ibb_solve_stats;

typedef struct {
    int n_broken;  /* springs broken in this update */
    int n_alive;   /* springs alive afterwards */
    double t_ms;   /* device time of the update */
    int n_fragments;  /* fragments after the update (-1: not tracked) */
    int n_detached;   /* of them, fragments without an anchored node (-1: not tracked) */
} ibb_lag_stats;

typedef struct ibb_ctx ibb_ctx;

/* --- sizes ------------------------------------------------------------ */

/* Number of closed-domain positions of a lattice in the compact layout.
 * kind: 0 cell centres, 1 faces normal to `axis`, 2 edges parallel to `axis`
 * (2D: axis 2 is the corner lattice).  dims (host, may be NULL) receives the
 * extent along x, y, z. */
ibb_status ibb_lattice_count(const ibb_desc *desc, int kind, int axis, int64_t *count, int dims[3]);

/* Workspace bytes needed for a context with up to max_nodes nodes and
 * max_springs springs. */
ibb_status ibb_footprint_bytes(const ibb_desc *desc, int64_t max_nodes, int64_t max_springs, size_t *bytes);

/* --- lifetime ------------------------------------------------------------ */

/* Validate desc, carve the workspace and set every field to zero.  The
 * multigrid hierarchy has one level per halving of the grid (Sec.
 * "Multigrid"). */
ibb_status ibb_create(const ibb_desc *desc, int64_t max_nodes, int64_t max_springs, void *workspace,
                      size_t workspace_bytes, void *stream, ibb_ctx **out);
ibb_status ibb_destroy(ibb_ctx *ctx);

/* --- state ------------------------------------------------------------- */

/* Velocity (compact, all face lattices, boundary faces included: the values
 * on fixed faces are the boundary data, e.g. the inflow profile) and
 * pressure (compact cells).  p may be NULL to leave the pressure as is. */
ibb_status ibb_set_state(ibb_ctx *ctx, const double *u, const double *p);
ibb_status ibb_get_state(ibb_ctx *ctx, double *u, double *p);

/* Reload a context with another problem of the same shape (a serving slot):
 * desc (host) replaces the descriptor the context was created with, and
 * must agree with it in every field except rho_b, d0_pow_d, mu_max (the
 * biofilm's density and viscosity, eq:discrDensCouple, eq:ViscExp),
 * break_ratio, track_fragments, attach_axis, attach_dist, rtol and
 * max_cycles (IBB_EINVAL otherwise, the context unchanged).  None of these
 * is an argument of a captured solver iteration, so the context's graphs
 * (and those of a group it belongs to) stay valid; nothing is allocated.
 * The coefficients must then be rebuilt (ibb_update_coefficients, after
 * ibb_set_nodes, which reads the attachment fields): ibb_projection_step
 * returns IBB_ESTATE until then.  Host only: no device work. */
ibb_status ibb_set_params(ibb_ctx *ctx, const ibb_desc *desc);

/* Node positions X [dim][n], n <= max_nodes. */
ibb_status ibb_set_nodes(ibb_ctx *ctx, int64_t n, const double *X);

/* Node positions, total spring force [dim][n] and spring alive flags [m]
 * (each may be NULL). */
ibb_status ibb_get_nodes(ibb_ctx *ctx, double *X, double *F, uint8_t *alive);

/* Spring network (eq:springF): endpoints ij [2][m] (int32, distinct node
 * indices), rest lengths r [m], stiffnesses K [m], alive flags [m] (NULL:
 * all alive).  Builds the per-node incidence lists used by the force pass. */
ibb_status ibb_set_springs(ibb_ctx *ctx, int64_t m, const int32_t *ij, const double *rest, const double *K,
                           const uint8_t *alive);

/* --- the step ------------------------------------------------------------ */

/* At the current node positions: spring forces (no breakage), the spread
 * force f and density rho on the faces (eq:discrForceCouple,
 * eq:discrDensCouple), the viscosity at cells and edges (eq:ViscExp), and
 * every coarse level's coefficients (full-weighting restriction, viscosity
 * scaled by gamma, eq:ViscCoarseGrid).  Call once after setting nodes and
 * springs; ibb_lagrangian_update repeats it after moving the nodes. */
ibb_status ibb_update_coefficients(ibb_ctx *ctx);

/* One projection step (eq:NSdis1-1, eq:NSdis4, eq:NSdis2): the momentum
 * right-hand side, the viscous multigrid solve for u~ (warm start u^n), the
 * pressure right-hand side, the pressure multigrid solve (warm start p^n),
 * and the projection to u^{n+1}.  stats (host, may be NULL) is filled. */
ibb_status ibb_projection_step(ibb_ctx *ctx, ibb_solve_stats *stats);

/* Lagrangian update: interpolate u^{n+1} to the nodes with width h
 * (eq:discrVelCouple), move them by dt / sigma times that velocity
 * (periodic axes wrap), break springs stretched beyond break_ratio times
 * their rest length, recompute forces, and rebuild the Eulerian
 * coefficients as in ibb_update_coefficients.  stats (host) may be NULL. */
ibb_status ibb_lagrangian_update(ibb_ctx *ctx, ibb_lag_stats *stats);

/* --- individual steps (for checking each against a reference) ----------- */

/* Level-l coefficient fields in compact layout (each may be NULL): force f
 * (level 0 only), density rho, cell viscosity mu_c, edge viscosity mu_e. */
ibb_status ibb_get_fields(ibb_ctx *ctx, int level, double *f, double *rho, double *mu_c, double *mu_e);

/* Momentum right-hand side of eq:NSdis1-1 at the current state, with the
 * fixed boundary values moved to the right (compact faces; only unknown
 * positions are written). */
ibb_status ibb_momentum_rhs(ibb_ctx *ctx, double *b);

/* Pressure right-hand side -(sigma / (eps dt)) D u~ of eq:NSdis4 (mean
 * removed when no outflow face exists) from a compact face field ut. */
ibb_status ibb_pressure_rhs(ibb_ctx *ctx, const double *ut, double *bp);

/* Multigrid solve of the viscous (which = 1) or pressure (which = 0) system
 * A x = b on the current coefficients (Sec. "Multigrid"), V-cycles until
 * ||b - A x|| <= rtol ||b||.  b and x are compact (faces or cells); x holds
 * the initial guess and receives the result at unknown positions.
 * cycles, relres (host) may be NULL.  max_cycles_override > 0 replaces
 * desc.max_cycles for this call; ncycles_exact > 0 runs exactly that many
 * cycles without a stopping test. */
ibb_status ibb_mg_solve(ibb_ctx *ctx, int which, const double *b, double *x, int max_cycles_override,
                        int ncycles_exact, int *cycles, double *relres);

/* Projection of eq:NSdis2 from u~ (compact faces) and p (compact cells). */
ibb_status ibb_project(ibb_ctx *ctx, const double *ut, const double *p, double *u);

/* Interpolation of a compact face field u to nodes X [dim][n] with delta
 * width `width` (eq:discrVelCouple uses width h); U [dim][n]. */
ibb_status ibb_interp(ibb_ctx *ctx, double width, int64_t n, const double *X, const double *u, double *U);

/* Spread of node vectors F [dim][n] at X to the face lattices with width
 * `width` (eq:discrForceCouple); out is compact faces. */
ibb_status ibb_spread(ibb_ctx *ctx, double width, int64_t n, const double *X, const double *F, double *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc): the spread of
 * ibb_spread without a context or workspace.  desc describes the grid (it
 * must pass the checks of ibb_create); X [dim][n] and F [dim][n] are node
 * positions and vectors, out receives the compact face field (every face
 * lattice, written in full).  The work is enqueued on `stream` (a
 * hipStream_t, NULL for the default stream) and the call does not wait for
 * it; it allocates nothing.  Its scratch (the bins of the nodes and one padded
 * face lattice of staging) is one static device array per GPU of
 * IBB_SPREAD_STATIC_MAX_BYTES, held until the process ends and shared by
 * every call on that GPU: calls that overlap on one GPU (several streams or
 * host threads) race and must be serialised by the caller.  The scratch
 * needs, each part rounded up to 256 bytes: 4 n (bin of each node) +
 * 4 B (counts) + 4 (B + 1) (starts) + 4 n (sorted ids) + 4 (ceil(max(B, n + 1)
 * / 1024) + 2) (scan sums) + 8 prod(n_a + 3) (staging), with B the number of
 * bins, prod over the axes of floor(n_a h / (2 width)) (at least 1 each);
 * IBB_ENOMEM if that exceeds the maximum (about 8 M padded grid points and a
 * few million nodes), IBB_EINVAL for bad arguments (as ibb_spread), both
 * before any work is enqueued; IBB_EDEVICE if the HIP runtime fails. */
#define IBB_SPREAD_STATIC_MAX_BYTES (64u << 20)
ibb_status ibb_spread_static(const ibb_desc *desc, double width, int64_t n, const double *X, const double *F,
                             double *out, void *stream);

/* Detached fragments (the results section observes pieces of biofilm
 * breaking off; the paper gives no algorithm): the connected components of
 * the graph of nodes joined by alive springs.  label (device, int32 [eta],
 * may be null) receives for every node the smallest node id of its fragment;
 * n_fragments and n_detached (host, may be null) receive the number of
 * fragments and of those with no anchored node (desc.attach_axis,
 * desc.attach_dist).  Exact integer results; IBB_ESTATE before nodes are
 * set.  Synchronises the stream. */
ibb_status ibb_fragments(ibb_ctx *ctx, int32_t *label, int *n_fragments, int *n_detached);

/* --- groups: several contexts stepped together (serving) ------------------
 *
 * A group steps independent contexts (different grids, dimensions,
 * coefficients, nodes) together so that their multigrid passes share
 * launches: every smoothing, residual, restriction and prolongation pass of
 * one level runs as one launch over all members of one dimension, and the
 * coarse part of every member's V-cycle runs in one launch with one
 * workgroup per member.  One tick of a solve (an FP64 V-cycle, or a refined
 * outer iteration with its inner FP32 V-cycles, then the FP64 residual and
 * its norm) is captured once as a HIP graph at creation and replayed; a
 * member that has met its stopping test is switched off by a device flag.
 * Each member follows exactly the sequence of operations of its own
 * ibb_projection_step / ibb_lagrangian_update, so its results are the same
 * as when it is stepped alone.
 *
 * Members must agree on precision, nu1, nu2 and (refined) inner_cycles,
 * may not use Galerkin coarse operators (IBB_EINVAL otherwise) and may not
 * repeat.  Members with krylov_restart > 0
 * are solved one by one (their GCR solves do not share launches); the other
 * members share them.  They must outlive the group and
 * keep their workspaces; a member can still be used on its own between group
 * calls.  The group's work runs on a stream of its own, ordered after each
 * member's stream on entry, with each member's stream ordered after it on
 * return.  The workspace (device memory, >= ibb_group_footprint_bytes,
 * owned by the caller, kept until ibb_group_destroy) holds the launch
 * tables, the member flags and the norms. */
typedef struct ibb_group ibb_group;

ibb_status ibb_group_footprint_bytes(ibb_ctx *const *ctxs, int n, size_t *bytes);
ibb_status ibb_group_create(ibb_ctx *const *ctxs, int n, void *workspace, size_t bytes, ibb_group **out);
ibb_status ibb_group_destroy(ibb_group *group);
/* Take member `member` (its index in ctxs at creation) out of the group's
 * later calls (active = 0) or back in (1); members start active.  A member
 * that is out gets no work from ibb_group_projection_step or
 * ibb_group_lagrangian_update (its statistics entries are zeroed), and may
 * meanwhile be reloaded on its own (ibb_set_params, ibb_set_state,
 * ibb_set_nodes, ibb_set_springs, ibb_update_coefficients).  The group's
 * graphs are not captured again: this is how a serving loop admits and
 * retires requests in slots of a fixed group.  Host only. */
ibb_status ibb_group_set_active(ibb_group *group, int member, int active);
/* One projection step of every member (as ibb_projection_step); per_ctx
 * (host, n entries, may be null) receives each member's statistics, with the
 * group's solve times.  A member that did not converge is reported in its
 * statistics and makes the call return its status; the others are stepped. */
ibb_status ibb_group_projection_step(ibb_group *group, ibb_solve_stats *per_ctx);
/* One Lagrangian update of every member (as ibb_lagrangian_update). */
ibb_status ibb_group_lagrangian_update(ibb_group *group, ibb_lag_stats *per_ctx);
const char *ibb_group_last_error(const ibb_group *group);

/* --- diagnostics ----------------------------------------------------------- */

/* Device timing of the solver kernels.  While enabled, every launch of a
 * multigrid solve (and the main kernels of the Lagrangian update) carries a
 * pair of HIP events that its dispatch records at
 * the kernel's start and end (on the context's stream; solver iterations are
 * then launched kernel by kernel instead of as graph replays); the durations
 * accumulate per kernel class until read.  kernel_class = site + 32 x level,
 * level the multigrid level the launch works on (for a restriction the
 * coarse one, for the one-workgroup coarse cycle its start level), site:
 *    0 viscous smoother colour pass FP64      1 pressure smoother FP64
 *    2 viscous smoother FP32                  3 pressure smoother FP32
 *    4 viscous residual FP64                  5 pressure residual FP64
 *    6 viscous residual FP32                  7 pressure residual FP32
 *    8 restriction FP64                       9 restriction FP32
 *   10 prolongation FP64                     11 prolongation FP32
 *   12 one-workgroup coarse cycle, viscous FP64   13 ... pressure FP64
 *   14 one-workgroup coarse cycle, viscous FP32   15 ... pressure FP32
 *   16 coarsest dense solve apply            17 outer-loop passes of level 0
 *      (norms, reductions, FP32 casts, clears, FP64 corrections)
 *   18 GCR vector passes                     19/20 constant-viscosity
 *      smoother FP64/FP32                    21/22 one-launch red-black
 *      sweep FP64/FP32
 * and, in the Lagrangian update (level 0): 23 spread of force and density
 * (per face lattice, units = its points), 24 viscosity gather (per cell or
 * edge lattice), 25 interpolation (units = nodes x dim), 26 spring forces
 * (units = nodes); with Galerkin coarse operators (level >= 1): 27 operator
 * build (units = the level's viscous unknowns), 28/29 smoother colour pass
 * FP64/FP32, 30/31 residual FP64/FP32
 * ibb_profile_read (host outputs) returns the launches, their summed device
 * time and the summed number of unknowns they updated or evaluated (for the
 * cycle, the start level's unknowns); enabling resets the totals. */
#define IBB_PROFILE_CLASSES 512
ibb_status ibb_profile_enable(ibb_ctx *ctx, int enable);
ibb_status ibb_profile_read(ibb_ctx *ctx, int kernel_class, long long *launches, double *total_ms,
                            long long *units);

const char *ibb_status_string(ibb_status s);
const char *ibb_last_error(const ibb_ctx *ctx);
/* number of multigrid levels and the cell counts of level l (host) */
ibb_status ibb_level_info(const ibb_ctx *ctx, int level, int *nlevels, int n[3]);

#ifdef __cplusplus
}
#endif

#endif /* IBMG_H */
