/*
 * ibmg_oracle.c -- plain, slow FP64 CPU oracle for the immersed-boundary
 * biofilm time step of Hammond, Stewart, Younger, Solomon and Bortz,
 * "Spatially heterogeneous biofilm simulations using an immersed boundary
 * method with Lagrangian nodes defined by bacterial locations".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code with the HIP library.
 *
 * What it computes, and where each part comes from:
 *   - the regularised delta (Sec. "Dirac Delta Approximation": eq:PhiPeskin,
 *     eq:PhiCosAlternative, eq:Dirac Delta Approx),
 *   - spread of force and density, interpolation of velocity
 *     (eq:discrForceCouple, eq:discrDensCouple, eq:discrVelCouple),
 *   - the viscosity field as a max over nodes (eq:ViscExp),
 *   - Hookean springs with breakage (eq:springF, eq:defineK and the
 *     twice-the-rest-length rule of the "Elastic Forces" section), and the
 *     detached fragments they leave (connected components, see
 *     orc_fragments),
 *   - the projection step (eq:NSdis1-1, eq:divergenceGrad,
 *     eq:divergencePartial, eq:NSdis2, eq:NSdis4) on a staggered MAC grid,
 *   - geometric multigrid with red-black Gauss-Seidel, full-weighting
 *     restriction, linear prolongation and V-cycles to a relative residual
 *     (Sec. "Multigrid"), with the coarse-viscosity scaling of
 *     eq:ViscCoarseGrid, or with Galerkin coarse operators R A P for the
 *     viscous system (the second remedy named in Sec. "Numerical
 *     Concerns"; see galerkin_level).
 *
 * Style: every field lives in a ghost-padded array.  Boundary conditions
 * are imposed by filling the ghost layer from a rule table, and the
 * interior stencil formula is then applied unchanged at every unknown.
 * The linear operators are assembled into CSR matrices by probing that
 * stencil; Gauss-Seidel, residuals and the coarsest direct solve then work
 * on the assembled matrix, which is the plain definition of each step.
 *
 * Compile: gcc -O2 -ffp-contract=off -fPIC -shared (no fused multiply-add).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* problem description (mirrored by a ctypes Structure in oracle/)     */
/* ------------------------------------------------------------------ */
enum { AX_PERIODIC = 0, AX_WALLS = 1, AX_INOUT = 2 };
enum { PHI_COS = 0, PHI_PESKIN4 = 1 };

typedef struct {
    int dim;            /* 2 or 3 */
    int n[3];           /* cells per axis (n[2] = 1 in 2D) */
    int axis_bc[3];     /* AX_* per axis */
    double h;           /* isotropic mesh width */
    double sigma, eps, inv_re, force_coef, dt;
    double body_force[3];
    double rho0, rho_b, d0_pow_d;
    double mu_out, mu_max, omega;
    int kernel;
    double break_ratio;
    int nu1, nu2, max_levels, max_cycles;
    double rtol;
    double gamma[16];
    int decoupled;      /* 1: constant-viscosity momentum operator, eq:NSdis1 */
    int galerkin;       /* 1: viscous coarse operators R A P (Sec. "Numerical Concerns") */
} orc_desc;

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_ENOMEM = 2, ORC_ENOCONV = 3, ORC_ENUMERIC = 4 };

/* largest coarsest-level system solved directly; above it the coarsest
 * level is only smoothed (so a one-level hierarchy is plain relaxation) */
#define DENSE_MAX 64

/* ------------------------------------------------------------------ */
/* the regularised delta                                               */
/* ------------------------------------------------------------------ */

/* phi_1, Peskin's four-point function, eq:PhiPeskin */
static double phi_peskin4(double r)
{
    double a = fabs(r);
    if (a <= 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) / 8.0;
    if (a < 2.0) return (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a)) / 8.0;
    return 0.0;
}

/* phi_2, the cosine function, eq:PhiCosAlternative */
static double phi_cos(double r)
{
    double a = fabs(r);
    if (a < 2.0) return 0.25 * (1.0 + cos(M_PI * a / 2.0));
    return 0.0;
}

static double phi(int kernel, double r)
{
    return kernel == PHI_PESKIN4 ? phi_peskin4(r) : phi_cos(r);
}

double orc_phi(int kernel, double r) { return phi(kernel, r); }

void orc_phi_v(int kernel, const double *r, double *out, long n)
{
    for (long i = 0; i < n; ++i) out[i] = phi(kernel, r[i]);
}

/* ------------------------------------------------------------------ */
/* grids, lattices and padded storage                                  */
/* ------------------------------------------------------------------ */
typedef struct {
    int D;
    int n[3];
    int bc[3];
    double h;
    int m[3];   /* padded extent per axis */
    int o[3];   /* offset of index 0 inside the padding */
    long size;
} grid_t;

static void grid_init(grid_t *g, int D, const int n[3], const int bc[3], double h)
{
    g->D = D;
    g->h = h;
    g->size = 1;
    for (int d = 0; d < 3; ++d) {
        g->n[d] = d < D ? n[d] : 1;
        g->bc[d] = d < D ? bc[d] : AX_PERIODIC;
        g->m[d] = d < D ? n[d] + 3 : 1;   /* indices -1 .. n+1 */
        g->o[d] = d < D ? 1 : 0;
        g->size *= g->m[d];
    }
}

static inline long P3(const grid_t *g, const int q[3])
{
    return ((long)(q[2] + g->o[2]) * g->m[1] + (q[1] + g->o[1])) * g->m[0] + (q[0] + g->o[0]);
}

static inline long Pijk(const grid_t *g, int i, int j, int k)
{
    int q[3] = {i, j, k};
    return P3(g, q);
}

/* A lattice: cell centres, the faces normal to axis a, or the edges parallel
 * to axis c (in 2D the only edge lattice is the corner lattice, c = 2). */
enum { LAT_CELL = 0, LAT_FACE = 1, LAT_EDGE = 2 };
typedef struct { int kind, axis; } lat_t;

static int is_vert(lat_t L, int d)
{
    if (L.kind == LAT_CELL) return 0;
    if (L.kind == LAT_FACE) return d == L.axis;
    return d != L.axis;
}

/* coordinate of lattice index q along axis d */
static double coord(const grid_t *g, lat_t L, int d, int q)
{
    return is_vert(L, d) ? q * g->h : (q + 0.5) * g->h;
}

/* positions held in the closed domain (these are exchanged with callers) */
static void stored_range(const grid_t *g, lat_t L, int d, int *lo, int *hi)
{
    if (d >= g->D) { *lo = *hi = 0; return; }
    *lo = 0;
    if (!is_vert(L, d)) { *hi = g->n[d] - 1; return; }
    *hi = g->bc[d] == AX_PERIODIC ? g->n[d] - 1 : g->n[d];
}

/* positions that are unknowns of the linear systems */
static void unknown_range(const grid_t *g, lat_t L, int d, int *lo, int *hi)
{
    if (d >= g->D) { *lo = *hi = 0; return; }
    if (!is_vert(L, d)) { *lo = 0; *hi = g->n[d] - 1; return; }
    switch (g->bc[d]) {
    case AX_PERIODIC: *lo = 0; *hi = g->n[d] - 1; break;
    case AX_WALLS: *lo = 1; *hi = g->n[d] - 1; break;
    default: *lo = 1; *hi = g->n[d]; break;      /* inflow face fixed, outflow face free */
    }
}

static long stored_count(const grid_t *g, lat_t L)
{
    long c = 1;
    for (int d = 0; d < 3; ++d) {
        int lo, hi;
        stored_range(g, L, d, &lo, &hi);
        c *= (hi - lo + 1);
    }
    return c;
}

/* ------------------------------------------------------------------ */
/* ghost rules                                                         */
/* ------------------------------------------------------------------ */
/*
 * ROLE_PRES    pressure and pressure corrections: zero normal derivative at
 *              walls and the inflow, p = 0 on the outflow face, wrap when
 *              periodic.
 * ROLE_VEL     a velocity component with homogeneous boundary data (the
 *              unknown part of the solve, corrections, residuals): zero
 *              normal velocity on walls and inflow, zero tangential velocity
 *              on walls and inflow (odd ghost), zero normal derivative at
 *              the outflow (even ghost; the outflow face itself is free).
 * ROLE_VELFULL the same rules with the stored boundary values kept (the
 *              inflow profile); one extra layer beyond a fixed face is the
 *              odd reflection through the face value.
 * ROLE_COEF    coefficient fields: even reflection, wrap when periodic.
 */
enum { ROLE_PRES = 0, ROLE_VEL = 1, ROLE_VELFULL = 2, ROLE_COEF = 3 };

/* padded index of q with its coordinate along axis d replaced by t */
static inline long along(const grid_t *g, const int q[3], int d, int t)
{
    int r[3] = {q[0], q[1], q[2]};
    r[d] = t;
    return P3(g, r);
}

static void fill_ghosts(const grid_t *g, lat_t L, int role, double *v)
{
    for (int d = 0; d < g->D; ++d) {
        int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
        int n = g->n[d];
        int vert = is_vert(L, d);
        int bc = g->bc[d];
        for (int a2 = -g->o[e2]; a2 < g->m[e2] - g->o[e2]; ++a2) {
            for (int a1 = -g->o[e1]; a1 < g->m[e1] - g->o[e1]; ++a1) {
                int q[3] = {0, 0, 0};
                q[e1] = a1;
                q[e2] = a2;
#define V(idx) v[along(g, q, d, (idx))]
                if (!vert) {
                    if (bc == AX_PERIODIC) {
                        V(-1) = V(n - 1);
                        V(n) = V(0);
                        V(n + 1) = NAN;
                    } else {
                        double sl, sh;
                        int out_hi = bc == AX_INOUT;
                        if (role == ROLE_PRES) { sl = 1.0; sh = out_hi ? -1.0 : 1.0; }
                        else if (role == ROLE_COEF) { sl = 1.0; sh = 1.0; }
                        else { sl = -1.0; sh = out_hi ? 1.0 : -1.0; }
                        V(-1) = sl * V(0);
                        V(n) = sh * V(n - 1);
                        V(n + 1) = NAN;
                    }
                } else {
                    if (bc == AX_PERIODIC) {
                        V(n) = V(0);
                        V(-1) = V(n - 1);
                        V(n + 1) = V(1);
                    } else if (role == ROLE_COEF) {
                        V(-1) = V(1);
                        V(n + 1) = V(n - 1);
                    } else if (role == ROLE_VEL) {
                        V(0) = 0.0;
                        V(-1) = NAN;
                        if (bc == AX_WALLS) { V(n) = 0.0; V(n + 1) = NAN; }
                        else V(n + 1) = V(n - 1);
                    } else if (role == ROLE_VELFULL) {
                        V(-1) = 2.0 * V(0) - V(1);
                        if (bc == AX_WALLS) V(n + 1) = 2.0 * V(n) - V(n - 1);
                        else V(n + 1) = V(n - 1);
                    } else {
                        V(-1) = NAN;
                        V(n + 1) = NAN;
                    }
                }
#undef V
            }
        }
    }
}

/* compact (exchange) layout <-> padded layout: the compact layout lists the
 * closed-domain positions of one lattice, x fastest */
static void compact_to_padded(const grid_t *g, lat_t L, const double *c, double *p)
{
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) stored_range(g, L, d, &lo[d], &hi[d]);
    long t = 0;
    for (int k = lo[2]; k <= hi[2]; ++k)
        for (int j = lo[1]; j <= hi[1]; ++j)
            for (int i = lo[0]; i <= hi[0]; ++i) p[Pijk(g, i, j, k)] = c[t++];
}

static void padded_to_compact(const grid_t *g, lat_t L, const double *p, double *c)
{
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) stored_range(g, L, d, &lo[d], &hi[d]);
    long t = 0;
    for (int k = lo[2]; k <= hi[2]; ++k)
        for (int j = lo[1]; j <= hi[1]; ++j)
            for (int i = lo[0]; i <= hi[0]; ++i) c[t++] = p[Pijk(g, i, j, k)];
}

static double *padded_alloc(const grid_t *g)
{
    double *p = (double *)malloc(sizeof(double) * g->size);
    if (p)
        for (long i = 0; i < g->size; ++i) p[i] = 0.0;
    return p;
}

static lat_t face_lat(int a) { lat_t L = {LAT_FACE, a}; return L; }
static lat_t cell_lat(void) { lat_t L = {LAT_CELL, 0}; return L; }
static lat_t edge_lat(int c) { lat_t L = {LAT_EDGE, c}; return L; }

/* edge lattices present: 3D edges parallel to x, y, z; 2D the corner lattice */
static int edge_first(int D) { return D == 3 ? 0 : 2; }

/* ------------------------------------------------------------------ */
/* unknown numbering                                                   */
/* ------------------------------------------------------------------ */
typedef struct {
    int ncomp;
    lat_t lat[3];
    int lo[3][3], hi[3][3];
    long cnt[3];
    long off[4];
} umap_t;

static void umap_init(umap_t *u, const grid_t *g, int velocity)
{
    u->ncomp = velocity ? g->D : 1;
    u->off[0] = 0;
    for (int c = 0; c < u->ncomp; ++c) {
        u->lat[c] = velocity ? face_lat(c) : cell_lat();
        u->cnt[c] = 1;
        for (int d = 0; d < 3; ++d) {
            unknown_range(g, u->lat[c], d, &u->lo[c][d], &u->hi[c][d]);
            u->cnt[c] *= (u->hi[c][d] - u->lo[c][d] + 1);
        }
        u->off[c + 1] = u->off[c] + u->cnt[c];
    }
}

static long umap_total(const umap_t *u) { return u->off[u->ncomp]; }

static void umap_pos(const umap_t *u, long r, int *comp, int q[3])
{
    int c = 0;
    while (r >= u->off[c + 1]) ++c;
    long t = r - u->off[c];
    int ex = u->hi[c][0] - u->lo[c][0] + 1, ey = u->hi[c][1] - u->lo[c][1] + 1;
    q[0] = u->lo[c][0] + (int)(t % ex);
    t /= ex;
    q[1] = u->lo[c][1] + (int)(t % ey);
    t /= ey;
    q[2] = u->lo[c][2] + (int)t;
    *comp = c;
}

static long umap_index(const umap_t *u, int c, const int q[3])
{
    int ex = u->hi[c][0] - u->lo[c][0] + 1, ey = u->hi[c][1] - u->lo[c][1] + 1;
    return u->off[c] + ((long)(q[2] - u->lo[c][2]) * ey + (q[1] - u->lo[c][1])) * ex + (q[0] - u->lo[c][0]);
}

/* vector of unknowns -> padded arrays (zero elsewhere), ghosts filled */
static void vec_to_padded(const grid_t *g, const umap_t *u, const double *x, double *const *pad, int velocity)
{
    for (int c = 0; c < u->ncomp; ++c) memset(pad[c], 0, sizeof(double) * g->size);
    long n = umap_total(u);
    for (long r = 0; r < n; ++r) {
        int c, q[3];
        umap_pos(u, r, &c, q);
        pad[c][P3(g, q)] = x[r];
    }
    for (int c = 0; c < u->ncomp; ++c) fill_ghosts(g, u->lat[c], velocity ? ROLE_VEL : ROLE_PRES, pad[c]);
}

static void padded_to_vec(const grid_t *g, const umap_t *u, double *const *pad, double *x)
{
    long n = umap_total(u);
    for (long r = 0; r < n; ++r) {
        int c, q[3];
        umap_pos(u, r, &c, q);
        x[r] = pad[c][P3(g, q)];
    }
}

/* ------------------------------------------------------------------ */
/* a multigrid level: grid, coefficients, assembled operators          */
/* ------------------------------------------------------------------ */
typedef struct {
    long nrow, nnz;
    long *rowptr;
    long *col;
    double *val;
} csr_t;

typedef struct {
    grid_t g;
    double *rho[3];   /* density on the faces normal to each axis */
    double *beta[3];  /* 1 / rho on the same faces */
    double *mu_c;     /* viscosity at cell centres */
    double *mu_e[3];  /* viscosity on edges parallel to axis c (2D: corners in [2]) */
    double mu0;       /* the constant viscosity of the decoupled operator on this level */
    umap_t up, uu;
    csr_t Ap, Au;
} level_t;

typedef struct {
    orc_desc d;
    int L;
    int singular_p;
    level_t lv[16];
} hier_t;

/* ------------------------------------------------------------------ */
/* the discrete operators (stencils on padded arrays)                  */
/* ------------------------------------------------------------------ */

/* pressure operator A_p = -D(beta G), eq:divergenceGrad with MAC faces */
static double apply_p_at(const level_t *L, const double *p, const int q[3])
{
    const grid_t *g = &L->g;
    double h2 = g->h * g->h;
    long c = P3(g, q);
    double s = 0.0;
    for (int d = 0; d < g->D; ++d) {
        int qp[3] = {q[0], q[1], q[2]}, qm[3] = {q[0], q[1], q[2]};
        qp[d] += 1;
        qm[d] -= 1;
        long cp = P3(g, qp), cm = P3(g, qm);
        /* faces normal to d: the high face of cell q has index q+e_d */
        s += L->beta[d][cp] * (p[c] - p[cp]) + L->beta[d][c] * (p[c] - p[cm]);
    }
    return s / h2;
}

/* viscous stress divergence [D.(mu (D u + D u^T))]_a at an a-face,
 * eq:divergenceGrad and eq:divergencePartial on MAC positions: the
 * same-axis term uses mu at the two neighbouring cell centres, a cross
 * term for axis b uses mu on the two edges between this face and its
 * b-neighbours. */
static double visc_at(const level_t *L, double *const *u, int a, const int q[3])
{
    const grid_t *g = &L->g;
    double h2 = g->h * g->h;
    long f = P3(g, q);
    int qa_p[3] = {q[0], q[1], q[2]}, qa_m[3] = {q[0], q[1], q[2]};
    qa_p[a] += 1;
    qa_m[a] -= 1;
    const double *ua = u[a];
    /* cells right (index q) and left (index q - e_a) of the face */
    double s = 2.0 * L->mu_c[f] * (ua[P3(g, qa_p)] - ua[f]) - 2.0 * L->mu_c[P3(g, qa_m)] * (ua[f] - ua[P3(g, qa_m)]);
    for (int b = 0; b < g->D; ++b) {
        if (b == a) continue;
        const double *ub = u[b];
        const double *me = L->mu_e[3 - a - b];
        int qb_p[3] = {q[0], q[1], q[2]}, qb_m[3] = {q[0], q[1], q[2]};
        qb_p[b] += 1;
        qb_m[b] -= 1;
        int qbp_am[3] = {qb_p[0], qb_p[1], qb_p[2]};
        qbp_am[a] -= 1;
        /* edge above (index q + e_b) and below (index q) along b */
        double dbua_p = ua[P3(g, qb_p)] - ua[f];
        double daub_p = ub[P3(g, qb_p)] - ub[P3(g, qbp_am)];
        double dbua_m = ua[f] - ua[P3(g, qb_m)];
        double daub_m = ub[f] - ub[P3(g, qa_m)];
        s += me[P3(g, qb_p)] * (dbua_p + daub_p) - me[f] * (dbua_m + daub_m);
    }
    return s / h2;
}

/* constant viscosity: mu0 L_h u_a, the 2D + 1 point Laplacian of eq:NSdis1
 * on the a-face lattice.  Each component only sees itself; the neighbours
 * across a boundary come from the same ghost images as in visc_at. */
static double lap_at(const level_t *L, double *const *u, int a, const int q[3])
{
    const grid_t *g = &L->g;
    double h2 = g->h * g->h;
    const double *ua = u[a];
    long f = P3(g, q);
    double s = 0.0;
    for (int b = 0; b < g->D; ++b) {
        int qp[3] = {q[0], q[1], q[2]}, qm[3] = {q[0], q[1], q[2]};
        qp[b] += 1;
        qm[b] -= 1;
        s += (ua[P3(g, qp)] - ua[f]) - (ua[f] - ua[P3(g, qm)]);
    }
    return L->mu0 * s / h2;
}

/* viscous operator A_u = (sigma rho / dt) I - Re^-1 V, eq:NSdis1-1; with
 * constant viscosity V is mu L_h applied to each component, eq:NSdis1 */
static double apply_u_at(const level_t *L, const orc_desc *d, double *const *u, int a, const int q[3])
{
    long f = P3(&L->g, q);
    double v = d->decoupled ? lap_at(L, u, a, q) : visc_at(L, u, a, q);
    return d->sigma / d->dt * L->rho[a][f] * u[a][f] - d->inv_re * v;
}

/* ------------------------------------------------------------------ */
/* CSR assembly by probing the stencil                                  */
/* ------------------------------------------------------------------ */
typedef struct { long r, c; double v; } trip_t;

static int trip_cmp(const void *x, const void *y)
{
    const trip_t *a = (const trip_t *)x, *b = (const trip_t *)y;
    if (a->r != b->r) return a->r < b->r ? -1 : 1;
    if (a->c != b->c) return a->c < b->c ? -1 : 1;
    return 0;
}

static void csr_free(csr_t *A)
{
    free(A->rowptr);
    free(A->col);
    free(A->val);
    memset(A, 0, sizeof(*A));
}

/* probing modulus along an axis: 4 separates the three candidates q-1, q,
 * q+1; a periodic axis whose length is not a multiple of 4 is probed point
 * by point so that wrapped candidates stay distinct */
static int probe_mod(const grid_t *g, int d)
{
    if (d >= g->D) return 1;
    if (g->bc[d] == AX_PERIODIC && g->n[d] % 4 != 0) return g->n[d];
    return 4;
}

static int assemble(const level_t *L, const orc_desc *dsc, int velocity, csr_t *A)
{
    const grid_t *g = &L->g;
    const umap_t *um = velocity ? &L->uu : &L->up;
    long n = umap_total(um);
    int nc = um->ncomp;
    double *x[3] = {0, 0, 0}, *y[3] = {0, 0, 0};
    for (int c = 0; c < nc; ++c) {
        x[c] = padded_alloc(g);
        y[c] = padded_alloc(g);
        if (!x[c] || !y[c]) return ORC_ENOMEM;
    }
    long cap = n * (velocity ? (1 + 2 * g->D + 4 * (g->D - 1)) : (1 + 2 * g->D)) + 16, nt = 0;
    trip_t *T = (trip_t *)malloc(sizeof(trip_t) * cap);
    if (!T) return ORC_ENOMEM;
    int M[3];
    for (int d = 0; d < 3; ++d) M[d] = probe_mod(g, d);

    for (int ca = 0; ca < nc; ++ca) {
        for (int o2 = 0; o2 < M[2]; ++o2)
            for (int o1 = 0; o1 < M[1]; ++o1)
                for (int o0 = 0; o0 < M[0]; ++o0) {
                    int o[3] = {o0, o1, o2};
                    /* probe vector: ones on the unknowns of component ca congruent to o */
                    for (int c = 0; c < nc; ++c) memset(x[c], 0, sizeof(double) * g->size);
                    int any = 0;
                    for (long r = um->off[ca]; r < um->off[ca + 1]; ++r) {
                        int c, q[3];
                        umap_pos(um, r, &c, q);
                        if (q[0] % M[0] == o0 && q[1] % M[1] == o1 && q[2] % M[2] == o2) {
                            x[ca][P3(g, q)] = 1.0;
                            any = 1;
                        }
                    }
                    if (!any) continue;
                    for (int c = 0; c < nc; ++c) fill_ghosts(g, um->lat[c], velocity ? ROLE_VEL : ROLE_PRES, x[c]);
                    for (long r = 0; r < n; ++r) {
                        int cb, q[3];
                        umap_pos(um, r, &cb, q);
                        double v = velocity ? apply_u_at(L, dsc, x, cb, q) : apply_p_at(L, x[0], q);
                        if (v == 0.0) continue;
                        if (v != v) { free(T); return ORC_ENUMERIC; }
                        /* the column: the probed unknown of component ca within one step */
                        int qc[3];
                        for (int d = 0; d < 3; ++d) {
                            qc[d] = INT32_MIN;
                            if (d >= g->D) { qc[d] = 0; continue; }
                            for (int s = -1; s <= 1; ++s) {
                                int t = q[d] + s;
                                if (g->bc[d] == AX_PERIODIC) t = (t + g->n[d]) % g->n[d];
                                if (t < um->lo[ca][d] || t > um->hi[ca][d]) continue;
                                if (t % M[d] == o[d]) { qc[d] = t; break; }
                            }
                        }
                        if (qc[0] == INT32_MIN || qc[1] == INT32_MIN || qc[2] == INT32_MIN) { free(T); return ORC_EINVAL; }
                        if (nt == cap) {
                            cap *= 2;
                            trip_t *T2 = (trip_t *)realloc(T, sizeof(trip_t) * cap);
                            if (!T2) { free(T); return ORC_ENOMEM; }
                            T = T2;
                        }
                        T[nt].r = r;
                        T[nt].c = umap_index(um, ca, qc);
                        T[nt].v = v;
                        ++nt;
                    }
                }
    }
    for (int c = 0; c < nc; ++c) { free(x[c]); free(y[c]); }
    qsort(T, nt, sizeof(trip_t), trip_cmp);
    A->nrow = n;
    A->nnz = nt;
    A->rowptr = (long *)calloc(n + 1, sizeof(long));
    A->col = (long *)malloc(sizeof(long) * (nt ? nt : 1));
    A->val = (double *)malloc(sizeof(double) * (nt ? nt : 1));
    if (!A->rowptr || !A->col || !A->val) { free(T); return ORC_ENOMEM; }
    for (long t = 0; t < nt; ++t) {
        A->rowptr[T[t].r + 1]++;
        A->col[t] = T[t].c;
        A->val[t] = T[t].v;
    }
    for (long r = 0; r < n; ++r) A->rowptr[r + 1] += A->rowptr[r];
    free(T);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* transfers: full weighting and linear interpolation, per axis         */
/* ------------------------------------------------------------------ */
/* restriction weights along one axis for coarse index I */
static int rst_axis(int vert, int I, int fq[4], double w[4])
{
    if (vert) {
        fq[0] = 2 * I - 1; w[0] = 0.25;
        fq[1] = 2 * I;     w[1] = 0.5;
        fq[2] = 2 * I + 1; w[2] = 0.25;
        return 3;
    }
    fq[0] = 2 * I - 1; w[0] = 0.125;
    fq[1] = 2 * I;     w[1] = 0.375;
    fq[2] = 2 * I + 1; w[2] = 0.375;
    fq[3] = 2 * I + 2; w[3] = 0.125;
    return 4;
}

/* prolongation weights along one axis for fine index f */
static int prl_axis(int vert, int f, int cq[2], double w[2])
{
    if (vert) {
        if (f % 2 == 0) { cq[0] = f / 2; w[0] = 1.0; return 1; }
        cq[0] = (f - 1) / 2; w[0] = 0.5;
        cq[1] = (f + 1) / 2; w[1] = 0.5;
        return 2;
    }
    int I = f / 2;
    cq[0] = I; w[0] = 0.75;
    cq[1] = (f % 2 == 0) ? I - 1 : I + 1; w[1] = 0.25;
    return 2;
}

/* restrict a padded fine field (ghosts filled) to coarse position qc */
static double restrict_at(const grid_t *gf, lat_t L, const double *fine, const int qc[3])
{
    int fq[3][4], nf[3];
    double w[3][4];
    for (int d = 0; d < 3; ++d) {
        if (d >= gf->D) { fq[d][0] = 0; w[d][0] = 1.0; nf[d] = 1; continue; }
        nf[d] = rst_axis(is_vert(L, d), qc[d], fq[d], w[d]);
    }
    double s = 0.0;
    for (int c = 0; c < nf[2]; ++c)
        for (int b = 0; b < nf[1]; ++b)
            for (int a = 0; a < nf[0]; ++a)
                s += w[0][a] * w[1][b] * w[2][c] * fine[Pijk(gf, fq[0][a], fq[1][b], fq[2][c])];
    return s;
}

static double prolong_at(const grid_t *gc, lat_t L, const double *coarse, const int qf[3])
{
    int cq[3][2], nc[3];
    double w[3][2];
    for (int d = 0; d < 3; ++d) {
        if (d >= gc->D) { cq[d][0] = 0; w[d][0] = 1.0; nc[d] = 1; continue; }
        nc[d] = prl_axis(is_vert(L, d), qf[d], cq[d], w[d]);
    }
    double s = 0.0;
    for (int c = 0; c < nc[2]; ++c)
        for (int b = 0; b < nc[1]; ++b)
            for (int a = 0; a < nc[0]; ++a)
                s += w[0][a] * w[1][b] * w[2][c] * coarse[Pijk(gc, cq[0][a], cq[1][b], cq[2][c])];
    return s;
}

/* restrict a coefficient field over every stored coarse position */
static void restrict_coef(const grid_t *gf, const grid_t *gc, lat_t L, const double *fine, double *coarse, double scale)
{
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) stored_range(gc, L, d, &lo[d], &hi[d]);
    for (int k = lo[2]; k <= hi[2]; ++k)
        for (int j = lo[1]; j <= hi[1]; ++j)
            for (int i = lo[0]; i <= hi[0]; ++i) {
                int qc[3] = {i, j, k};
                coarse[P3(gc, qc)] = scale * restrict_at(gf, L, fine, qc);
            }
    fill_ghosts(gc, L, ROLE_COEF, coarse);
}

/* ------------------------------------------------------------------ */
/* hierarchy                                                           */
/* ------------------------------------------------------------------ */
static int level_alloc(level_t *L, const grid_t *g)
{
    memset(L, 0, sizeof(*L));
    L->g = *g;
    for (int a = 0; a < g->D; ++a) {
        L->rho[a] = padded_alloc(g);
        L->beta[a] = padded_alloc(g);
        if (!L->rho[a] || !L->beta[a]) return ORC_ENOMEM;
    }
    L->mu_c = padded_alloc(g);
    if (!L->mu_c) return ORC_ENOMEM;
    for (int c = edge_first(g->D); c < 3; ++c) {
        L->mu_e[c] = padded_alloc(g);
        if (!L->mu_e[c]) return ORC_ENOMEM;
    }
    umap_init(&L->up, g, 0);
    umap_init(&L->uu, g, 1);
    return ORC_OK;
}

static void level_free(level_t *L)
{
    for (int a = 0; a < 3; ++a) { free(L->rho[a]); free(L->beta[a]); free(L->mu_e[a]); }
    free(L->mu_c);
    csr_free(&L->Ap);
    csr_free(&L->Au);
}

static void level_betas(level_t *L)
{
    const grid_t *g = &L->g;
    for (int a = 0; a < g->D; ++a) {
        for (long t = 0; t < g->size; ++t) L->beta[a][t] = 1.0 / L->rho[a][t];
    }
}

/* number of levels: halve while every axis stays even and at least 2 */
static int count_levels(const orc_desc *d)
{
    int n[3] = {d->n[0], d->n[1], d->dim == 3 ? d->n[2] : 2};
    int L = 1;
    while (L < 16) {
        int ok = 1;
        for (int a = 0; a < d->dim; ++a)
            if (n[a] % 2 != 0 || n[a] / 2 < 2) ok = 0;
        if (!ok) break;
        for (int a = 0; a < d->dim; ++a) n[a] /= 2;
        ++L;
    }
    if (d->max_levels > 0 && d->max_levels < L) L = d->max_levels;
    return L;
}

static int galerkin_level(hier_t *H, int l);

static int desc_check(const orc_desc *d)
{
    if (d->dim != 2 && d->dim != 3) return ORC_EINVAL;
    for (int a = 0; a < d->dim; ++a) {
        if (d->n[a] < 2 || d->n[a] % 2) return ORC_EINVAL;
        if (d->axis_bc[a] < 0 || d->axis_bc[a] > 2) return ORC_EINVAL;
    }
    if (!(d->h > 0) || !(d->dt > 0) || !(d->sigma > 0)) return ORC_EINVAL;
    if (d->decoupled != 0 && d->decoupled != 1) return ORC_EINVAL;
    /* the decoupled form holds only where the viscosity is one constant */
    if (d->decoupled && d->mu_max != d->mu_out) return ORC_EINVAL;
    if (d->galerkin != 0 && d->galerkin != 1) return ORC_EINVAL;
    /* the Galerkin levels replace the coupled operator's coarse levels */
    if (d->galerkin && d->decoupled) return ORC_EINVAL;
    return ORC_OK;
}

void orc_hier_destroy(void *hp)
{
    hier_t *H = (hier_t *)hp;
    if (!H) return;
    for (int l = 0; l < H->L; ++l) level_free(&H->lv[l]);
    free(H);
}

/* Build every level from the finest coefficients (compact layouts):
 * rho on the D face lattices, mu at cells, mu on the edge lattices.
 * Coarse coefficients are the full-weighting restriction of the next finer
 * level; viscosity is multiplied by gamma[l] on level l (eq:ViscCoarseGrid). */
void *orc_hier_create(const orc_desc *d, const double *rho_faces, const double *mu_c, const double *mu_e, int *status)
{
    *status = desc_check(d);
    if (*status) return NULL;
    hier_t *H = (hier_t *)calloc(1, sizeof(hier_t));
    if (!H) { *status = ORC_ENOMEM; return NULL; }
    H->d = *d;
    H->L = count_levels(d);
    H->singular_p = 1;
    for (int a = 0; a < d->dim; ++a)
        if (d->axis_bc[a] == AX_INOUT) H->singular_p = 0;
    grid_t g;
    grid_init(&g, d->dim, d->n, d->axis_bc, d->h);
    for (int l = 0; l < H->L; ++l) {
        if ((*status = level_alloc(&H->lv[l], &g))) { orc_hier_destroy(H); return NULL; }
        int nn[3] = {g.n[0] / 2, g.n[1] / 2, g.n[2] / 2};
        if (d->dim == 2) nn[2] = 1;
        grid_t gc;
        grid_init(&gc, d->dim, nn, d->axis_bc, 2.0 * g.h);
        g = gc;
    }
    /* finest coefficients */
    level_t *L0 = &H->lv[0];
    long off = 0;
    for (int a = 0; a < d->dim; ++a) {
        compact_to_padded(&L0->g, face_lat(a), rho_faces + off, L0->rho[a]);
        fill_ghosts(&L0->g, face_lat(a), ROLE_COEF, L0->rho[a]);
        off += stored_count(&L0->g, face_lat(a));
    }
    compact_to_padded(&L0->g, cell_lat(), mu_c, L0->mu_c);
    fill_ghosts(&L0->g, cell_lat(), ROLE_COEF, L0->mu_c);
    off = 0;
    for (int c = edge_first(d->dim); c < 3; ++c) {
        compact_to_padded(&L0->g, edge_lat(c), mu_e + off, L0->mu_e[c]);
        fill_ghosts(&L0->g, edge_lat(c), ROLE_COEF, L0->mu_e[c]);
        off += stored_count(&L0->g, edge_lat(c));
    }
    level_betas(L0);
    L0->mu0 = d->mu_out;
    for (int l = 1; l < H->L; ++l) {
        level_t *F = &H->lv[l - 1], *C = &H->lv[l];
        double gm = d->gamma[l] > 0 ? d->gamma[l] : 1.0;
        C->mu0 = F->mu0 * gm;
        for (int a = 0; a < d->dim; ++a) restrict_coef(&F->g, &C->g, face_lat(a), F->rho[a], C->rho[a], 1.0);
        restrict_coef(&F->g, &C->g, cell_lat(), F->mu_c, C->mu_c, gm);
        for (int c = edge_first(d->dim); c < 3; ++c) restrict_coef(&F->g, &C->g, edge_lat(c), F->mu_e[c], C->mu_e[c], gm);
        level_betas(C);
    }
    for (int l = 0; l < H->L; ++l) {
        if ((*status = assemble(&H->lv[l], d, 0, &H->lv[l].Ap))) { orc_hier_destroy(H); return NULL; }
        if (d->galerkin && l > 0) *status = galerkin_level(H, l);
        else *status = assemble(&H->lv[l], d, 1, &H->lv[l].Au);
        if (*status) { orc_hier_destroy(H); return NULL; }
    }
    return H;
}

int orc_hier_levels(void *hp, int *dims /* [L][3] */, long *nunk /* [L][2]: pressure, velocity */)
{
    hier_t *H = (hier_t *)hp;
    for (int l = 0; l < H->L; ++l) {
        for (int d = 0; d < 3; ++d) dims[3 * l + d] = H->lv[l].g.n[d];
        nunk[2 * l] = umap_total(&H->lv[l].up);
        nunk[2 * l + 1] = umap_total(&H->lv[l].uu);
    }
    return H->L;
}

/* ------------------------------------------------------------------ */
/* smoother, residual, coarsest solve, V-cycle                          */
/* ------------------------------------------------------------------ */
static int row_colour(const umap_t *u, long r)
{
    int c, q[3];
    umap_pos(u, r, &c, q);
    return (q[0] + q[1] + q[2]) & 1;
}

/* one red-black Gauss-Seidel sweep: components in order, red then black
 * within a component; each row is x_i = (b_i - sum_{j!=i} a_ij x_j) / a_ii */
static void gs_sweep(const csr_t *A, const umap_t *u, const double *b, double *x)
{
    for (int c = 0; c < u->ncomp; ++c)
        for (int colour = 0; colour < 2; ++colour)
            for (long r = u->off[c]; r < u->off[c + 1]; ++r) {
                if (row_colour(u, r) != colour) continue;
                double s = b[r], diag = 0.0;
                for (long t = A->rowptr[r]; t < A->rowptr[r + 1]; ++t) {
                    if (A->col[t] == r) diag = A->val[t];
                    else s -= A->val[t] * x[A->col[t]];
                }
                x[r] = s / diag;
            }
}

static void residual(const csr_t *A, const double *b, const double *x, double *r)
{
    for (long i = 0; i < A->nrow; ++i) {
        double s = b[i];
        for (long t = A->rowptr[i]; t < A->rowptr[i + 1]; ++t) s -= A->val[t] * x[A->col[t]];
        r[i] = s;
    }
}

static double norm2(const double *v, long n)
{
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += v[i] * v[i];
    return sqrt(s);
}

/* dense Gaussian elimination with partial pivoting; a singular pressure
 * system gets a rank-one term alpha 1 1^T so that the solution satisfies
 * A x = b minus its mean */
static int dense_solve(const csr_t *A, int singular, const double *b, double *x)
{
    long n = A->nrow;
    double *M = (double *)calloc(n * n, sizeof(double));
    double *y = (double *)malloc(sizeof(double) * n);
    if (!M || !y) { free(M); free(y); return ORC_ENOMEM; }
    double tr = 0.0;
    for (long i = 0; i < n; ++i)
        for (long t = A->rowptr[i]; t < A->rowptr[i + 1]; ++t) {
            M[i * n + A->col[t]] += A->val[t];
            if (A->col[t] == i) tr += A->val[t];
        }
    if (singular) {
        double alpha = tr / ((double)n * (double)n);
        for (long i = 0; i < n * n; ++i) M[i] += alpha;
    }
    for (long i = 0; i < n; ++i) y[i] = b[i];
    for (long k = 0; k < n; ++k) {
        long p = k;
        for (long i = k + 1; i < n; ++i)
            if (fabs(M[i * n + k]) > fabs(M[p * n + k])) p = i;
        if (p != k) {
            for (long j = 0; j < n; ++j) { double t = M[k * n + j]; M[k * n + j] = M[p * n + j]; M[p * n + j] = t; }
            double t = y[k]; y[k] = y[p]; y[p] = t;
        }
        for (long i = k + 1; i < n; ++i) {
            double f = M[i * n + k] / M[k * n + k];
            for (long j = k; j < n; ++j) M[i * n + j] -= f * M[k * n + j];
            y[i] -= f * y[k];
        }
    }
    for (long i = n - 1; i >= 0; --i) {
        double s = y[i];
        for (long j = i + 1; j < n; ++j) s -= M[i * n + j] * x[j];
        x[i] = s / M[i * n + i];
    }
    free(M);
    free(y);
    return ORC_OK;
}

typedef struct { long sweeps_fine_equiv_num; double work_units; } wu_t;

static void restrict_residual(hier_t *H, int l, int velocity, const double *r, double *bc)
{
    level_t *F = &H->lv[l], *C = &H->lv[l + 1];
    const umap_t *uf = velocity ? &F->uu : &F->up, *uc = velocity ? &C->uu : &C->up;
    double *pad[3] = {0, 0, 0};
    for (int c = 0; c < uf->ncomp; ++c) pad[c] = padded_alloc(&F->g);
    vec_to_padded(&F->g, uf, r, pad, velocity);
    long n = umap_total(uc);
    for (long i = 0; i < n; ++i) {
        int c, q[3];
        umap_pos(uc, i, &c, q);
        bc[i] = restrict_at(&F->g, uc->lat[c], pad[c], q);
    }
    for (int c = 0; c < uf->ncomp; ++c) free(pad[c]);
}

static void prolong_add(hier_t *H, int l, int velocity, const double *xc, double *x)
{
    level_t *F = &H->lv[l], *C = &H->lv[l + 1];
    const umap_t *uf = velocity ? &F->uu : &F->up, *uc = velocity ? &C->uu : &C->up;
    double *pad[3] = {0, 0, 0};
    for (int c = 0; c < uc->ncomp; ++c) pad[c] = padded_alloc(&C->g);
    vec_to_padded(&C->g, uc, xc, pad, velocity);
    long n = umap_total(uf);
    for (long i = 0; i < n; ++i) {
        int c, q[3];
        umap_pos(uf, i, &c, q);
        x[i] += prolong_at(&C->g, uf->lat[c], pad[c], q);
    }
    for (int c = 0; c < uc->ncomp; ++c) free(pad[c]);
}

/* ------------------------------------------------------------------ */
/* Galerkin coarse operators                                            */
/* ------------------------------------------------------------------ */
/* Sec. "Numerical Concerns" names, as the second way to restore fast
 * convergence at large mu_max, coarse operators that satisfy the Galerkin
 * condition: A_{l+1} = R_l A_l P_l, with R_l and P_l the restriction and
 * prolongation of the V-cycle between levels l and l+1.  Here R_l and P_l
 * are the matrices of restrict_residual and prolong_add (boundary rules
 * included), assembled by probing, and the product is formed as
 * R_l (A_l P_l) with sparse matrix products. */

/* C = A B (A: n x k, B: k x ncol), row by row with a dense accumulator;
 * the columns of each row of C are sorted */
static int lcmp(const void *x, const void *y)
{
    long a = *(const long *)x, b = *(const long *)y;
    return a < b ? -1 : (a > b);
}

static int csr_mul(const csr_t *A, const csr_t *B, long ncol, csr_t *C)
{
    long n = A->nrow;
    long *mark = (long *)malloc(sizeof(long) * (ncol ? ncol : 1));
    double *acc = (double *)calloc(ncol ? ncol : 1, sizeof(double));
    long *cols = (long *)malloc(sizeof(long) * (ncol ? ncol : 1));
    C->nrow = n;
    C->rowptr = (long *)calloc(n + 1, sizeof(long));
    if (!mark || !acc || !cols || !C->rowptr) { free(mark); free(acc); free(cols); return ORC_ENOMEM; }
    for (long j = 0; j < ncol; ++j) mark[j] = -1;
    /* row lengths */
    for (long i = 0; i < n; ++i) {
        long len = 0;
        for (long t = A->rowptr[i]; t < A->rowptr[i + 1]; ++t) {
            long k = A->col[t];
            for (long u = B->rowptr[k]; u < B->rowptr[k + 1]; ++u)
                if (mark[B->col[u]] != i) { mark[B->col[u]] = i; ++len; }
        }
        C->rowptr[i + 1] = C->rowptr[i] + len;
    }
    C->nnz = C->rowptr[n];
    C->col = (long *)malloc(sizeof(long) * (C->nnz ? C->nnz : 1));
    C->val = (double *)malloc(sizeof(double) * (C->nnz ? C->nnz : 1));
    if (!C->col || !C->val) { free(mark); free(acc); free(cols); return ORC_ENOMEM; }
    for (long j = 0; j < ncol; ++j) mark[j] = -1;
    for (long i = 0; i < n; ++i) {
        long len = 0;
        for (long t = A->rowptr[i]; t < A->rowptr[i + 1]; ++t) {
            long k = A->col[t];
            double a = A->val[t];
            for (long u = B->rowptr[k]; u < B->rowptr[k + 1]; ++u) {
                long j = B->col[u];
                if (mark[j] != i) { mark[j] = i; acc[j] = 0.0; cols[len++] = j; }
                acc[j] += a * B->val[u];
            }
        }
        qsort(cols, len, sizeof(long), lcmp);
        for (long q = 0; q < len; ++q) {
            C->col[C->rowptr[i] + q] = cols[q];
            C->val[C->rowptr[i] + q] = acc[cols[q]];
        }
    }
    free(mark);
    free(acc);
    free(cols);
    return ORC_OK;
}

/* The matrix of the restriction (restrict_ = 1: coarse rows, fine columns)
 * or of the prolongation (fine rows, coarse columns) between levels l and
 * l+1.  Probing: the input unknowns of one component whose positions are
 * congruent to o modulo m (per axis) are set to one together; an output
 * row reads inputs only within a few points of its own position (in fine
 * units: |2t - q| <= 3 for the prolongation, |t - 2q| <= 3 for the
 * restriction), and there the congruence leaves exactly one candidate
 * (checked), which is the column of the value the row receives. */
static int probe_transfer(hier_t *H, int l, int restrict_, csr_t *M)
{
    level_t *F = &H->lv[l], *C = &H->lv[l + 1];
    const umap_t *uin = restrict_ ? &F->uu : &C->uu, *uout = restrict_ ? &C->uu : &F->uu;
    const grid_t *gin = restrict_ ? &F->g : &C->g;
    long nin = umap_total(uin), nout = umap_total(uout);
    int m[3];
    for (int d = 0; d < 3; ++d) {
        m[d] = d >= gin->D ? 1 : (restrict_ ? 8 : 4);
        if (d < gin->D && gin->bc[d] == AX_PERIODIC && gin->n[d] % m[d] != 0) m[d] = gin->n[d];
    }
    double *in = (double *)malloc(sizeof(double) * (nin ? nin : 1));
    double *out = (double *)malloc(sizeof(double) * (nout ? nout : 1));
    long cap = 16 * nout + 16, nt = 0;
    trip_t *T = (trip_t *)malloc(sizeof(trip_t) * cap);
    int st = ORC_OK;
    if (!in || !out || !T) st = ORC_ENOMEM;
    for (int ca = 0; ca < uin->ncomp && !st; ++ca)
        for (int o2 = 0; o2 < m[2] && !st; ++o2)
            for (int o1 = 0; o1 < m[1] && !st; ++o1)
                for (int o0 = 0; o0 < m[0] && !st; ++o0) {
                    int o[3] = {o0, o1, o2}, any = 0;
                    memset(in, 0, sizeof(double) * nin);
                    for (long r = uin->off[ca]; r < uin->off[ca + 1]; ++r) {
                        int c, q[3];
                        umap_pos(uin, r, &c, q);
                        if (q[0] % m[0] == o0 && q[1] % m[1] == o1 && q[2] % m[2] == o2) { in[r] = 1.0; any = 1; }
                    }
                    if (!any) continue;
                    if (restrict_) restrict_residual(H, l, 1, in, out);
                    else {
                        memset(out, 0, sizeof(double) * nout);
                        prolong_add(H, l, 1, in, out);
                    }
                    for (long r = 0; r < nout; ++r) {
                        if (out[r] == 0.0) continue;
                        int cb, q[3], t[3];
                        umap_pos(uout, r, &cb, q);
                        for (int d = 0; d < 3; ++d) {
                            t[d] = INT32_MIN;
                            if (d >= gin->D) { t[d] = 0; continue; }
                            int lo = restrict_ ? 2 * q[d] - 3 : (q[d] - 3 + 1) / 2 - 1;
                            int hi = restrict_ ? 2 * q[d] + 3 : (q[d] + 3) / 2 + 1;
                            for (int v = lo; v <= hi; ++v) {
                                if (!restrict_ && abs(2 * v - q[d]) > 3) continue;
                                int w = v;
                                if (gin->bc[d] == AX_PERIODIC) w = ((w % gin->n[d]) + gin->n[d]) % gin->n[d];
                                if (w < uin->lo[ca][d] || w > uin->hi[ca][d] || w % m[d] != o[d]) continue;
                                if (t[d] != INT32_MIN && t[d] != w) { st = ORC_EINVAL; break; }
                                t[d] = w;
                            }
                        }
                        if (st) break;
                        if (t[0] == INT32_MIN || t[1] == INT32_MIN || t[2] == INT32_MIN) { st = ORC_EINVAL; break; }
                        if (nt == cap) {
                            cap *= 2;
                            trip_t *T2 = (trip_t *)realloc(T, sizeof(trip_t) * cap);
                            if (!T2) { st = ORC_ENOMEM; break; }
                            T = T2;
                        }
                        T[nt].r = r;
                        T[nt].c = umap_index(uin, ca, t);
                        T[nt].v = out[r];
                        ++nt;
                    }
                }
    free(in);
    free(out);
    if (st) { free(T); return st; }
    qsort(T, nt, sizeof(trip_t), trip_cmp);
    M->nrow = nout;
    M->nnz = nt;
    M->rowptr = (long *)calloc(nout + 1, sizeof(long));
    M->col = (long *)malloc(sizeof(long) * (nt ? nt : 1));
    M->val = (double *)malloc(sizeof(double) * (nt ? nt : 1));
    if (!M->rowptr || !M->col || !M->val) { free(T); return ORC_ENOMEM; }
    for (long t = 0; t < nt; ++t) {
        M->rowptr[T[t].r + 1]++;
        M->col[t] = T[t].c;
        M->val[t] = T[t].v;
    }
    for (long r = 0; r < nout; ++r) M->rowptr[r + 1] += M->rowptr[r];
    free(T);
    return ORC_OK;
}

/* viscous operator of level l >= 1 as R_{l-1} (A_{l-1} P_{l-1}) */
static int galerkin_level(hier_t *H, int l)
{
    csr_t R = {0}, P = {0}, AP = {0};
    long nc = umap_total(&H->lv[l].uu);
    int st = probe_transfer(H, l - 1, 1, &R);
    if (!st) st = probe_transfer(H, l - 1, 0, &P);
    if (!st) st = csr_mul(&H->lv[l - 1].Au, &P, nc, &AP);
    if (!st) st = csr_mul(&R, &AP, nc, &H->lv[l].Au);
    csr_free(&R);
    csr_free(&P);
    csr_free(&AP);
    return st;
}

/* A red-black sweep on a Galerkin level.  R A P couples points of one
 * colour, so the rows of each (component, colour) set are all updated from
 * the values the set had before its pass: Jacobi within a set, Gauss-Seidel
 * from set to set, in the order of gs_sweep.  Where no two rows of a set
 * couple (every rediscretised level) this is gs_sweep itself. */
static void gs_sweep_sets(const csr_t *A, const umap_t *u, const double *b, double *x)
{
    long n = A->nrow;
    double *xn = (double *)malloc(sizeof(double) * (n ? n : 1));
    for (int c = 0; c < u->ncomp; ++c)
        for (int colour = 0; colour < 2; ++colour) {
            for (long r = u->off[c]; r < u->off[c + 1]; ++r) {
                if (row_colour(u, r) != colour) continue;
                double s = b[r], diag = 0.0;
                for (long t = A->rowptr[r]; t < A->rowptr[r + 1]; ++t) {
                    if (A->col[t] == r) diag = A->val[t];
                    else s -= A->val[t] * x[A->col[t]];
                }
                xn[r] = s / diag;
            }
            for (long r = u->off[c]; r < u->off[c + 1]; ++r)
                if (row_colour(u, r) == colour) x[r] = xn[r];
        }
    free(xn);
}

/* one smoothing sweep of level l */
static void smooth_level(hier_t *H, int velocity, int l, const double *b, double *x)
{
    level_t *L = &H->lv[l];
    if (velocity && H->d.galerkin && l > 0) gs_sweep_sets(&L->Au, &L->uu, b, x);
    else gs_sweep(velocity ? &L->Au : &L->Ap, velocity ? &L->uu : &L->up, b, x);
}

/* V(nu1, nu2) cycle on level l (Sec. "Multigrid") */
static void vcycle(hier_t *H, int velocity, int l, const double *b, double *x, double *wu)
{
    level_t *L = &H->lv[l];
    const csr_t *A = velocity ? &L->Au : &L->Ap;
    long n = A->nrow;
    double frac = (double)n / (double)(velocity ? H->lv[0].Au.nrow : H->lv[0].Ap.nrow);
    int singular = !velocity && H->singular_p;
    if (l == H->L - 1) {
        if (n <= DENSE_MAX) {
            dense_solve(A, singular, b, x);
        } else {
            for (int s = 0; s < H->d.nu1 + H->d.nu2; ++s) smooth_level(H, velocity, l, b, x);
            *wu += (H->d.nu1 + H->d.nu2) * frac;
        }
        return;
    }
    for (int s = 0; s < H->d.nu1; ++s) smooth_level(H, velocity, l, b, x);
    double *r = (double *)malloc(sizeof(double) * n);
    residual(A, b, x, r);
    level_t *C = &H->lv[l + 1];
    long nc = velocity ? C->Au.nrow : C->Ap.nrow;
    double *bc = (double *)malloc(sizeof(double) * nc);
    double *xc = (double *)calloc(nc, sizeof(double));
    restrict_residual(H, l, velocity, r, bc);
    vcycle(H, velocity, l + 1, bc, xc, wu);
    prolong_add(H, l, velocity, xc, x);
    for (int s = 0; s < H->d.nu2; ++s) smooth_level(H, velocity, l, b, x);
    *wu += (H->d.nu1 + H->d.nu2) * frac;
    free(r);
    free(bc);
    free(xc);
}

/* compact lattice layout <-> vector of unknowns on level 0 */
static void compact_to_vec(hier_t *H, int velocity, const double *c, double *x)
{
    level_t *L = &H->lv[0];
    const umap_t *u = velocity ? &L->uu : &L->up;
    double *pad[3] = {0, 0, 0};
    long off = 0;
    for (int k = 0; k < u->ncomp; ++k) {
        pad[k] = padded_alloc(&L->g);
        compact_to_padded(&L->g, u->lat[k], c + off, pad[k]);
        off += stored_count(&L->g, u->lat[k]);
    }
    padded_to_vec(&L->g, u, pad, x);
    for (int k = 0; k < u->ncomp; ++k) free(pad[k]);
}

static void vec_to_compact(hier_t *H, int velocity, const double *x, double *c)
{
    /* only the unknown positions of c are written */
    level_t *L = &H->lv[0];
    const umap_t *u = velocity ? &L->uu : &L->up;
    long off[3] = {0, 0, 0};
    for (int k = 1; k < u->ncomp; ++k) off[k] = off[k - 1] + stored_count(&L->g, u->lat[k - 1]);
    long n = umap_total(u);
    for (long r = 0; r < n; ++r) {
        int k, q[3], lo[3], hi[3];
        umap_pos(u, r, &k, q);
        for (int d = 0; d < 3; ++d) stored_range(&L->g, u->lat[k], d, &lo[d], &hi[d]);
        long t = ((long)(q[2] - lo[2]) * (hi[1] - lo[1] + 1) + (q[1] - lo[1])) * (hi[0] - lo[0] + 1) + (q[0] - lo[0]);
        c[off[k] + t] = x[r];
    }
}

/* Iterate V-cycles from the initial guess in x until
 * ||b - A x||_2 <= rtol ||b||_2, checking before the first cycle and after
 * every cycle.  b and x use the compact lattice layout; positions that are
 * not unknowns are ignored in b and left untouched in x. */
int orc_solve(void *hp, int velocity, const double *bc, double *xc, int *cycles, double *relres, double *wu_out,
              double *hist, int hist_len)
{
    hier_t *H = (hier_t *)hp;
    level_t *L = &H->lv[0];
    const csr_t *A = velocity ? &L->Au : &L->Ap;
    long n = A->nrow;
    double *b = (double *)malloc(sizeof(double) * n);
    double *x = (double *)malloc(sizeof(double) * n);
    double *r = (double *)malloc(sizeof(double) * n);
    compact_to_vec(H, velocity, bc, b);
    compact_to_vec(H, velocity, xc, x);
    double nb = norm2(b, n), wu = 0.0;
    int status = ORC_OK, k = 0;
    double rel = 0.0;
    if (nb == 0.0) {
        for (long i = 0; i < n; ++i) x[i] = 0.0;
    } else {
        residual(A, b, x, r);
        rel = norm2(r, n) / nb;
        if (hist && hist_len > 0) hist[0] = rel;
        while (!(rel <= H->d.rtol)) {
            if (rel != rel) { status = ORC_ENUMERIC; break; }
            if (k >= H->d.max_cycles) { status = ORC_ENOCONV; break; }
            vcycle(H, velocity, 0, b, x, &wu);
            wu += 1.0; /* the residual check is one finest-grid pass */
            ++k;
            residual(A, b, x, r);
            rel = norm2(r, n) / nb;
            if (hist && k < hist_len) hist[k] = rel;
        }
    }
    vec_to_compact(H, velocity, x, xc);
    *cycles = k;
    *relres = rel;
    if (wu_out) *wu_out = wu;
    free(b);
    free(x);
    free(r);
    return status;
}

/* Multigrid-preconditioned GCR (generalised conjugate residuals), the
 * Krylov acceleration the paper names as its main future direction for
 * high viscosity contrast.  Each iteration:
 *   z = M r             one V(nu1, nu2) cycle on A z = r from z = 0
 *   q = A z
 *   for the stored directions i (modified Gram-Schmidt):
 *       beta = (q, q_i) / (q_i, q_i);  q -= beta q_i;  z -= beta z_i
 *   alpha = (r, q) / (q, q);  x += alpha z
 *   r = b - A x          (the true residual: same stopping test as orc_solve)
 *   store (z, q); after m directions the store is emptied (restart).
 * The iteration count is capped by max_cycles; kmax > 0 runs exactly kmax
 * iterations without a stopping test. */
static double dot(const double *a, const double *b, long n)
{
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

int orc_solve_gcr(void *hp, int velocity, int m, int kmax, const double *bc, double *xc, int *iters, double *relres)
{
    hier_t *H = (hier_t *)hp;
    const csr_t *A = velocity ? &H->lv[0].Au : &H->lv[0].Ap;
    long n = A->nrow;
    if (m < 1) return ORC_EINVAL;
    double *b = malloc(sizeof(double) * n), *x = malloc(sizeof(double) * n), *r = malloc(sizeof(double) * n);
    double *Z = malloc(sizeof(double) * n * (size_t)m), *Q = malloc(sizeof(double) * n * (size_t)m);
    double *qq = malloc(sizeof(double) * (size_t)m);
    if (!b || !x || !r || !Z || !Q || !qq) { free(b); free(x); free(r); free(Z); free(Q); free(qq); return ORC_ENOMEM; }
    compact_to_vec(H, velocity, bc, b);
    compact_to_vec(H, velocity, xc, x);
    double nb = norm2(b, n), rel = 0.0, wu = 0.0;
    int status = ORC_OK, k = 0, j = 0;
    if (nb == 0.0) {
        for (long i = 0; i < n; ++i) x[i] = 0.0;
    } else {
        residual(A, b, x, r);
        rel = norm2(r, n) / nb;
        for (;;) {
            if (kmax > 0) {
                if (k >= kmax) break;
            } else {
                if (rel <= H->d.rtol) break;
                if (rel != rel) { status = ORC_ENUMERIC; break; }
                if (k >= H->d.max_cycles) { status = ORC_ENOCONV; break; }
            }
            double *z = Z + (size_t)j * n, *q = Q + (size_t)j * n;
            for (long i = 0; i < n; ++i) z[i] = 0.0;
            vcycle(H, velocity, 0, r, z, &wu);
            for (long i = 0; i < n; ++i) {               /* q = A z */
                double s = 0.0;
                for (long t = A->rowptr[i]; t < A->rowptr[i + 1]; ++t) s += A->val[t] * z[A->col[t]];
                q[i] = s;
            }
            for (int i = 0; i < j; ++i) {
                const double *zi = Z + (size_t)i * n, *qi = Q + (size_t)i * n;
                double beta = dot(q, qi, n) / qq[i];
                for (long t = 0; t < n; ++t) {
                    q[t] -= beta * qi[t];
                    z[t] -= beta * zi[t];
                }
            }
            qq[j] = dot(q, q, n);
            double alpha = dot(r, q, n) / qq[j];
            for (long t = 0; t < n; ++t) x[t] += alpha * z[t];
            residual(A, b, x, r);
            rel = norm2(r, n) / nb;
            ++k;
            j = j + 1 == m ? 0 : j + 1;
        }
    }
    vec_to_compact(H, velocity, x, xc);
    *iters = k;
    *relres = rel;
    free(b); free(x); free(r); free(Z); free(Q); free(qq);
    return status;
}

/* exactly k V-cycles from the initial guess (iterate-level comparisons) */
int orc_vcycles(void *hp, int velocity, const double *bc, double *xc, int k)
{
    hier_t *H = (hier_t *)hp;
    const csr_t *A = velocity ? &H->lv[0].Au : &H->lv[0].Ap;
    long n = A->nrow;
    double *b = (double *)malloc(sizeof(double) * n);
    double *x = (double *)malloc(sizeof(double) * n);
    compact_to_vec(H, velocity, bc, b);
    compact_to_vec(H, velocity, xc, x);
    double wu = 0.0;
    for (int i = 0; i < k; ++i) vcycle(H, velocity, 0, b, x, &wu);
    vec_to_compact(H, velocity, x, xc);
    free(b);
    free(x);
    return ORC_OK;
}

/* exactly k smoothing sweeps on level 0 */
int orc_smooth(void *hp, int velocity, const double *bc, double *xc, int k)
{
    hier_t *H = (hier_t *)hp;
    level_t *L = &H->lv[0];
    const csr_t *A = velocity ? &L->Au : &L->Ap;
    long n = A->nrow;
    double *b = (double *)malloc(sizeof(double) * n);
    double *x = (double *)malloc(sizeof(double) * n);
    compact_to_vec(H, velocity, bc, b);
    compact_to_vec(H, velocity, xc, x);
    for (int i = 0; i < k; ++i) gs_sweep(A, velocity ? &L->uu : &L->up, b, x);
    vec_to_compact(H, velocity, x, xc);
    free(b);
    free(x);
    return ORC_OK;
}

/* exactly k smoothing sweeps of level l on vectors of that level's
 * unknowns (the smoother the V-cycle uses there) */
int orc_smooth_level(void *hp, int velocity, int level, const double *b, double *x, int k)
{
    hier_t *H = (hier_t *)hp;
    if (level < 0 || level >= H->L) return ORC_EINVAL;
    for (int i = 0; i < k; ++i) smooth_level(H, velocity, level, b, x);
    return ORC_OK;
}

/* relative residual ||b - A x|| / ||b|| of a compact-layout pair on level 0 */
double orc_relres(void *hp, int velocity, const double *bc, const double *xc)
{
    hier_t *H = (hier_t *)hp;
    const csr_t *A = velocity ? &H->lv[0].Au : &H->lv[0].Ap;
    long n = A->nrow;
    double *b = (double *)malloc(sizeof(double) * n);
    double *x = (double *)malloc(sizeof(double) * n);
    double *r = (double *)malloc(sizeof(double) * n);
    compact_to_vec(H, velocity, bc, b);
    compact_to_vec(H, velocity, xc, x);
    residual(A, b, x, r);
    double nb = norm2(b, n);
    double rel = nb > 0 ? norm2(r, n) / nb : norm2(r, n);
    free(b);
    free(x);
    free(r);
    return rel;
}

/* ------------------------------------------------------------------ */
/* matrix export and matrix-free application (for the tests)           */
/* ------------------------------------------------------------------ */
long orc_csr_nnz(void *hp, int velocity, int level)
{
    hier_t *H = (hier_t *)hp;
    return velocity ? H->lv[level].Au.nnz : H->lv[level].Ap.nnz;
}

long orc_csr_export(void *hp, int velocity, int level, long *rowptr, long *col, double *val)
{
    hier_t *H = (hier_t *)hp;
    const csr_t *A = velocity ? &H->lv[level].Au : &H->lv[level].Ap;
    memcpy(rowptr, A->rowptr, sizeof(long) * (A->nrow + 1));
    memcpy(col, A->col, sizeof(long) * A->nnz);
    memcpy(val, A->val, sizeof(double) * A->nnz);
    return A->nrow;
}

/* unknown positions of level l: comp and (i,j,k) per row */
int orc_unknowns(void *hp, int velocity, int level, int *comp, int *pos)
{
    hier_t *H = (hier_t *)hp;
    const umap_t *u = velocity ? &H->lv[level].uu : &H->lv[level].up;
    long n = umap_total(u);
    for (long r = 0; r < n; ++r) {
        int c, q[3];
        umap_pos(u, r, &c, q);
        comp[r] = c;
        pos[3 * r] = q[0];
        pos[3 * r + 1] = q[1];
        pos[3 * r + 2] = q[2];
    }
    return ORC_OK;
}

/* apply the operator of level l to a vector of unknowns directly through
 * the stencil (no matrix), y = A x */
int orc_apply_vec(void *hp, int velocity, int level, const double *x, double *y)
{
    hier_t *H = (hier_t *)hp;
    level_t *L = &H->lv[level];
    const umap_t *u = velocity ? &L->uu : &L->up;
    double *pad[3] = {0, 0, 0};
    for (int c = 0; c < u->ncomp; ++c) pad[c] = padded_alloc(&L->g);
    vec_to_padded(&L->g, u, x, pad, velocity);
    long n = umap_total(u);
    for (long r = 0; r < n; ++r) {
        int c, q[3];
        umap_pos(u, r, &c, q);
        y[r] = velocity ? apply_u_at(L, &H->d, pad, c, q) : apply_p_at(L, pad[0], q);
    }
    for (int c = 0; c < u->ncomp; ++c) free(pad[c]);
    return ORC_OK;
}

/* restriction / prolongation of unknown vectors between levels l and l+1 */
int orc_restrict_vec(void *hp, int velocity, int level, const double *r, double *bc)
{
    restrict_residual((hier_t *)hp, level, velocity, r, bc);
    return ORC_OK;
}

int orc_prolong_vec(void *hp, int velocity, int level, const double *xc, double *x)
{
    prolong_add((hier_t *)hp, level, velocity, xc, x);
    return ORC_OK;
}

/* coefficient arrays of level l in compact layout (rho faces, mu cells, mu edges) */
int orc_level_coefs(void *hp, int level, double *rho_faces, double *mu_c, double *mu_e)
{
    hier_t *H = (hier_t *)hp;
    level_t *L = &H->lv[level];
    long off = 0;
    for (int a = 0; a < L->g.D; ++a) {
        padded_to_compact(&L->g, face_lat(a), L->rho[a], rho_faces + off);
        off += stored_count(&L->g, face_lat(a));
    }
    padded_to_compact(&L->g, cell_lat(), L->mu_c, mu_c);
    off = 0;
    for (int c = edge_first(L->g.D); c < 3; ++c) {
        padded_to_compact(&L->g, edge_lat(c), L->mu_e[c], mu_e + off);
        off += stored_count(&L->g, edge_lat(c));
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* compact lattice sizes                                               */
/* ------------------------------------------------------------------ */
/* kind: 0 cell, 1 face (axis), 2 edge (axis) */
long orc_lattice_count(const orc_desc *d, int kind, int axis, int *dims)
{
    grid_t g;
    grid_init(&g, d->dim, d->n, d->axis_bc, d->h);
    lat_t L = {kind, axis};
    for (int a = 0; a < 3; ++a) {
        int lo, hi;
        stored_range(&g, L, a, &lo, &hi);
        dims[a] = hi - lo + 1;
    }
    return stored_count(&g, L);
}

/* ------------------------------------------------------------------ */
/* immersed boundary: spread, viscosity, interpolation                 */
/* ------------------------------------------------------------------ */
static int check_period(const grid_t *g, double width)
{
    for (int d = 0; d < g->D; ++d)
        if (g->bc[d] == AX_PERIODIC && 4.0 * width > g->n[d] * g->h) return ORC_EINVAL;
    return ORC_OK;
}


/* Closed-domain points of lattice L inside the support of delta~(x - X, w):
 * the padded index of each point (after periodic wrapping) and its weight
 * delta~ = w^-D prod_d phi((x_d - X_d) / w).  Points outside a non-periodic
 * domain are dropped (they neither receive nor contribute). */
typedef struct { long *idx; double *w; long n, cap; } support_t;

static int support_of(const grid_t *g, lat_t L, int kernel, double width, const double X[3], support_t *S)
{
    int qlo[3], qhi[3];
    for (int d = 0; d < 3; ++d) {
        if (d >= g->D) { qlo[d] = qhi[d] = 0; continue; }
        double off = is_vert(L, d) ? 0.0 : 0.5;
        qlo[d] = (int)floor((X[d] - 2.0 * width) / g->h - off) - 1;
        qhi[d] = (int)ceil((X[d] + 2.0 * width) / g->h - off) + 1;
    }
    S->n = 0;
    double scale = 1.0;
    for (int d = 0; d < g->D; ++d) scale /= width;
    for (int k = qlo[2]; k <= qhi[2]; ++k)
        for (int j = qlo[1]; j <= qhi[1]; ++j)
            for (int i = qlo[0]; i <= qhi[0]; ++i) {
                int q[3] = {i, j, k}, qs[3] = {0, 0, 0};
                double w = scale;
                int keep = 1;
                for (int d = 0; d < g->D; ++d) {
                    double r = (coord(g, L, d, q[d]) - X[d]) / width;
                    if (!(fabs(r) < 2.0)) { keep = 0; break; }
                    int lo, hi;
                    stored_range(g, L, d, &lo, &hi);
                    int t = q[d];
                    if (g->bc[d] == AX_PERIODIC) t = ((t % g->n[d]) + g->n[d]) % g->n[d];
                    else if (t < lo || t > hi) { keep = 0; break; }
                    qs[d] = t;
                    w *= phi(kernel, r);
                }
                if (!keep) continue;
                if (S->n == S->cap) {
                    S->cap = S->cap ? 2 * S->cap : 256;
                    S->idx = (long *)realloc(S->idx, sizeof(long) * S->cap);
                    S->w = (double *)realloc(S->w, sizeof(double) * S->cap);
                    if (!S->idx || !S->w) return ORC_ENOMEM;
                }
                S->idx[S->n] = P3(g, qs);
                S->w[S->n] = w;
                S->n++;
            }
    return ORC_OK;
}

static void node_pos(const double *X, long eta, long s, int D, double out[3])
{
    for (int d = 0; d < 3; ++d) out[d] = d < D ? X[d * eta + s] : 0.0;
}

/* lattice selector for the compact concatenations used at the interface:
 * velocity-like fields list the D face lattices; edge fields list the edge
 * lattices (3D: parallel to x, y, z; 2D: corners) */
static int lattices_of(int D, int which, lat_t *Ls)
{
    if (which == 0) { for (int a = 0; a < D; ++a) Ls[a] = face_lat(a); return D; }
    if (which == 1) { Ls[0] = cell_lat(); return 1; }
    int n = 0;
    for (int c = edge_first(D); c < 3; ++c) Ls[n++] = edge_lat(c);
    return n;
}

/* Spread a node vector onto the face lattices with width w:
 * out_a(x) = sum_s F_a(s) delta~(x - X_s, w)   (eq:discrForceCouple). */
int orc_spread_vec(const orc_desc *d, double width, long eta, const double *X, const double *F, double *out)
{
    grid_t g;
    grid_init(&g, d->dim, d->n, d->axis_bc, d->h);
    if (check_period(&g, width)) return ORC_EINVAL;
    support_t S = {0, 0, 0, 0};
    long off = 0;
    double *pad = padded_alloc(&g);
    for (int a = 0; a < d->dim; ++a) {
        lat_t L = face_lat(a);
        memset(pad, 0, sizeof(double) * g.size);
        for (long s = 0; s < eta; ++s) {
            double Xs[3];
            node_pos(X, eta, s, d->dim, Xs);
            if (support_of(&g, L, d->kernel, width, Xs, &S)) return ORC_ENOMEM;
            for (long t = 0; t < S.n; ++t) pad[S.idx[t]] += F[a * eta + s] * S.w[t];
        }
        padded_to_compact(&g, L, pad, out + off);
        off += stored_count(&g, L);
    }
    free(pad);
    free(S.idx);
    free(S.w);
    return ORC_OK;
}

/* Interpolate face fields to nodes with width w:
 * U_a(s) = sum_x u_a(x) delta~(x - X_s, w) h^D   (eq:discrVelCouple).
 * The sum runs over closed-domain points; fixed boundary faces contribute
 * the values they hold. */
int orc_interp_vec(const orc_desc *d, double width, long eta, const double *X, const double *u, double *U)
{
    grid_t g;
    grid_init(&g, d->dim, d->n, d->axis_bc, d->h);
    if (check_period(&g, width)) return ORC_EINVAL;
    support_t S = {0, 0, 0, 0};
    double hD = 1.0;
    for (int a = 0; a < d->dim; ++a) hD *= d->h;
    long off = 0;
    double *pad = padded_alloc(&g);
    for (int a = 0; a < d->dim; ++a) {
        lat_t L = face_lat(a);
        compact_to_padded(&g, L, u + off, pad);
        for (long s = 0; s < eta; ++s) {
            double Xs[3];
            node_pos(X, eta, s, d->dim, Xs);
            if (support_of(&g, L, d->kernel, width, Xs, &S)) return ORC_ENOMEM;
            double acc = 0.0;
            for (long t = 0; t < S.n; ++t) acc += pad[S.idx[t]] * S.w[t];
            U[a * eta + s] = acc * hD;
        }
        off += stored_count(&g, L);
    }
    free(pad);
    free(S.idx);
    free(S.w);
    return ORC_OK;
}

/* Density on the face lattices, eq:discrDensCouple:
 * rho_a(x) = rho0 + sum_s rho_b delta~(x - X_s, omega) d0^D. */
int orc_density(const orc_desc *d, long eta, const double *X, double *rho_faces)
{
    grid_t g;
    grid_init(&g, d->dim, d->n, d->axis_bc, d->h);
    if (check_period(&g, d->omega)) return ORC_EINVAL;
    support_t S = {0, 0, 0, 0};
    long off = 0;
    double *pad = padded_alloc(&g);
    for (int a = 0; a < d->dim; ++a) {
        lat_t L = face_lat(a);
        memset(pad, 0, sizeof(double) * g.size);
        for (long s = 0; s < eta; ++s) {
            double Xs[3];
            node_pos(X, eta, s, d->dim, Xs);
            if (support_of(&g, L, d->kernel, d->omega, Xs, &S)) return ORC_ENOMEM;
            for (long t = 0; t < S.n; ++t) pad[S.idx[t]] += d->rho_b * S.w[t] * d->d0_pow_d;
        }
        long cnt = stored_count(&g, L);
        padded_to_compact(&g, L, pad, rho_faces + off);
        for (long t = 0; t < cnt; ++t) rho_faces[off + t] = d->rho0 + rho_faces[off + t];
        off += cnt;
    }
    free(pad);
    free(S.idx);
    free(S.w);
    return ORC_OK;
}

/* Viscosity, eq:ViscExp: mu(x) = max_s [(2 omega)^D (mu_max - mu_out)
 * delta~(x - X_s, omega) + mu_out]; points reached by no node hold mu_out.
 * which = 1: cell centres; which = 2: the edge lattices. */
int orc_viscosity(const orc_desc *d, int which, long eta, const double *X, double *mu)
{
    grid_t g;
    grid_init(&g, d->dim, d->n, d->axis_bc, d->h);
    if (check_period(&g, d->omega)) return ORC_EINVAL;
    lat_t Ls[3];
    int nl = lattices_of(d->dim, which, Ls);
    double scale = 1.0;
    for (int a = 0; a < d->dim; ++a) scale *= 2.0 * d->omega;
    support_t S = {0, 0, 0, 0};
    long off = 0;
    double *pad = padded_alloc(&g);
    for (int l = 0; l < nl; ++l) {
        for (long t = 0; t < g.size; ++t) pad[t] = d->mu_out;
        for (long s = 0; s < eta; ++s) {
            double Xs[3];
            node_pos(X, eta, s, d->dim, Xs);
            if (support_of(&g, Ls[l], d->kernel, d->omega, Xs, &S)) return ORC_ENOMEM;
            for (long t = 0; t < S.n; ++t) {
                double cand = scale * (d->mu_max - d->mu_out) * S.w[t] + d->mu_out;
                if (cand > pad[S.idx[t]]) pad[S.idx[t]] = cand;
            }
        }
        padded_to_compact(&g, Ls[l], pad, mu + off);
        off += stored_count(&g, Ls[l]);
    }
    free(pad);
    free(S.idx);
    free(S.w);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* springs: breakage then Hookean force (eq:springF, eq:defineK)       */
/* ------------------------------------------------------------------ */
/* separation X_j - X_i, nearest image along periodic axes */
static void separation(const orc_desc *d, const double *X, long eta, long i, long j, double out[3])
{
    for (int a = 0; a < 3; ++a) {
        out[a] = 0.0;
        if (a >= d->dim) continue;
        double v = X[a * eta + j] - X[a * eta + i];
        if (d->axis_bc[a] == AX_PERIODIC) {
            double Lx = d->n[a] * d->h;
            v -= Lx * floor(v / Lx + 0.5);
        }
        out[a] = v;
    }
}

/* alive springs whose squared length exceeds (break_ratio * rest)^2 are
 * removed for good; the force on node s is the sum over its surviving
 * springs of K (l - r) times the unit vector from s to its partner */
int orc_springs(const orc_desc *d, long eta, const double *X, long m, const int *ij, const double *rest, const double *K,
                unsigned char *alive, double *F, int do_break, long *n_broken)
{
    long nb = 0;
    for (long t = 0; t < d->dim * eta; ++t) F[t] = 0.0;
    for (long e = 0; e < m; ++e) {
        long i = ij[e], j = ij[m + e];
        double v[3];
        separation(d, X, eta, i, j, v);
        double l2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        double lim = d->break_ratio * rest[e];
        if (do_break && alive[e] && l2 > lim * lim) { alive[e] = 0; ++nb; }
    }
    for (long e = 0; e < m; ++e) {
        if (!alive[e]) continue;
        long i = ij[e], j = ij[m + e];
        double v[3];
        separation(d, X, eta, i, j, v);
        double l = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (l == 0.0) continue;
        double T = K[e] * (l - rest[e]);
        for (int a = 0; a < d->dim; ++a) {
            F[a * eta + i] += T * v[a] / l;
            F[a * eta + j] -= T * v[a] / l;
        }
    }
    if (n_broken) *n_broken = nb;
    return ORC_OK;
}

/* Detached fragments (the "break off" observation of the results section;
 * the paper gives no algorithm): the fragments are the connected components
 * of the graph whose vertices are the nodes and whose edges are the alive
 * springs.  Each fragment is labelled by its smallest node id.  A fragment is
 * detached when none of its nodes was anchored (within the attachment
 * distance of the attachment wall at t = 0).
 *
 * Plain breadth-first search from every unvisited node in increasing id
 * order: the node a search starts from is the smallest id of its component,
 * because every smaller id was visited by an earlier search. */
int orc_fragments(long eta, long m, const int *ij, const unsigned char *alive, const unsigned char *anchored,
                  int *label, long *n_fragments, long *n_detached)
{
    long *deg = calloc((size_t)eta + 1, sizeof(long));
    long *adj = malloc(sizeof(long) * (size_t)(2 * m + 1));
    long *fill = calloc((size_t)eta + 1, sizeof(long));
    long *queue = malloc(sizeof(long) * (size_t)(eta + 1));
    if (!deg || !adj || !fill || !queue) { free(deg); free(adj); free(fill); free(queue); return ORC_ENOMEM; }
    for (long e = 0; e < m; ++e)
        if (alive[e]) { deg[ij[e] + 1]++; deg[ij[m + e] + 1]++; }
    for (long s = 0; s < eta; ++s) deg[s + 1] += deg[s];          /* row starts */
    for (long e = 0; e < m; ++e) {
        if (!alive[e]) continue;
        long i = ij[e], j = ij[m + e];
        adj[deg[i] + fill[i]++] = j;
        adj[deg[j] + fill[j]++] = i;
    }
    for (long s = 0; s < eta; ++s) label[s] = -1;
    long nf = 0, nd = 0;
    for (long s = 0; s < eta; ++s) {
        if (label[s] >= 0) continue;
        long head = 0, tail = 0;
        int anchored_any = 0;
        label[s] = (int)s;
        queue[tail++] = s;
        while (head < tail) {
            long v = queue[head++];
            if (anchored[v]) anchored_any = 1;
            for (long k = deg[v]; k < deg[v + 1]; ++k) {
                long w = adj[k];
                if (label[w] < 0) { label[w] = (int)s; queue[tail++] = w; }
            }
        }
        ++nf;
        if (!anchored_any) ++nd;
    }
    free(deg); free(adj); free(fill); free(queue);
    *n_fragments = nf;
    *n_detached = nd;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* projection-step pieces on the finest grid                           */
/* ------------------------------------------------------------------ */
typedef struct {
    grid_t g;
    double *u[3];    /* ROLE_VELFULL padded velocity */
    double *rho[3];  /* ROLE_COEF padded density */
    double *mu_c, *mu_e[3];
} fine_t;

static void fine_free(fine_t *F)
{
    for (int a = 0; a < 3; ++a) { free(F->u[a]); free(F->rho[a]); free(F->mu_e[a]); }
    free(F->mu_c);
}

static void load_faces(const grid_t *g, const double *c, int role, double **pad)
{
    long off = 0;
    for (int a = 0; a < g->D; ++a) {
        pad[a] = padded_alloc(g);
        compact_to_padded(g, face_lat(a), c + off, pad[a]);
        fill_ghosts(g, face_lat(a), role, pad[a]);
        off += stored_count(g, face_lat(a));
    }
}

/* the skew-symmetric advection term of eq:NSdis1-1 at an a-face:
 * N_a = 1/2 sum_b [ ub_b D0_b u_a + D0_b (ub_b u_a) ], where ub_b is u_b
 * averaged to the a-face positions (four surrounding b-faces, or u_a itself
 * for b = a) and D0_b the central difference over 2h */
static double ubar(const grid_t *g, double *const *u, int a, int b, const int p[3])
{
    if (b == a) return u[a][P3(g, p)];
    int q1[3] = {p[0], p[1], p[2]}, q2[3], q3[3], q4[3];
    memcpy(q2, q1, sizeof q1);
    q2[b] += 1;
    memcpy(q3, q1, sizeof q1);
    q3[a] -= 1;
    memcpy(q4, q2, sizeof q1);
    q4[a] -= 1;
    return 0.25 * (u[b][P3(g, q1)] + u[b][P3(g, q2)] + u[b][P3(g, q3)] + u[b][P3(g, q4)]);
}

static double advection_at(const grid_t *g, double *const *u, int a, const int q[3])
{
    double s = 0.0;
    for (int b = 0; b < g->D; ++b) {
        int qp[3] = {q[0], q[1], q[2]}, qm[3] = {q[0], q[1], q[2]};
        qp[b] += 1;
        qm[b] -= 1;
        double uap = u[a][P3(g, qp)], uam = u[a][P3(g, qm)];
        double bc = ubar(g, u, a, b, q), bp = ubar(g, u, a, b, qp), bm = ubar(g, u, a, b, qm);
        s += bc * (uap - uam) / (2.0 * g->h) + (bp * uap - bm * uam) / (2.0 * g->h);
    }
    return 0.5 * s;
}

/* Right-hand side of the viscous system (eq:NSdis1-1 rearranged):
 * b_a = rho_a (sigma u_a / dt - N_a(u)) + C_f f_a + g_a + Re^-1 V(u_bd)_a,
 * where u_bd holds only the fixed boundary values (so that the matrix acts
 * on the unknowns alone).  All arrays in compact layout; b is written at
 * unknown positions only. */
int orc_momentum_rhs(const orc_desc *d, const double *u, const double *rho_faces, const double *mu_c,
                     const double *mu_e, const double *f, double *b, int with_boundary)
{
    level_t L;
    grid_t g;
    grid_init(&g, d->dim, d->n, d->axis_bc, d->h);
    if (level_alloc(&L, &g)) return ORC_ENOMEM;
    long off = 0;
    for (int a = 0; a < d->dim; ++a) {
        compact_to_padded(&g, face_lat(a), rho_faces + off, L.rho[a]);
        fill_ghosts(&g, face_lat(a), ROLE_COEF, L.rho[a]);
        off += stored_count(&g, face_lat(a));
    }
    compact_to_padded(&g, cell_lat(), mu_c, L.mu_c);
    fill_ghosts(&g, cell_lat(), ROLE_COEF, L.mu_c);
    off = 0;
    for (int c = edge_first(d->dim); c < 3; ++c) {
        compact_to_padded(&g, edge_lat(c), mu_e + off, L.mu_e[c]);
        fill_ghosts(&g, edge_lat(c), ROLE_COEF, L.mu_e[c]);
        off += stored_count(&g, edge_lat(c));
    }
    double *uf[3] = {0, 0, 0}, *ff[3] = {0, 0, 0}, *ubd[3] = {0, 0, 0};
    load_faces(&g, u, ROLE_VELFULL, uf);
    load_faces(&g, f, ROLE_COEF, ff);
    /* boundary-only copy: zero at every unknown, boundary values kept */
    for (int a = 0; a < d->dim; ++a) {
        ubd[a] = padded_alloc(&g);
        memcpy(ubd[a], uf[a], sizeof(double) * g.size);
        int lo[3], hi[3];
        for (int e = 0; e < 3; ++e) unknown_range(&g, face_lat(a), e, &lo[e], &hi[e]);
        for (int k = lo[2]; k <= hi[2]; ++k)
            for (int j = lo[1]; j <= hi[1]; ++j)
                for (int i = lo[0]; i <= hi[0]; ++i) ubd[a][Pijk(&g, i, j, k)] = 0.0;
    }
    for (int a = 0; a < d->dim; ++a) fill_ghosts(&g, face_lat(a), ROLE_VELFULL, ubd[a]);
    off = 0;
    for (int a = 0; a < d->dim; ++a) {
        lat_t La = face_lat(a);
        int lo[3], hi[3], so[3], sh[3];
        for (int e = 0; e < 3; ++e) {
            unknown_range(&g, La, e, &lo[e], &hi[e]);
            stored_range(&g, La, e, &so[e], &sh[e]);
        }
        for (int k = lo[2]; k <= hi[2]; ++k)
            for (int j = lo[1]; j <= hi[1]; ++j)
                for (int i = lo[0]; i <= hi[0]; ++i) {
                    int q[3] = {i, j, k};
                    long p = P3(&g, q);
                    double N = advection_at(&g, uf, a, q);
                    double v = L.rho[a][p] * (d->sigma * uf[a][p] / d->dt - N) + d->force_coef * ff[a][p] +
                               d->body_force[a];
                    if (with_boundary) v += d->inv_re * visc_at(&L, ubd, a, q);
                    long t = ((long)(k - so[2]) * (sh[1] - so[1] + 1) + (j - so[1])) * (sh[0] - so[0] + 1) + (i - so[0]);
                    b[off + t] = v;
                }
        off += stored_count(&g, La);
    }
    for (int a = 0; a < 3; ++a) { free(uf[a]); free(ff[a]); free(ubd[a]); }
    level_free(&L);
    return ORC_OK;
}

/* the viscous operator applied to a full velocity field in compact layout,
 * boundary values included: y_a = (sigma rho_a / dt) u_a - Re^-1 V(u)_a at
 * every unknown face (used to check the split into matrix and boundary
 * terms) */
int orc_momentum_apply_full(const orc_desc *d, const double *u, const double *rho_faces, const double *mu_c,
                            const double *mu_e, double *y)
{
    level_t L;
    grid_t g;
    grid_init(&g, d->dim, d->n, d->axis_bc, d->h);
    if (level_alloc(&L, &g)) return ORC_ENOMEM;
    long off = 0;
    for (int a = 0; a < d->dim; ++a) {
        compact_to_padded(&g, face_lat(a), rho_faces + off, L.rho[a]);
        fill_ghosts(&g, face_lat(a), ROLE_COEF, L.rho[a]);
        off += stored_count(&g, face_lat(a));
    }
    compact_to_padded(&g, cell_lat(), mu_c, L.mu_c);
    fill_ghosts(&g, cell_lat(), ROLE_COEF, L.mu_c);
    off = 0;
    for (int c = edge_first(d->dim); c < 3; ++c) {
        compact_to_padded(&g, edge_lat(c), mu_e + off, L.mu_e[c]);
        fill_ghosts(&g, edge_lat(c), ROLE_COEF, L.mu_e[c]);
        off += stored_count(&g, edge_lat(c));
    }
    double *uf[3] = {0, 0, 0};
    load_faces(&g, u, ROLE_VELFULL, uf);
    off = 0;
    for (int a = 0; a < d->dim; ++a) {
        lat_t La = face_lat(a);
        int lo[3], hi[3], so[3], sh[3];
        for (int e = 0; e < 3; ++e) {
            unknown_range(&g, La, e, &lo[e], &hi[e]);
            stored_range(&g, La, e, &so[e], &sh[e]);
        }
        for (int k = lo[2]; k <= hi[2]; ++k)
            for (int j = lo[1]; j <= hi[1]; ++j)
                for (int i = lo[0]; i <= hi[0]; ++i) {
                    int q[3] = {i, j, k};
                    long t = ((long)(k - so[2]) * (sh[1] - so[1] + 1) + (j - so[1])) * (sh[0] - so[0] + 1) + (i - so[0]);
                    y[off + t] = apply_u_at(&L, d, uf, a, q);
                }
        off += stored_count(&g, La);
    }
    for (int a = 0; a < 3; ++a) free(uf[a]);
    level_free(&L);
    return ORC_OK;
}

/* Right-hand side of the pressure system, eq:NSdis4 with A_p = -D(beta G):
 * b_p = -(sigma / (eps dt)) D u~, with the mean removed when the system is
 * singular (no outflow face). */
int orc_pressure_rhs(const orc_desc *d, const double *ut, double *bp)
{
    grid_t g;
    grid_init(&g, d->dim, d->n, d->axis_bc, d->h);
    double *uf[3] = {0, 0, 0};
    load_faces(&g, ut, ROLE_VELFULL, uf);
    int singular = 1;
    for (int a = 0; a < d->dim; ++a)
        if (d->axis_bc[a] == AX_INOUT) singular = 0;
    double c = -d->sigma / (d->eps * d->dt);
    long t = 0;
    double mean = 0.0;
    for (int k = 0; k < g.n[2]; ++k)
        for (int j = 0; j < g.n[1]; ++j)
            for (int i = 0; i < g.n[0]; ++i) {
                int q[3] = {i, j, k};
                double div = 0.0;
                for (int a = 0; a < d->dim; ++a) {
                    int qp[3] = {i, j, k};
                    qp[a] += 1;
                    div += (uf[a][P3(&g, qp)] - uf[a][P3(&g, q)]) / d->h;
                }
                bp[t] = c * div;
                mean += bp[t];
                ++t;
            }
    if (singular) {
        mean /= (double)t;
        for (long s = 0; s < t; ++s) bp[s] -= mean;
    }
    for (int a = 0; a < 3; ++a) free(uf[a]);
    return ORC_OK;
}

/* discrete divergence D u at cell centres (compact), boundary values kept */
int orc_divergence(const orc_desc *d, const double *u, double *div)
{
    grid_t g;
    grid_init(&g, d->dim, d->n, d->axis_bc, d->h);
    double *uf[3] = {0, 0, 0};
    load_faces(&g, u, ROLE_VELFULL, uf);
    long t = 0;
    for (int k = 0; k < g.n[2]; ++k)
        for (int j = 0; j < g.n[1]; ++j)
            for (int i = 0; i < g.n[0]; ++i) {
                int q[3] = {i, j, k};
                double s = 0.0;
                for (int a = 0; a < d->dim; ++a) {
                    int qp[3] = {i, j, k};
                    qp[a] += 1;
                    s += (uf[a][P3(&g, qp)] - uf[a][P3(&g, q)]) / d->h;
                }
                div[t++] = s;
            }
    for (int a = 0; a < 3; ++a) free(uf[a]);
    return ORC_OK;
}

/* Projection, eq:NSdis2: u_a = u~_a - (eps dt / sigma) beta_a G_a p at every
 * unknown face; fixed faces keep their values. */
int orc_project(const orc_desc *d, const double *ut, const double *p, const double *rho_faces, double *u)
{
    grid_t g;
    grid_init(&g, d->dim, d->n, d->axis_bc, d->h);
    double *pp = padded_alloc(&g);
    compact_to_padded(&g, cell_lat(), p, pp);
    fill_ghosts(&g, cell_lat(), ROLE_PRES, pp);
    double c = d->eps * d->dt / d->sigma;
    long off = 0;
    for (int a = 0; a < d->dim; ++a) {
        lat_t La = face_lat(a);
        long cnt = stored_count(&g, La);
        memcpy(u + off, ut + off, sizeof(double) * cnt);
        double *rho = padded_alloc(&g);
        compact_to_padded(&g, La, rho_faces + off, rho);
        int lo[3], hi[3], so[3], sh[3];
        for (int e = 0; e < 3; ++e) {
            unknown_range(&g, La, e, &lo[e], &hi[e]);
            stored_range(&g, La, e, &so[e], &sh[e]);
        }
        for (int k = lo[2]; k <= hi[2]; ++k)
            for (int j = lo[1]; j <= hi[1]; ++j)
                for (int i = lo[0]; i <= hi[0]; ++i) {
                    int q[3] = {i, j, k}, qm[3] = {i, j, k};
                    qm[a] -= 1;
                    long t = ((long)(k - so[2]) * (sh[1] - so[1] + 1) + (j - so[1])) * (sh[0] - so[0] + 1) + (i - so[0]);
                    double grad = (pp[P3(&g, q)] - pp[P3(&g, qm)]) / d->h;
                    u[off + t] = ut[off + t] - c * grad / rho[P3(&g, q)];
                }
        free(rho);
        off += cnt;
    }
    free(pp);
    return ORC_OK;
}
