// Argument bundles and host launchers of the library's kernels.
#pragma once

#include <hip/hip_ext.h>

#include "common.h"

namespace ibmg {

// grid-stride reductions use at most NORM_BLOCKS blocks per component, or
// on large lattices as many as keep about 16 points per thread, up to
// NORM_BLOCKS_MAX (per-thread loops are latency-bound once they grow long)
constexpr unsigned NORM_BLOCKS = 1024;
constexpr unsigned NORM_BLOCKS_MAX = 8192;

// a box of lattice positions: lo[d] .. lo[d] + ext[d] - 1
struct Box {
    int lo[3];
    int ext[3];
};
struct VelBox {
    Box b[3];
};

// unknown boxes and their colour classes
__host__ __device__ inline Box unk_box(const Grid &g, int vmask)
{
    Box b;
    for (int d = 0; d < 3; ++d) {
        int lo, hi;
        unk_range(g, d, (vmask >> d) & 1, lo, hi);
        b.lo[d] = lo;
        b.ext[d] = hi - lo + 1;
    }
    return b;
}

__host__ __device__ inline bool box_pos(const Box &b, int t, int &i, int &j, int &k)
{
    const int n = b.ext[0] * b.ext[1] * b.ext[2];
    if (t >= n) return false;
    i = b.lo[0] + t % b.ext[0];
    t /= b.ext[0];
    j = b.lo[1] + t % b.ext[1];
    k = b.lo[2] + t / b.ext[1];
    return true;
}

// t-th point of colour `colour` ((i + j + k) mod 2) in the box
__host__ __device__ inline bool box_colour_pos(const Box &b, int colour, int t, int &i, int &j, int &k)
{
    const int half = (b.ext[0] + 1) >> 1;
    if (t >= half * b.ext[1] * b.ext[2]) return false;
    const int ih = t % half;
    t /= half;
    j = b.lo[1] + t % b.ext[1];
    k = b.lo[2] + t / b.ext[1];
    i = b.lo[0] + 2 * ih + ((b.lo[0] + j + k + colour) & 1);
    return i < b.lo[0] + b.ext[0];
}

// Division of 0 <= t < 2^31 by a fixed d >= 1 through one 64-bit multiply:
// with 2^(l-1) < d <= 2^l and m = ceil(2^(31+l) / d), floor(t / d) equals
// (t m) >> (31 + l) exactly (Granlund and Montgomery, "Division by invariant
// integers using multiplication", 1994).  m <= 2^32, so t m < 2^63.
struct Div {
    unsigned long long m;
    int sh;
};

__host__ __device__ inline Div make_div(int d)
{
    int l = 0;
    while ((1ll << l) < (long long)d) ++l;
    Div r;
    r.sh = 31 + l;
    r.m = ((1ull << r.sh) + (unsigned long long)d - 1) / (unsigned long long)d;
    return r;
}

__host__ __device__ inline int div_by(const Div &v, int t)
{
    return (int)(((unsigned long long)(unsigned)t * v.m) >> v.sh);
}

// the divisors of a box's point and colour decodes, made once per box (the
// one-workgroup cycle reads them from its level tables; a launched pass,
// with one point per thread, is faster dividing than waiting for them)
struct BoxDiv {
    Div x, half, y;   // ext[0], (ext[0] + 1) / 2, ext[1]
};

__host__ __device__ inline BoxDiv box_div(const Box &b)
{
    return BoxDiv{make_div(b.ext[0] > 0 ? b.ext[0] : 1), make_div(b.ext[0] > 0 ? (b.ext[0] + 1) >> 1 : 1),
                  make_div(b.ext[1] > 0 ? b.ext[1] : 1)};
}

// box_pos and box_colour_pos with the divisions made through bd
__host__ __device__ inline bool box_pos(const Box &b, const BoxDiv &bd, int t, int &i, int &j, int &k)
{
    const int n = b.ext[0] * b.ext[1] * b.ext[2];
    if (t >= n) return false;
    const int r = div_by(bd.x, t);
    i = b.lo[0] + (t - r * b.ext[0]);
    const int kk = div_by(bd.y, r);
    j = b.lo[1] + (r - kk * b.ext[1]);
    k = b.lo[2] + kk;
    return true;
}

__host__ __device__ inline bool box_colour_pos(const Box &b, const BoxDiv &bd, int colour, int t, int &i, int &j,
                                               int &k)
{
    const int half = (b.ext[0] + 1) >> 1;
    if (t >= half * b.ext[1] * b.ext[2]) return false;
    const int r = div_by(bd.half, t);
    const int ih = t - r * half;
    const int kk = div_by(bd.y, r);
    j = b.lo[1] + (r - kk * b.ext[1]);
    k = b.lo[2] + kk;
    i = b.lo[0] + 2 * ih + ((b.lo[0] + j + k + colour) & 1);
    return i < b.lo[0] + b.ext[0];
}

// Taps of the transfers along one axis (vert: the lattice is vertex-centred
// along it): full weighting of the fine points around coarse index I, and
// linear interpolation of fine index f from its coarse neighbours.
__host__ __device__ inline int rst_weights(int vert, int I, int *fq, double *w)
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

__host__ __device__ inline int prl_weights(int vert, int f, int *cq, double *w)
{
    if (vert) {
        if ((f & 1) == 0) { cq[0] = f >> 1; w[0] = 1.0; return 1; }
        cq[0] = (f - 1) >> 1; w[0] = 0.5;
        cq[1] = (f + 1) >> 1; w[1] = 0.5;
        return 2;
    }
    const int I = f >> 1;
    cq[0] = I; w[0] = 0.75;
    cq[1] = (f & 1) ? I + 1 : I - 1; w[1] = 0.25;
    return 2;
}

template <typename T>
struct VelArr {
    T *c[3];
};
template <typename T>
struct VelArrC {
    const T *c[3];
};

// pressure operator coefficients: beta = 1 / rho on the D face lattices
template <typename T>
struct CoefP {
    const T *beta[3];
};
// viscous operator coefficients: rho on the faces, mu at cells, mu on the
// edge lattices indexed by their parallel axis (2D: corners in mue[2])
template <typename T>
struct CoefU {
    const T *rho[3];
    const T *muc;
    const T *mue[3];
    int dec;  // constant viscosity (eq:NSdis1): muc and mue are not read
};

template <typename T>
inline VelArrC<T> cview(const VelArr<T> &v)
{
    return VelArrC<T>{{v.c[0], v.c[1], v.c[2]}};
}

// ---- multigrid (mg.hip) ----
template <typename T>
void launch_smooth_p(const Grid &g, const T *b, T *x, const CoefP<T> &cf, T cvisc, int colour, hipStream_t s,
                     int zb = 0);
template <typename T>
void launch_smooth_u(const Grid &g, int a, const T *b, const VelArr<T> &x, const CoefU<T> &cf, T mass, T cvisc,
                     int colour, hipStream_t s, int zb = 0);
// one colour of every component of the constant-viscosity system, one launch
template <typename T>
void launch_smooth_u_dec(const Grid &g, const VelArrC<T> &b, const VelArr<T> &x, const CoefU<T> &cf, T mass, T cvisc,
                         int colour, hipStream_t s);
template <typename T>
int launch_resid_p(const Grid &g, const T *b, const T *x, const CoefP<T> &cf, T cvisc, T *r, double *partial,
                   hipStream_t s);
template <typename T>
int launch_resid_u(const Grid &g, const VelArrC<T> &b, const VelArr<T> &x, const CoefU<T> &cf, T mass, T cvisc,
                   const VelArr<T> &r, double *partial, hipStream_t s);
template <typename T>
int launch_norm2(const Grid &g, int ncomp, const int *vmasks, const VelArrC<T> &v, double *partial, hipStream_t s);
void launch_reduce_final(const double *partial, long long n, double *out, hipStream_t s);
// zero_x (may be null): coarse arrays cleared at the restricted positions
template <typename T>
void launch_restrict(const Grid &gf, const Grid &gc, int ncomp, const int *vmasks, int role, bool all_stored,
                     const VelArrC<T> &fine, const VelArr<T> &coarse, T scale, hipStream_t s,
                     const VelArr<T> *zero_x = nullptr);
template <typename T>
void launch_prolong_add(const Grid &gc, const Grid &gf, int ncomp, const int *vmasks, int role,
                        const VelArrC<T> &coarse, const VelArr<T> &fine, hipStream_t s);
// largest coarsest system that is inverted (its matrix is held in LDS)
constexpr int DENSE_LDS = 64;
// inverse M of the coarsest operator (n <= DENSE_LDS unknowns listed by
// uidx/ucomp): column j is assembled by applying the operator to e_j in its
// own scratch (tmp: n * ncomp * nel doubles), Aw receives A (n x n)
void launch_dense_inverse(const Grid &g, int velocity, int n, const long long *uidx, const int *ucomp,
                          const CoefP<double> &cp, const CoefU<double> &cu, double mass, double cvisc, double *tmp,
                          int singular, double *Aw, double *M, hipStream_t s);
template <typename T>
void launch_dense_apply(const Grid &g, int velocity, int n, const long long *uidx, const int *ucomp, const double *M,
                        const VelArrC<T> &b, const VelArr<T> &x, hipStream_t s);
// dst = src at the unknowns of each lattice (src component may be null: zero),
// with dst's ghost images written (velocity: face lattices, else cells)
template <typename T>
void launch_load_unknowns(const Grid &g, int ncomp, const int *vmasks, const VelArrC<T> &src, const VelArr<T> &dst,
                          hipStream_t s);
// Arrays of one level that one launch treats together (blockIdx.y picks
// the array): up to D face densities and inverse densities, the cell and
// the edge viscosities.
constexpr int COEF_SET = 10;
template <typename T>
struct CoefSet {
    int n;
    int vmask[COEF_SET];   // lattice of each array
    T *v[COEF_SET];
};
// fill the ghost layers of the set's fields from their stored positions
template <typename T>
void launch_coef_ghosts(const Grid &g, const CoefSet<T> &set, hipStream_t s);
template <typename T>
void launch_fill(T *p, long long n, T v, hipStream_t s);
template <typename Ts, typename Td>
void launch_cast_unknowns(const Grid &g, int ncomp, const int *vmasks, const VelArrC<Ts> &src, const VelArr<Td> &dst,
                          hipStream_t s);
// b32 = (float) r at the unknowns and x32 = 0 everywhere, for ncomp
// lattices (the start of a refined iteration's FP32 cycles)
void launch_inner_start(const Grid &g, int ncomp, const int *vmasks, const VelArrC<double> &r, const VelArr<float> &b32,
                        const VelArr<float> &x32, hipStream_t s);
void launch_add_correction(const Grid &g, int ncomp, const int *vmasks, const VelArrC<float> &e,
                           const VelArr<double> &x, hipStream_t s);

// One level of the hierarchy as seen by the single-workgroup coarse cycle
// (kept in device memory, written once when the context is created).
template <typename T>
struct LevTab {
    Grid g;
    T *xu[3], *bu[3], *ru[3];
    T *xp, *bp, *rp;
    const T *rho[3], *beta[3], *muc, *mue[3];
    T mass, cvu, cvp;
    long long nu, np;
    int dec;  // constant viscosity, as CoefU::dec
    const BoxDiv *bd;  // device array [4]: divisors of the unknown boxes (components 0..2, pressure)
};

// the V-cycle from level l0 down to the coarsest level and back inside one
// workgroup of WG_THREADS threads; ndense > 0: the coarsest level is solved
// with the inverse M
// (512 threads leave each thread up to 256 registers, so the fully inlined
// cycle does not spill)
constexpr int WG_THREADS = 512;
__host__ __device__ constexpr int wg_threads(int, int) { return WG_THREADS; }
// Where the one-workgroup cycle keeps a level: arrays of levels l >= ls
// with an offset >= 0 below live in the workgroup's LDS arena (byte
// offsets), every other array stays where it is in global memory.  Staged
// coefficients are copied in and staged solver arrays cleared when the
// kernel starts.  The start level may be staged too, then with at least its
// solver arrays: its x and b are copied in and x is copied back at the end;
// nothing else of the staged levels is needed after the kernel.
struct LdsLevel {
    int xu[3], bu[3], ru[3], rho[3], beta[3], mue[3];
    int xp, bp, rp, muc;
};
constexpr int WG_MAXLEV = 16;
struct LdsPlan {
    const LdsLevel *lev;   // device array [WG_MAXLEV]
    int ls;                // first level in LDS (L: none)
    int bytes;             // arena size
};

// The part of a V-cycle below the start level of the one-workgroup cycle,
// as its linear map.  That part (smoothing, residuals and transfers down to
// the coarsest level and back) starts from a zero iterate, so its result is
// a fixed matrix times the restricted right-hand side.  Tm holds that matrix
// (n rows, n columns, in the precision of the cycle) in blocks of 16 bytes'
// worth of columns, each block row after row, built by running the same
// passes on every unit right-hand side;
// idx and comp list the n unknowns of level `level` (padded index and
// component, in the order comp, z, y, x).  n == 0: no tail, the cycle
// recurses to the coarsest level.
constexpr int TAIL_MAX = 512;
struct Tail {
    const void *Tm;
    const long long *idx;
    const int *comp;
    int n, level;
};

// sets the dynamic-LDS limit of the one-workgroup kernels (once per process)
void wg_prepare();
template <typename T>
void launch_coarse_vcycle(int D, const LevTab<T> *tab, int l0, int L, int vel, int nu1, int nu2, int ndense,
                          const long long *uidx, const int *ucomp, const double *M, const LdsPlan &plan,
                          const Tail &tail, hipStream_t s);
// columns of a tail: one workgroup per unknown of level tail.level runs the
// cycle from there on that unit right-hand side (every level of it staged in
// LDS by `plan`) and writes the result into column j of tail.Tm
template <typename T>
void launch_tail_columns(int D, const LevTab<T> *tab, int L, int vel, int nu1, int nu2, int ndense,
                         const long long *uidx, const int *ucomp, const double *M, const LdsPlan &plan,
                         const Tail &tail, hipStream_t s);
// largest LDS arena the coarse cycle may use on the current device (bytes)
int wg_lds_budget();

// GCR on the finest level (FP64): q = A z at the unknowns; per-block sums of
// x . y (returns the number of partial sums); q -= (num/den) qi and
// z -= (num/den) zi; x += (num/den) z with ghost images
void launch_apply(const Grid &g, int velocity, const VelArr<double> &z, const CoefP<double> &cp,
                  const CoefU<double> &cu, double mass, double cvisc, const VelArr<double> &q, hipStream_t s);
int launch_dot(const Grid &g, int velocity, const VelArrC<double> &x, const VelArrC<double> &y, double *partial,
               hipStream_t s);
void launch_gcr_axpy2(const Grid &g, int velocity, const double *num, const double *den, const VelArrC<double> &qi,
                      const VelArrC<double> &zi, const VelArr<double> &q, const VelArr<double> &z, hipStream_t s);
void launch_gcr_update(const Grid &g, int velocity, const double *num, const double *den, const VelArrC<double> &z,
                       const VelArr<double> &x, hipStream_t s);

// One red-black sweep (red then black) of component a (vel) or of the
// pressure in one launch: reads xin (all components), writes the updated
// component, with its ghost images, to xout (a second buffer; the other
// entries of xout must already hold the field's fixed values)
template <typename T>
void launch_smooth_rb(const Grid &g, int vel, int a, const VelArrC<T> &xin, const T *b, const CoefU<T> &cu,
                      const CoefP<T> &cp, T mass, T cvisc, T *xout, hipStream_t s);

// The same sweep for velocity component a of a 3D level (coupled viscous
// system), with every workgroup marching along z through a run of planes
// and holding a window of u_a in LDS; same contract as launch_smooth_rb.
// zm_fits: the level's periodic axes are long enough for the window and even.
template <typename T>
void launch_smooth_zm(const Grid &g, int a, const VelArrC<T> &xin, const T *b, const CoefU<T> &cu, T mass, T cvisc,
                      T *xout, hipStream_t s);
bool zm_fits(const Grid &g);

// Arm a start/stop event pair for the next smoother or residual launch of
// this thread: the dispatch itself records the kernel's start and end.
void set_launch_events(hipEvent_t start, hipEvent_t stop);
// the armed pair, handed to the next launch and disarmed (false: none armed)
bool take_launch_events(hipEvent_t *start, hipEvent_t *stop);

// launch `kernel`; when a pair of events is armed, its dispatch records the
// kernel's own start and end into them
template <typename K, typename... Args>
inline void launch_timed_shm(K kernel, dim3 grid, dim3 block, unsigned shm, hipStream_t s, Args... args)
{
    hipEvent_t e0, e1;
    if (take_launch_events(&e0, &e1)) hipExtLaunchKernelGGL(kernel, grid, block, shm, s, e0, e1, 0, args...);
    else hipLaunchKernelGGL(kernel, grid, block, shm, s, args...);
}

template <typename K, typename... Args>
inline void launch_timed(K kernel, dim3 grid, dim3 block, hipStream_t s, Args... args)
{
    launch_timed_shm(kernel, grid, block, 0, s, args...);
}

// ---- Galerkin coarse operators of the viscous system (galerkin.hip) ----
// Row (a, I) of R A P couples unknown (b, I + delta) only for delta in a box
// per axis: same component: [-1, 1] along a and [-2, 2] across it; another
// component b: [-2, 1] along a, [-1, 2] along b, [-2, 2] along the third
// axis (the reach of full weighting, the 7 + 8 point rows and linear
// prolongation, which R A P keeps from level to level once the third axis
// has grown from [-1, 1] on the first coarse level; a product landing
// outside is reported, never dropped).
// The entries of the rows of component a are stored slot-major: slot s of
// the row at position e is v[a][s * nel + e]; a row's slots list column
// component b = 0 .. D-1 in turn, each box x fastest.  On a periodic axis a
// column that several offsets of the box reach sits in the offset of least
// magnitude (the more negative one on a tie), so every column is in exactly
// one slot and the diagonal is offset 0 of the row's own component.
struct GalBox {
    int lo[3], n[3];
};
__host__ __device__ constexpr GalBox gal_box(int D, int a, int b)
{
    GalBox x{};
    for (int d = 0; d < 3; ++d) {
        if (d >= D) { x.lo[d] = 0; x.n[d] = 1; continue; }
        if (a == b) { x.lo[d] = d == a ? -1 : -2; x.n[d] = d == a ? 3 : 5; }
        else if (d == a) { x.lo[d] = -2; x.n[d] = 4; }
        else if (d == b) { x.lo[d] = -1; x.n[d] = 4; }
        else { x.lo[d] = -2; x.n[d] = 5; }
    }
    return x;
}
__host__ __device__ constexpr int gal_box_slots(int D, int a, int b)
{
    return gal_box(D, a, b).n[0] * gal_box(D, a, b).n[1] * gal_box(D, a, b).n[2];
}
__host__ __device__ constexpr int gal_first_slot(int D, int a, int b)
{
    int s = 0;
    for (int c = 0; c < b; ++c) s += gal_box_slots(D, a, c);
    return s;
}
__host__ __device__ constexpr int gal_row_slots(int D, int a) { return gal_first_slot(D, a, D); }
constexpr int GAL_MAX_BOX = 80;

template <typename T>
struct GalOp {
    T *v[3];
};
template <typename T>
struct GalOpC {
    const T *v[3];
};

// The operator of level l+1 (grid gc) from level l (grid gf), in FP64.
// fine == nullptr: level l is the finest, whose rows are the viscous stencil
// on the coefficients cu (mass = sigma / dt, cvisc = Re^-1 / h^2); otherwise
// level l's own Galerkin operator.  *err is set to 1 when a product falls
// outside its box.
void launch_gal_build(int D, const Grid &gf, const Grid &gc, const CoefU<double> &cu, double mass, double cvisc,
                      const GalOpC<double> *fine, const GalOp<double> &out, int *err, hipStream_t s);
// FP32 copy of a level's operator
void launch_gal_to_f32(int D, const Grid &g, const GalOpC<double> &src, const GalOp<float> &dst, hipStream_t s);
// One colour pass over component a: every row of that colour from the
// values x held before the pass, written to y together with the other
// colour's unchanged values (y then replaces x[a]).
template <typename T>
void launch_gal_smooth(int D, const Grid &g, int a, int colour, const GalOpC<T> &op, const T *b, const VelArrC<T> &x,
                       T *y, hipStream_t s);
// r = b - A x at every unknown
template <typename T>
void launch_gal_resid(int D, const Grid &g, const GalOpC<T> &op, const VelArrC<T> &b, const VelArrC<T> &x,
                      const VelArr<T> &r, hipStream_t s);
// inverse of a coarsest Galerkin operator of n <= DENSE_LDS unknowns
void launch_gal_dense_inverse(int D, const Grid &g, int n, const long long *uidx, const int *ucomp,
                              const GalOpC<double> &op, double *Aw, double *M, hipStream_t s);
// Gauss-Jordan inverse of the n x n matrix Aw (mg.hip)
void launch_dense_gj(int n, int singular, const double *Aw, double *M, hipStream_t s);

// ---- batched passes over several contexts (mg.hip) ----
// One entry per block of a batched launch: the context's level table(s) at
// the pass's level, the first block of that context in the launch, and for
// residual norms the context's partial-sum buffer and block count.
struct BEntry {
    const void *tab;    // LevTab<T> at the level of the pass (FP64 table for prep / add)
    const void *tab2;   // FP32 level-0 table (prep / add)
    double *partial;    // residual norms: per-block sums (null: none)
    int base;           // first block of this context in the launch
    int nb;             // residual: blocks of this context; reduce: partial sums
    int ctx;            // member index (flag, norm slot)
    int pad;
};

// the coarse part of a context's V-cycle (one workgroup)
struct BCoarse {
    const void *tab;    // LevTab<T> array of the context (all levels)
    const long long *uidx;
    const int *ucomp;
    const double *M;
    const LdsLevel *lds;   // the member's LDS plan (levels >= lds_from)
    int l0, L, ndense, ctx;
    int lds_from, pad;
    Tail tail;             // the member's tail (n == 0: none)
};

// pass kinds
enum { BK_SWEEP = 0, BK_RESID = 1, BK_RESTRICT = 2, BK_PROLONG = 3, BK_PREP = 4, BK_ADD = 5 };
// blocks one context needs in a batched pass of kind `kind` on level grid g
// (gc: the next coarser grid, for restriction); A: component of a sweep
int batch_blocks(int kind, const Grid &g, const Grid &gc, int vel, int A);
template <typename T>
void launch_bpass(int kind, int D, int vel, int A, int colour, const BEntry *ent, unsigned nblocks, const int *flags,
                  hipStream_t s);
void launch_breduce(const BEntry *ent, unsigned nitems, const int *flags, double *norms, hipStream_t s);
template <typename T>
void launch_bcoarse(int D, int vel, const BCoarse *items, unsigned nitems, const int *flags, int nu1, int nu2,
                    int lds_bytes, hipStream_t s);

// ---- fields (fields.hip) ----
struct Phys {
    double sigma, eps, inv_re, force_coef, dt;
    double body_force[3];
    double rho0, rho_b, d0_pow_d, mu_out, mu_max, omega;
    int kernel;
};
// compact <-> uniform layout of one lattice (vmask), to_uniform selects direction
void launch_layout(const Grid &g, int vmask, const double *src, double *dst, bool to_uniform, hipStream_t s);
void launch_momentum_rhs(const Grid &g, const Phys &ph, const VelArrC<double> &u, const CoefU<double> &cf,
                         const VelArrC<double> &f, const VelArr<double> &b, hipStream_t s);
void launch_pressure_div(const Grid &g, const Phys &ph, const VelArrC<double> &ut, const VelArrC<double> &ubd,
                         double *bp, hipStream_t s);
void launch_add_scalar_cells(const Grid &g, double *v, const double *sum, double scale, hipStream_t s);
void launch_project(const Grid &g, const Phys &ph, const VelArrC<double> &ut, const double *p,
                    const CoefP<double> &beta, const VelArr<double> &u, hipStream_t s);
void launch_copy(const double *src, double *dst, long long n, hipStream_t s);
// beta_a = 1 / rho_a at the stored positions of every face lattice a < D
void launch_beta_faces(const Grid &g, const VelArrC<double> &rho, const VelArr<double> &beta, hipStream_t s);
int launch_sum_cells(const Grid &g, const double *v, double *partial, hipStream_t s);
// FP32 copies of whole arrays of n entries: dst[q][t] = (float) src.v[q][t]
void launch_to_f32(const CoefSet<double> &src, float *const dst[COEF_SET], long long n, hipStream_t s);

// ---- immersed boundary (ib.hip) ----
struct Bins {
    int nb[3];          // bins per axis
    double bs[3];       // bin width per axis
    int nbins;
    int *bin_of;        // [eta] bin of each node
    int *count;         // [nbins] nodes per bin, then a cursor
    int *start;         // [nbins + 1] exclusive prefix
    int *sorted;        // [eta] node ids grouped by bin, ascending within a bin
    unsigned char *near;  // [nbins] 1 when a node lies in the bin or a neighbouring bin
                          // (where its points look); null: not kept, every point looks
};
void launch_bin_nodes(const Grid &g, const Bins &bins, const double *X, long long stride, int eta, int *scan_tmp,
                      hipStream_t s);
// spread of the face force (F may be null) and density, or of the viscosity
// max at cells and edges; kind: 0 faces (axis a), 1 cells, 2 edges (axis c)
void launch_spread_face(const Grid &g, const Phys &ph, const Bins &bins, const double *X, const double *F,
                        long long stride, int a, double width, double *f_out, double *rho_out, hipStream_t s);
void launch_spread_visc(const Grid &g, const Phys &ph, const Bins &bins, const double *X, long long stride, int vmask,
                        double *mu_out, hipStream_t s);
void launch_interp(const Grid &g, int kernel, double width, const VelArrC<double> &u, const double *X,
                   long long xstride, int eta, double *U, long long ustride, hipStream_t s);
void launch_euler(const Grid &g, double c, const double *U, double *X, long long stride, int eta, hipStream_t s);
void launch_spring_break(const Grid &g, double ratio, const double *X, long long stride, const int *ij, int m,
                         const double *rest, unsigned char *alive, int *n_broken, hipStream_t s);
void launch_spring_force(const Grid &g, const double *X, long long stride, int eta, const int *ij, int m,
                         const double *rest, const double *K, const unsigned char *alive, const int *inc_start,
                         const int *inc_list, double *F, hipStream_t s);
// counting sort of keys[0..n) into buckets [0, nbuckets): start (exclusive
// prefix, nbuckets + 1 entries) and ids grouped by bucket, ascending in
// id % mod within a bucket (mod = 0: ascending id)
// detached fragments (connected components of the alive springs)
void launch_frag_anchor(const Grid &g, const double *X, long long stride, int eta, int axis, double dist,
                        unsigned char *anchored, hipStream_t s);
void launch_frag_init(int *label, int eta, hipStream_t s);
// one hook + shortcut round; *changed (device) is set when a label moved
void launch_frag_round(const int *ij, int m, const unsigned char *alive, int *label, int eta, int *changed,
                       hipStream_t s);
// counts[0] = fragments, counts[1] = fragments without an anchored node
void launch_frag_count(const int *label, const unsigned char *anchored, int eta, int *root_anchored, int *counts,
                       hipStream_t s);

// ints of scratch the bucket sort needs for nb buckets
int scan_scratch_ints(long long nb);
void launch_bucket_sort(const int *keys, int n, int nbuckets, int *count, int *start, int *ids, int mod,
                        int *scan_tmp, hipStream_t s);
void launch_incidence_keys(const int *ij, int m, int *keys, hipStream_t s);
void launch_count_alive(const unsigned char *alive, int m, int *out, hipStream_t s);

}  // namespace ibmg
