// Host side of the library: context and workspace, the multigrid drivers
// (FP64 V-cycles, and FP32 V-cycles inside FP64 defect correction), the
// projection step and the Lagrangian update, and the C interface declared
// in include/ibmg.h.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ibmg.h"
#include "common.h"
#include "kernels.h"

using namespace ibmg;

namespace {

constexpr int DENSE_MAX = DENSE_LDS;   // coarsest systems up to this size are inverted
constexpr int MAXLEV = 16;

struct Level {
    Grid g;
    long long np = 0, nu = 0;
    // FP64 solver arrays (level 0: x is u~ / the pressure iterate)
    double *xp = nullptr, *bp = nullptr, *rp = nullptr;
    double *xu[3] = {}, *bu[3] = {}, *ru[3] = {};
    double *rho[3] = {}, *beta[3] = {}, *muc = nullptr, *mue[3] = {};
    // FP32 copies for the inner cycles of the refined solver
    float *xp32 = nullptr, *bp32 = nullptr, *rp32 = nullptr;
    float *xu32[3] = {}, *bu32[3] = {}, *ru32[3] = {};
    float *rho32[3] = {}, *beta32[3] = {}, *muc32 = nullptr, *mue32[3] = {};
    // second iterate buffers of the one-launch red-black sweep (swapped with
    // x after every sweep; an even number of sweeps per V-cycle brings them
    // back), and whether this level uses that sweep: the tiled one for both
    // systems (fused), or the z-marching one for the velocity (zm)
    double *xu_alt[3] = {}, *xp_alt = nullptr;
    float *xu32_alt[3] = {}, *xp32_alt = nullptr;
    bool fused = false, zm = false;
    // Re^-1 / h^2 of the viscous rows; with constant viscosity (eq:NSdis1)
    // times mu_out and the product of gamma down to this level
    double cvu = 0;
    int dec = 0;
    // colour passes of this level z-blocked (3D launched levels)
    int zb = 0;
    // Galerkin operator of the viscous system on this level (levels >= 1
    // when the descriptor asks for it), FP64 and, refined, FP32, and the
    // second buffer of its colour passes (swapped with x after each pass)
    bool gal = false;
    double *gv[3] = {}, *gy[3] = {};
    float *gv32[3] = {}, *gy32[3] = {};
};

struct Carver {
    char *base;
    size_t off = 0;
    bool dry;
    template <typename T>
    T *take(size_t n)
    {
        off = (off + 255) & ~(size_t)255;
        T *p = dry ? nullptr : reinterpret_cast<T *>(base + off);
        off += n * sizeof(T);
        return p;
    }
};

}  // namespace

struct ibb_ctx {
    ibb_desc d;
    hipStream_t s = nullptr;
    int L = 0;
    int E = 0;              // edge lattices (3 in 3D, 1 in 2D)
    int edge_axis[3] = {};  // their parallel axes
    Level lv[MAXLEV];
    bool singular_p = false;
    Phys ph;
    // state
    double *u[3] = {}, *p = nullptr, *f[3] = {};
    // coarsest dense inverses
    long long *uidx_p = nullptr, *uidx_u = nullptr;
    int *ucomp_p = nullptr, *ucomp_u = nullptr;
    double *Mp = nullptr, *Mu = nullptr, *Aw = nullptr, *Atmp = nullptr;
    int *scan_tmp = nullptr;   // block sums of the multi-block scan
    // reductions
    double *partial = nullptr, *scalar = nullptr;
    // level tables for the one-workgroup coarse cycle, and where it starts
    LevTab<double> *tab64 = nullptr;
    LevTab<float> *tab32 = nullptr;
    BoxDiv *boxdiv = nullptr;   // [MAXLEV][4], pointed to by the level tables
    int lc_u = MAXLEV, lc_p = MAXLEV;
    // levels of the one-workgroup cycle kept in LDS, per precision (0: FP64,
    // 1: FP32) and system (0: pressure, 1: velocity)
    LdsLevel *ldslev[2][2] = {};
    int lds_ls[2][2] = {}, lds_bytes[2][2] = {};
    // tails of the one-workgroup cycle per system (0 pressure, 1 velocity),
    // in the precision of the context's V-cycles: matrix, unknown list, and
    // the plan that stages every level of the tail for the column build
    Tail tail[2] = {};
    LdsLevel *tplan[2] = {};
    int tplan_bytes[2] = {};
    // nodes and springs
    long long eta_max = 0, m_max = 0;
    int eta = 0, m = 0;
    double *X = nullptr, *F = nullptr, *U = nullptr;
    Bins bins;
    int nbins_cap = 0;
    int *ij = nullptr;
    double *rest = nullptr, *K = nullptr;
    unsigned char *alive = nullptr;
    int *inc_keys = nullptr, *inc_count = nullptr, *inc_start = nullptr, *inc_list = nullptr;
    int *counters = nullptr;   // [0] broken this update, [1] alive, [2] fragments, [3] detached
    int *gal_err = nullptr;    // set when a Galerkin product leaves its stencil box
    // GCR on the finest level: right-hand side, iterate, residual, and the
    // stored directions z_j, q_j (component arrays of the finest level)
    double *gb[3] = {}, *gx[3] = {}, *gr[3] = {};
    std::vector<double *> gz, gq;   // [m * 3]
    double *gs = nullptr;           // scalars: (q_j, q_j) for j < m, then scratch
    // detached fragments
    unsigned char *anchored = nullptr;
    int *frag_label = nullptr, *frag_root = nullptr, *frag_flag = nullptr;
    bool have_nodes = false, have_springs = false, have_coefs = false;
    hipEvent_t ev[4] = {};
    // one solver iteration with the residual norm after it, per system
    // (pressure, velocity), captured once on a private stream and replayed
    // on the context's stream
    hipStream_t cap = nullptr;
    hipGraphExec_t tick[2] = {};
    // GCR: one graph per system and position in the restart window (the
    // number of Gram-Schmidt steps depends on it)
    std::vector<hipGraphExec_t> gtick[2];
    // finest-level kernel timing (ibb_profile_*)
    bool prof = false;
    std::vector<hipEvent_t> pev;           // pairs: start, stop
    std::vector<int> pcls;                 // class of each recorded pair
    std::vector<long long> punits;         // unknowns of each recorded pair
    int pused = 0;
    long long plaunch[IBB_PROFILE_CLASSES] = {};
    double pms[IBB_PROFILE_CLASSES] = {};
    long long punit_tot[IBB_PROFILE_CLASSES] = {};
    std::string err;
};

namespace {

ibb_status fail(ibb_ctx *c, ibb_status st, const char *msg)
{
    if (c) c->err = msg;
    return st;
}

#define HIPCHK(expr)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) {                                                              \
            if (c) c->err = std::string(#expr) + ": " + hipGetErrorString(e_);               \
            return IBB_EDEVICE;                                                              \
        }                                                                                    \
    } while (0)

constexpr int PROF_PAIRS = 2048;

// launch sites of the solvers (ibb_profile_read class = site + 32 x level)
enum ProfSite {
    PS_SMOOTH_U64 = 0, PS_SMOOTH_P64 = 1, PS_SMOOTH_U32 = 2, PS_SMOOTH_P32 = 3,
    PS_RESID_U64 = 4, PS_RESID_P64 = 5, PS_RESID_U32 = 6, PS_RESID_P32 = 7,
    PS_RESTRICT64 = 8, PS_RESTRICT32 = 9, PS_PROLONG64 = 10, PS_PROLONG32 = 11,
    PS_COARSE_U64 = 12, PS_COARSE_P64 = 13, PS_COARSE_U32 = 14, PS_COARSE_P32 = 15,
    PS_DENSE = 16, PS_OUTER = 17, PS_GCR = 18, PS_SMOOTH_UDEC64 = 19, PS_SMOOTH_UDEC32 = 20,
    PS_SMOOTH_RB64 = 21, PS_SMOOTH_RB32 = 22,
    // the Lagrangian update (level 0)
    PS_SPREAD_FACE = 23, PS_SPREAD_VISC = 24, PS_INTERP = 25, PS_SPRING_FORCE = 26,
    PS_GAL_BUILD = 27, PS_GAL_SMOOTH64 = 28, PS_GAL_SMOOTH32 = 29, PS_GAL_RESID64 = 30, PS_GAL_RESID32 = 31
};

inline int prof_class(int site, int level) { return site + 32 * level; }

int prof_begin(ibb_ctx *c, int cls, long long units);
void prof_end(ibb_ctx *, int k);

// times the next launch within its scope (when kernel timing is on)
struct Timed {
    ibb_ctx *c;
    int k;
    Timed(ibb_ctx *c_, int site, int level, long long units) : c(c_), k(prof_begin(c_, prof_class(site, level), units)) {}
    ~Timed() { prof_end(c, k); }
};

void prof_flush(ibb_ctx *c);

// time the next launch (of class cls): its dispatch records the kernel's
// start and end into the slot's event pair; returns the slot or -1
int prof_begin(ibb_ctx *c, int cls, long long units)
{
    if (!c->prof || cls < 0 || cls >= IBB_PROFILE_CLASSES) return -1;
    if (c->pused >= PROF_PAIRS) prof_flush(c);
    const int k = c->pused++;
    c->pcls[k] = cls;
    c->punits[k] = units;
    set_launch_events(c->pev[2 * k], c->pev[2 * k + 1]);
    return k;
}

// disarm the pair if the launcher had nothing to launch
void prof_end(ibb_ctx *, int k)
{
    if (k >= 0) set_launch_events(nullptr, nullptr);
}

// fold the recorded pairs into the totals (synchronises on the last event)
void prof_flush(ibb_ctx *c)
{
    if (!c->prof || c->pused == 0) return;
    (void)hipEventSynchronize(c->pev[2 * (c->pused - 1) + 1]);
    for (int k = 0; k < c->pused; ++k) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, c->pev[2 * k], c->pev[2 * k + 1]) == hipSuccess) {
            c->plaunch[c->pcls[k]] += 1;
            c->pms[c->pcls[k]] += ms;
            c->punit_tot[c->pcls[k]] += c->punits[k];
        }
    }
    c->pused = 0;
}

// message of the last failed ibb_create on this thread
thread_local std::string create_err;

ibb_status check_desc(const ibb_desc *d)
{
    if (!d) return IBB_EINVAL;
    if (d->dim != 2 && d->dim != 3) return IBB_EINVAL;
    for (int a = 0; a < d->dim; ++a) {
        if (d->n[a] < 2 || d->n[a] % 2) return IBB_EINVAL;
        if (d->axis_bc[a] < 0 || d->axis_bc[a] > 2) return IBB_EINVAL;
    }
    if (!(d->h > 0) || !(d->dt > 0) || !(d->sigma > 0) || !(d->eps > 0)) return IBB_EINVAL;
    if (!(d->omega > 0) || !(d->rho0 > 0) || !(d->mu_out > 0)) return IBB_EINVAL;
    if (d->kernel != 0 && d->kernel != 1) return IBB_EINVAL;
    if (d->nu1 < 0 || d->nu2 < 0 || d->nu1 + d->nu2 < 1 || d->max_cycles < 1) return IBB_EINVAL;
    if (d->precision != IBB_FP64 && d->precision != IBB_FP32_REFINED) return IBB_EINVAL;
    if (d->precision == IBB_FP32_REFINED && d->inner_cycles < 1) return IBB_EINVAL;
    if (d->attach_axis < 0 || d->attach_axis >= d->dim || !(d->attach_dist >= 0)) return IBB_EINVAL;
    if (d->krylov_restart < 0 || d->krylov_restart > 64) return IBB_EINVAL;
    if (d->smoother_passes < 0 || d->smoother_passes > 3) return IBB_EINVAL;
    // the decoupled form holds only where the viscosity is one constant
    if (d->decoupled != 0 && d->decoupled != 1) return IBB_EINVAL;
    if (d->decoupled && d->mu_max != d->mu_out) return IBB_EINVAL;
    if (d->galerkin != 0 && d->galerkin != 1) return IBB_EINVAL;
    if (d->galerkin && d->decoupled) return IBB_EINVAL;
    for (int a = 0; a < d->dim; ++a)
        if (d->axis_bc[a] == IBB_AXIS_PERIODIC && 4.0 * d->omega > d->n[a] * d->h) return IBB_EINVAL;
    // array indices are formed in 32-bit arithmetic: every padded array
    // (n + 3 entries per axis) must hold fewer than 2^31 entries
    long long nel = 1;
    for (int a = 0; a < d->dim; ++a) nel *= (long long)d->n[a] + 3;
    if (nel >= (1ll << 31)) return IBB_EINVAL;
    return IBB_OK;
}

int count_levels(const ibb_desc *d)
{
    int n[3] = {d->n[0], d->n[1], d->dim == 3 ? d->n[2] : 2};
    int L = 1;
    while (L < MAXLEV) {
        bool ok = true;
        for (int a = 0; a < d->dim; ++a)
            if (n[a] % 2 || n[a] / 2 < 2) ok = false;
        if (!ok) break;
        for (int a = 0; a < d->dim; ++a) n[a] /= 2;
        ++L;
    }
    if (d->max_levels > 0 && d->max_levels < L) L = d->max_levels;
    return L;
}

Grid make_grid(const ibb_desc *d, int l)
{
    Grid g;
    g.D = d->dim;
    for (int a = 0; a < 3; ++a) {
        g.n[a] = a < d->dim ? d->n[a] >> l : 1;
        g.bc[a] = a < d->dim ? d->axis_bc[a] : 0;
    }
    g.NX = g.n[0] + 3;
    g.NY = g.n[1] + 3;
    g.NXY = (long long)g.NX * g.NY;
    g.nel = g.NXY * (d->dim == 3 ? g.n[2] + 3 : 1);
    g.h = d->h * (double)(1 << l);
    return g;
}

long long unknowns_of(const Grid &g, int vmask)
{
    long long n = 1;
    for (int d = 0; d < 3; ++d) {
        int lo, hi;
        unk_range(g, d, (vmask >> d) & 1, lo, hi);
        n *= (hi - lo + 1);
    }
    return n;
}

long long lattice_count(const Grid &g, int vmask)
{
    long long n = 1;
    for (int d = 0; d < 3; ++d) n *= stored_extent(g, d, (vmask >> d) & 1);
    return n;
}

// bins at least w wide: a point's support (|x - X| < 2 w) lies within two
// bins on each side of its own
void bins_for_width(const ibb_desc *d, double w, int nb[3], double bs[3])
{
    for (int a = 0; a < 3; ++a) {
        if (a >= d->dim) { nb[a] = 1; bs[a] = 1.0; continue; }
        const double L = d->n[a] * d->h;
        int k = (int)floor(L / w);
        if (k < 1) k = 1;
        nb[a] = k;
        bs[a] = L / k;
    }
}

// carve every array out of the workspace (dry run: only count bytes)
size_t carve(ibb_ctx *c, char *base, bool dry)
{
    Carver cv{base, 0, dry};
    const ibb_desc *d = &c->d;
    const int D = d->dim;
    const bool refined = d->precision == IBB_FP32_REFINED;
    for (int l = 0; l < c->L; ++l) {
        Level &L = c->lv[l];
        const size_t n = (size_t)L.g.nel;
        L.xp = cv.take<double>(n);
        L.bp = cv.take<double>(n);
        L.rp = cv.take<double>(n);
        for (int a = 0; a < D; ++a) {
            L.xu[a] = cv.take<double>(n);
            L.bu[a] = cv.take<double>(n);
            L.ru[a] = cv.take<double>(n);
            L.rho[a] = cv.take<double>(n);
            L.beta[a] = cv.take<double>(n);
        }
        L.muc = cv.take<double>(n);
        for (int e = 0; e < c->E; ++e) L.mue[c->edge_axis[e]] = cv.take<double>(n);
        if (L.fused || L.zm) {
            L.xp_alt = cv.take<double>(n);
            for (int a = 0; a < D; ++a) L.xu_alt[a] = cv.take<double>(n);
            if (refined) {
                L.xp32_alt = cv.take<float>(n);
                for (int a = 0; a < D; ++a) L.xu32_alt[a] = cv.take<float>(n);
            }
        }
        if (L.gal) {
            for (int a = 0; a < D; ++a) {
                const size_t ns = (size_t)gal_row_slots(D, a) * n;
                L.gv[a] = cv.take<double>(ns);
                L.gy[a] = cv.take<double>(n);
                if (refined) {
                    L.gv32[a] = cv.take<float>(ns);
                    L.gy32[a] = cv.take<float>(n);
                }
            }
        }
        if (refined) {
            L.xp32 = cv.take<float>(n);
            L.bp32 = cv.take<float>(n);
            L.rp32 = cv.take<float>(n);
            for (int a = 0; a < D; ++a) {
                L.xu32[a] = cv.take<float>(n);
                L.bu32[a] = cv.take<float>(n);
                L.ru32[a] = cv.take<float>(n);
                L.rho32[a] = cv.take<float>(n);
                L.beta32[a] = cv.take<float>(n);
            }
            L.muc32 = cv.take<float>(n);
            for (int e = 0; e < c->E; ++e) L.mue32[c->edge_axis[e]] = cv.take<float>(n);
        }
    }
    const size_t n0 = (size_t)c->lv[0].g.nel;
    for (int a = 0; a < D; ++a) {
        c->u[a] = cv.take<double>(n0);
        c->f[a] = cv.take<double>(n0);
    }
    c->p = cv.take<double>(n0);
    c->uidx_p = cv.take<long long>(DENSE_MAX);
    c->uidx_u = cv.take<long long>(DENSE_MAX);
    c->ucomp_p = cv.take<int>(DENSE_MAX);
    c->ucomp_u = cv.take<int>(DENSE_MAX);
    c->Mp = cv.take<double>(DENSE_MAX * DENSE_MAX);
    c->Mu = cv.take<double>(DENSE_MAX * DENSE_MAX);
    c->Aw = cv.take<double>(DENSE_MAX * DENSE_MAX);
    c->Atmp = cv.take<double>((size_t)DENSE_MAX * 3 * (size_t)c->lv[c->L - 1].g.nel);
    c->tab64 = cv.take<LevTab<double>>(MAXLEV);
    c->tab32 = cv.take<LevTab<float>>(MAXLEV);
    c->boxdiv = cv.take<BoxDiv>((size_t)MAXLEV * 4);
    for (int pr = 0; pr < 2; ++pr)
        for (int v = 0; v < 2; ++v) c->ldslev[pr][v] = cv.take<LdsLevel>(WG_MAXLEV);
    for (int v = 0; v < 2; ++v) {
        Tail &t = c->tail[v];
        if (t.n <= 0) continue;
        const size_t w = refined ? sizeof(float) : sizeof(double);
        const size_t ld = w == 4 ? ((size_t)t.n + 3) & ~(size_t)3 : ((size_t)t.n + 1) & ~(size_t)1;
        t.Tm = cv.take<char>((size_t)t.n * ld * w);
        t.idx = cv.take<long long>((size_t)t.n);
        t.comp = cv.take<int>((size_t)t.n);
        c->tplan[v] = cv.take<LdsLevel>(WG_MAXLEV);
    }
    c->partial = cv.take<double>(3 * NORM_BLOCKS_MAX);
    c->scalar = cv.take<double>(8);
    const size_t em = (size_t)(c->eta_max > 0 ? c->eta_max : 1);
    const size_t mm = (size_t)(c->m_max > 0 ? c->m_max : 1);
    c->X = cv.take<double>(3 * em);
    c->F = cv.take<double>(3 * em);
    c->U = cv.take<double>(3 * em);
    c->bins.bin_of = cv.take<int>(em);
    c->bins.sorted = cv.take<int>(em);
    c->bins.count = cv.take<int>((size_t)c->nbins_cap);
    c->bins.start = cv.take<int>((size_t)c->nbins_cap + 1);
    c->bins.near = cv.take<unsigned char>((size_t)c->nbins_cap);
    c->ij = cv.take<int>(2 * mm);
    c->rest = cv.take<double>(mm);
    c->K = cv.take<double>(mm);
    c->alive = cv.take<unsigned char>(mm);
    c->inc_keys = cv.take<int>(2 * mm);
    c->inc_list = cv.take<int>(2 * mm);
    c->inc_count = cv.take<int>(em);
    c->inc_start = cv.take<int>(em + 1);
    c->counters = cv.take<int>(8);
    c->gal_err = cv.take<int>(1);
    if (d->krylov_restart > 0) {
        const int m = d->krylov_restart;
        c->gz.assign(3 * (size_t)m, nullptr);
        c->gq.assign(3 * (size_t)m, nullptr);
        for (int a = 0; a < D; ++a) {
            c->gb[a] = cv.take<double>(n0);
            c->gx[a] = cv.take<double>(n0);
            c->gr[a] = cv.take<double>(n0);
            for (int j = 0; j < m; ++j) {
                c->gz[3 * j + a] = cv.take<double>(n0);
                c->gq[3 * j + a] = cv.take<double>(n0);
            }
        }
        c->gs = cv.take<double>((size_t)m + 8);
    }
    c->anchored = cv.take<unsigned char>(em);
    c->frag_label = cv.take<int>(em);
    c->frag_root = cv.take<int>(em);
    c->frag_flag = cv.take<int>(4);
    c->scan_tmp = cv.take<int>(scan_scratch_ints((long long)std::max<size_t>((size_t)c->nbins_cap, em + 1)));
    return cv.off + 256;
}

// LDS per workgroup that the tail decision assumes (gfx950: 160 KB, less
// the kernels' own shared data); fixed, so that footprints do not depend on
// the device queried
constexpr int TAIL_LDS_BUDGET = 163840 - (int)(WG_MAXLEV * sizeof(LevTab<double>)) - 1024 -
                                (int)(TAIL_MAX * sizeof(double));

// bytes of one level's array in the arena, and of every level from lt down
// staged whole (solver arrays and coefficients of one system)
int arena_array_bytes(const Grid &g, int wsz) { return (int)(((g.nel * wsz + 15) / 16) * 16); }

long long tail_lds_bytes(const ibb_ctx *c, bool f32, bool vel, int lt)
{
    const int D = c->d.dim;
    const int nsolve = vel ? 3 * D : 3, ncoef = vel ? D + 1 + c->E : D;
    long long b = 0;
    for (int l = lt; l < c->L; ++l) b += (long long)arena_array_bytes(c->lv[l].g, f32 ? 4 : 8) * (nsolve + ncoef);
    return b;
}

void setup_shapes(ibb_ctx *c, const ibb_desc *d, int64_t max_nodes, int64_t max_springs)
{
    c->d = *d;
    c->L = count_levels(d);
    c->E = d->dim == 3 ? 3 : 1;
    if (d->dim == 3) { c->edge_axis[0] = 0; c->edge_axis[1] = 1; c->edge_axis[2] = 2; }
    else c->edge_axis[0] = 2;
    double mu = d->mu_out;
    for (int l = 0; l < c->L; ++l) {
        Level &L = c->lv[l];
        L.g = make_grid(d, l);
        L.np = unknowns_of(L.g, 0);
        L.nu = 0;
        for (int a = 0; a < d->dim; ++a) L.nu += unknowns_of(L.g, face_mask(a));
        if (l > 0) mu *= d->gamma[l] > 0 ? d->gamma[l] : 1.0;
        L.cvu = d->inv_re * (d->decoupled ? mu : 1.0) / (L.g.h * L.g.h);
        L.dec = d->decoupled ? 1 : 0;
    }
    c->singular_p = true;
    for (int a = 0; a < d->dim; ++a)
        if (d->axis_bc[a] == IBB_AXIS_INOUT) c->singular_p = false;
    // first level whose largest colour class fits one workgroup pass budget
    const long long wgmax = d->wg_coarse_max == 0 ? WG_THREADS : d->wg_coarse_max;
    c->lc_u = c->lc_p = MAXLEV;
    if (d->wg_coarse_max >= 0) {
        // the sizes shrink with the level, so the first level that fits starts it
        for (int l = 0; l < c->L; ++l) {
            const Grid &g = c->lv[l].g;
            long long mu = 0;
            for (int a = 0; a < d->dim; ++a) {
                const long long n = unknowns_of(g, face_mask(a));
                mu = n > mu ? n : mu;
            }
            if ((mu + 1) / 2 <= wgmax) { c->lc_u = l; break; }
        }
        for (int l = 0; l < c->L; ++l)
            if ((c->lv[l].np + 1) / 2 <= wgmax) { c->lc_p = l; break; }
    }
    // Galerkin coarse operators: the velocity V-cycles run launched passes
    // down to the coarsest level
    for (int l = 0; l < c->L; ++l) c->lv[l].gal = d->galerkin && l > 0;
    if (d->galerkin) c->lc_u = MAXLEV;
    // tails: the levels below the one-workgroup start level as one matrix,
    // when the level below the start has at most TAIL_MAX unknowns and all
    // levels from there fit the LDS arena of one workgroup (gfx950: 160 KB,
    // less the kernels' own shared data), so that the columns can be built
    // one workgroup each
    for (int v = 0; v < 2; ++v) {
        c->tail[v] = Tail{};
        const int lc = v ? c->lc_u : c->lc_p;
        if (d->coarse_tail < 0 || lc >= c->L - 1) continue;
        const int lt = lc + 1;
        const long long n = v ? c->lv[lt].nu : c->lv[lt].np;
        if (n < 1 || n > TAIL_MAX) continue;
        if (tail_lds_bytes(c, d->precision == IBB_FP32_REFINED, v == 1, lt) > TAIL_LDS_BUDGET) continue;
        c->tail[v].n = (int)n;
        c->tail[v].level = lt;
    }
    // z-blocked colour passes on every 3D level when asked for (measured
    // slower than the flat passes, so not the default)
    for (int l = 0; l < c->L; ++l) c->lv[l].zb = d->dim == 3 && d->smoother_zblock > 0 ? 1 : 0;
    // levels swept with launched passes may use the one-launch red-black
    // sweep: an even number of sweeps per cycle, even periodic extents
    for (int l = 0; l < c->L; ++l) {
        Level &L = c->lv[l];
        bool ok = d->smoother_passes == 1 && !d->decoupled && (d->nu1 + d->nu2) % 2 == 0 && l < c->L - 1 &&
                  l < std::max(c->lc_u, c->lc_p);
        for (int a = 0; a < d->dim; ++a)
            if (d->axis_bc[a] == IBB_AXIS_PERIODIC && L.g.n[a] % 2) ok = false;
        L.fused = ok;
        // the z-marching sweep: velocity levels swept with launched passes
        L.zm = d->smoother_passes == 3 && !d->decoupled && (d->nu1 + d->nu2) % 2 == 0 && l < c->L - 1 &&
               l < c->lc_u && zm_fits(L.g);
    }
    c->eta_max = max_nodes;
    c->m_max = max_springs;
    int nb[3];
    double bs[3];
    bins_for_width(d, d->omega < d->h ? d->omega : d->h, nb, bs);
    c->nbins_cap = nb[0] * nb[1] * nb[2];
    Phys &ph = c->ph;
    ph.sigma = d->sigma;
    ph.eps = d->eps;
    ph.inv_re = d->inv_re;
    ph.force_coef = d->force_coef;
    ph.dt = d->dt;
    for (int a = 0; a < 3; ++a) ph.body_force[a] = a < d->dim ? d->body_force[a] : 0.0;
    ph.rho0 = d->rho0;
    ph.rho_b = d->rho_b;
    ph.d0_pow_d = d->d0_pow_d;
    ph.mu_out = d->mu_out;
    ph.mu_max = d->mu_max;
    ph.omega = d->omega;
    ph.kernel = d->kernel;
}

// views of a level in one precision
template <typename T>
struct View {
    T *xp, *bp, *rp;
    VelArr<T> xu, bu, ru;
    CoefP<T> cp;
    CoefU<T> cu;
};

View<double> view64(Level &L)
{
    View<double> v;
    v.xp = L.xp;
    v.bp = L.bp;
    v.rp = L.rp;
    for (int a = 0; a < 3; ++a) {
        v.xu.c[a] = L.xu[a];
        v.bu.c[a] = L.bu[a];
        v.ru.c[a] = L.ru[a];
        v.cp.beta[a] = L.beta[a];
        v.cu.rho[a] = L.rho[a];
        v.cu.mue[a] = L.mue[a];
    }
    v.cu.muc = L.muc;
    v.cu.dec = L.dec;
    return v;
}

View<float> view32(Level &L)
{
    View<float> v;
    v.xp = L.xp32;
    v.bp = L.bp32;
    v.rp = L.rp32;
    for (int a = 0; a < 3; ++a) {
        v.xu.c[a] = L.xu32[a];
        v.bu.c[a] = L.bu32[a];
        v.ru.c[a] = L.ru32[a];
        v.cp.beta[a] = L.beta32[a];
        v.cu.rho[a] = L.rho32[a];
        v.cu.mue[a] = L.mue32[a];
    }
    v.cu.muc = L.muc32;
    v.cu.dec = L.dec;
    return v;
}

template <typename T>
View<T> view(Level &L);
template <>
View<double> view<double>(Level &L) { return view64(L); }
template <>
View<float> view<float>(Level &L) { return view32(L); }

void vel_masks(int D, int *m)
{
    for (int a = 0; a < 3; ++a) m[a] = a < D ? face_mask(a) : 0;
}

// the two iterate buffers of a level in precision T
template <typename T>
T **cur_x(Level &L, bool vel, int a);
template <>
double **cur_x<double>(Level &L, bool vel, int a) { return vel ? &L.xu[a] : &L.xp; }
template <>
float **cur_x<float>(Level &L, bool vel, int a) { return vel ? &L.xu32[a] : &L.xp32; }
template <typename T>
T **alt_x(Level &L, bool vel, int a);
template <>
double **alt_x<double>(Level &L, bool vel, int a) { return vel ? &L.xu_alt[a] : &L.xp_alt; }
template <>
float **alt_x<float>(Level &L, bool vel, int a) { return vel ? &L.xu32_alt[a] : &L.xp32_alt; }

template <typename T>
GalOpC<T> gal_op(const Level &L);
template <>
GalOpC<double> gal_op<double>(const Level &L) { return GalOpC<double>{{L.gv[0], L.gv[1], L.gv[2]}}; }
template <>
GalOpC<float> gal_op<float>(const Level &L) { return GalOpC<float>{{L.gv32[0], L.gv32[1], L.gv32[2]}}; }
template <typename T>
T **gal_y(Level &L, int a);
template <>
double **gal_y<double>(Level &L, int a) { return &L.gy[a]; }
template <>
float **gal_y<float>(Level &L, int a) { return &L.gy32[a]; }

template <typename T>
void sweep(ibb_ctx *c, bool vel, int l)
{
    Level &L = c->lv[l];
    if (vel && L.gal) {
        // each colour pass writes the second buffer, which then becomes x:
        // two exchanges per component bring every buffer back
        const int cls = prof_class(sizeof(T) == 4 ? PS_GAL_SMOOTH32 : PS_GAL_SMOOTH64, l);
        for (int a = 0; a < c->d.dim; ++a)
            for (int colour = 0; colour < 2; ++colour) {
                View<T> v = view<T>(L);
                const int k = prof_begin(c, cls, unknowns_of(L.g, face_mask(a)) / 2);
                launch_gal_smooth<T>(c->d.dim, L.g, a, colour, gal_op<T>(L), v.bu.c[a], cview(v.xu), *gal_y<T>(L, a),
                                     c->s);
                prof_end(c, k);
                std::swap(*cur_x<T>(L, true, a), *gal_y<T>(L, a));
            }
        return;
    }
    if (vel && L.zm) {
        const T cvu = (T)L.cvu;
        const T mass = (T)(c->d.sigma / c->d.dt);
        const int cls = prof_class(sizeof(T) == 4 ? PS_SMOOTH_RB32 : PS_SMOOTH_RB64, l);
        for (int a = 0; a < c->d.dim; ++a) {
            View<T> v = view<T>(L);
            const int k = prof_begin(c, cls, unknowns_of(L.g, face_mask(a)));
            launch_smooth_zm<T>(L.g, a, cview(v.xu), v.bu.c[a], v.cu, mass, cvu, *alt_x<T>(L, true, a), c->s);
            prof_end(c, k);
            std::swap(*cur_x<T>(L, true, a), *alt_x<T>(L, true, a));
        }
        return;
    }
    if (L.fused && l < (vel ? c->lc_u : c->lc_p)) {
        const T cvp = (T)(1.0 / (L.g.h * L.g.h));
        const T cvu = (T)L.cvu;
        const T mass = (T)(c->d.sigma / c->d.dt);
        const int cls = prof_class(sizeof(T) == 4 ? PS_SMOOTH_RB32 : PS_SMOOTH_RB64, l);
        for (int a = 0; a < (vel ? c->d.dim : 1); ++a) {
            View<T> v = view<T>(L);
            const VelArrC<T> xin = vel ? cview(v.xu) : VelArrC<T>{{v.xp, nullptr, nullptr}};
            const int k = prof_begin(c, cls, unknowns_of(L.g, vel ? face_mask(a) : 0));
            launch_smooth_rb<T>(L.g, vel ? 1 : 0, a, xin, vel ? v.bu.c[a] : v.bp, v.cu, v.cp, mass, vel ? cvu : cvp,
                                *alt_x<T>(L, vel, a), c->s);
            prof_end(c, k);
            std::swap(*cur_x<T>(L, vel, a), *alt_x<T>(L, vel, a));
        }
        return;
    }
    View<T> v = view<T>(L);
    const T cvp = (T)(1.0 / (L.g.h * L.g.h));
    const T cvu = (T)L.cvu;
    const T mass = (T)(c->d.sigma / c->d.dt);
    const int cls = prof_class((vel ? 0 : 1) + (sizeof(T) == 4 ? 2 : 0), l);
    if (vel && L.dec) {
        for (int colour = 0; colour < 2; ++colour) {
            long long units = 0;
            for (int a = 0; a < c->d.dim; ++a) units += unknowns_of(L.g, face_mask(a)) / 2;
            const int k = prof_begin(c, prof_class(sizeof(T) == 4 ? PS_SMOOTH_UDEC32 : PS_SMOOTH_UDEC64, l), units);
            launch_smooth_u_dec<T>(L.g, cview(v.bu), v.xu, v.cu, mass, cvu, colour, c->s);
            prof_end(c, k);
        }
    } else if (vel) {
        for (int a = 0; a < c->d.dim; ++a)
            for (int colour = 0; colour < 2; ++colour) {
                const int k = prof_begin(c, cls, unknowns_of(L.g, face_mask(a)) / 2);
                launch_smooth_u<T>(L.g, a, v.bu.c[a], v.xu, v.cu, mass, cvu, colour, c->s, L.zb);
                prof_end(c, k);
            }
    } else {
        for (int colour = 0; colour < 2; ++colour) {
            const int k = prof_begin(c, cls, L.np / 2);
            launch_smooth_p<T>(L.g, v.bp, v.xp, v.cp, cvp, colour, c->s, L.zb);
            prof_end(c, k);
        }
    }
}

// residual of level l (written to r), optional squared-norm partial sums
template <typename T>
int residual(ibb_ctx *c, bool vel, int l, double *partial)
{
    Level &L = c->lv[l];
    View<T> v = view<T>(L);
    const T cvp = (T)(1.0 / (L.g.h * L.g.h));
    const T cvu = (T)L.cvu;
    const T mass = (T)(c->d.sigma / c->d.dt);
    if (vel && L.gal) {
        // coarse levels only: no norm partials
        const int k = prof_begin(c, prof_class(sizeof(T) == 4 ? PS_GAL_RESID32 : PS_GAL_RESID64, l), L.nu);
        launch_gal_resid<T>(c->d.dim, L.g, gal_op<T>(L), cview(v.bu), cview(v.xu), v.ru, c->s);
        prof_end(c, k);
        return 0;
    }
    const int site = (vel ? PS_RESID_U64 : PS_RESID_P64) + (sizeof(T) == 4 ? 2 : 0);
    const int k = prof_begin(c, prof_class(site, l), vel ? L.nu : L.np);
    const int np = vel ? launch_resid_u<T>(L.g, cview(v.bu), v.xu, v.cu, mass, cvu, v.ru, partial, c->s)
                       : launch_resid_p<T>(L.g, v.bp, v.xp, v.cp, cvp, v.rp, partial, c->s);
    prof_end(c, k);
    return np;
}

// LDS plan of the one-workgroup cycle: the deepest levels whose arrays fit
// the workgroup's LDS budget, laid out level by level
// whether the context's V-cycles in precision prec (0 FP64, 1 FP32) use the
// tail of system vel
bool has_tail(const ibb_ctx *c, int prec, bool vel)
{
    return c->tail[vel ? 1 : 0].n > 0 && prec == (c->d.precision == IBB_FP32_REFINED ? 1 : 0);
}

void clear_plan(std::vector<LdsLevel> &out)
{
    out.assign(WG_MAXLEV, LdsLevel{});
    for (LdsLevel &o : out) {
        for (int a = 0; a < 3; ++a) o.xu[a] = o.bu[a] = o.ru[a] = o.rho[a] = o.beta[a] = o.mue[a] = -1;
        o.xp = o.bp = o.rp = o.muc = -1;
    }
}

// place level l's arrays of one system in the arena from offset *off:
// solver arrays (x only, or x, b and r) and, with coefs, the coefficients
void place_level(const ibb_ctx *c, bool vel, int l, int wsz, bool x_only, bool coefs, LdsLevel &o, int *off)
{
    const int one = arena_array_bytes(c->lv[l].g, wsz);
    auto take = [&]() { const int r = *off; *off += one; return r; };
    if (vel) {
        for (int a = 0; a < c->d.dim; ++a) {
            o.xu[a] = take();
            if (!x_only) {
                o.bu[a] = take();
                o.ru[a] = take();
            }
            if (coefs) o.rho[a] = take();
        }
        if (coefs) {
            o.muc = take();
            for (int e = 0; e < c->E; ++e) o.mue[c->edge_axis[e]] = take();
        }
    } else {
        o.xp = take();
        if (!x_only) {
            o.bp = take();
            o.rp = take();
        }
        if (coefs)
            for (int a = 0; a < c->d.dim; ++a) o.beta[a] = take();
    }
}

// LDS plan of a tail's column build: every level from the tail's level down,
// whole (the tail exists only when they fit)
void plan_tail_build(ibb_ctx *c, bool vel, std::vector<LdsLevel> &out)
{
    clear_plan(out);
    const Tail &t = c->tail[vel ? 1 : 0];
    const int wsz = c->d.precision == IBB_FP32_REFINED ? 4 : 8;
    int off = 0;
    for (int l = t.level; l < c->L; ++l) place_level(c, vel, l, wsz, false, true, out[l], &off);
    c->tplan_bytes[vel ? 1 : 0] = off;
}

void plan_lds(ibb_ctx *c, int prec, bool vel, std::vector<LdsLevel> &out)
{
    const int wsz = prec ? 4 : 8;
    const int D = c->d.dim;
    const int lc = std::min(vel ? c->lc_u : c->lc_p, c->L - 1);
    const int budget = wg_lds_budget();
    clear_plan(out);
    if (has_tail(c, prec, vel)) {
        // the cycle works on the start level and writes the tail level's
        // iterate: stage the start level whole, or its solver arrays, and
        // the tail level's x
        const int lt = c->tail[vel ? 1 : 0].level;
        const int nsolve = vel ? 3 * D : 3, ncoef = vel ? D + 1 + c->E : D;
        const long long one = arena_array_bytes(c->lv[lc].g, wsz);
        const long long xt = (long long)arena_array_bytes(c->lv[lt].g, wsz) * (vel ? D : 1);
        int off = 0;
        int ls = lt;
        if (one * (nsolve + ncoef) + xt <= budget) {
            place_level(c, vel, lc, wsz, false, true, out[lc], &off);
            ls = lc;
        } else if (one * nsolve + xt <= budget) {
            place_level(c, vel, lc, wsz, false, false, out[lc], &off);
            ls = lc;
        }
        if (xt <= budget) place_level(c, vel, lt, wsz, true, false, out[lt], &off);
        else ls = c->L;
        c->lds_ls[prec][vel ? 1 : 0] = ls;
        c->lds_bytes[prec][vel ? 1 : 0] = off;
        return;
    }
    // bytes of one level's arrays in this system: solver arrays (x, b, r)
    // and coefficients
    auto one_bytes = [&](int l) { return ((c->lv[l].g.nel * wsz + 15) / 16) * 16; };
    const int nsolve = vel ? 3 * D : 3, ncoef = vel ? D + 1 + c->E : D;
    // the levels below the start level, deepest first, while they fit
    int ls = c->L;
    long long total = 0;
    for (int l = c->L - 1; l > lc; --l) {
        const long long b = one_bytes(l) * (nsolve + ncoef);
        if (total + b > budget) break;
        total += b;
        ls = l;
    }
    // then the start level, whole or its solver arrays alone, when
    // everything below it is staged
    bool start_coefs = false;
    if (ls == lc + 1) {
        if (total + one_bytes(lc) * (nsolve + ncoef) <= budget) {
            ls = lc;
            start_coefs = true;
        } else if (total + one_bytes(lc) * nsolve <= budget) {
            ls = lc;
        }
    }
    int off = 0;
    for (int l = ls; l < c->L; ++l) {
        const int one = (int)one_bytes(l);
        const bool coefs = l > lc || start_coefs;
        LdsLevel &o = out[l];
        auto take = [&]() { const int r = off; off += one; return r; };
        if (vel) {
            for (int a = 0; a < D; ++a) {
                o.xu[a] = take();
                o.bu[a] = take();
                o.ru[a] = take();
                if (coefs) o.rho[a] = take();
            }
            if (coefs) {
                o.muc = take();
                for (int e = 0; e < c->E; ++e) o.mue[c->edge_axis[e]] = take();
            }
        } else {
            o.xp = take();
            o.bp = take();
            o.rp = take();
            if (coefs)
                for (int a = 0; a < D; ++a) o.beta[a] = take();
        }
    }
    c->lds_ls[prec][vel ? 1 : 0] = ls;
    c->lds_bytes[prec][vel ? 1 : 0] = off;
}

LdsPlan lds_plan(ibb_ctx *c, int prec, bool vel)
{
    const int v = vel ? 1 : 0;
    return LdsPlan{c->ldslev[prec][v], c->lds_ls[prec][v], c->lds_bytes[prec][v]};
}

template <typename T>
const LevTab<T> *level_table(ibb_ctx *c);
template <>
const LevTab<double> *level_table<double>(ibb_ctx *c) { return c->tab64; }
template <>
const LevTab<float> *level_table<float>(ibb_ctx *c) { return c->tab32; }

template <typename T>
void vcycle(ibb_ctx *c, bool vel, int l)
{
    Level &L = c->lv[l];
    const int D = c->d.dim;
    int vm[3];
    vel_masks(D, vm);
    const int pm[3] = {0, 0, 0};
    if (l >= (vel ? c->lc_u : c->lc_p)) {
        Level &LC = c->lv[c->L - 1];
        const long long nc = vel ? LC.nu : LC.np;
        const int ndense = nc <= DENSE_MAX ? (int)nc : 0;
        Timed t(c, (vel ? PS_COARSE_U64 : PS_COARSE_P64) + (sizeof(T) == 4 ? 2 : 0), l, vel ? L.nu : L.np);
        const int prec = sizeof(T) == 4 ? 1 : 0;
        launch_coarse_vcycle<T>(D, level_table<T>(c), l, c->L, vel ? 1 : 0, c->d.nu1, c->d.nu2, ndense,
                                vel ? c->uidx_u : c->uidx_p, vel ? c->ucomp_u : c->ucomp_p, vel ? c->Mu : c->Mp,
                                lds_plan(c, prec, vel), has_tail(c, prec, vel) ? c->tail[vel ? 1 : 0] : Tail{},
                                c->s);
        return;
    }
    View<T> v = view<T>(L);
    if (l == c->L - 1) {
        const long long n = vel ? L.nu : L.np;
        if (n <= DENSE_MAX) {
            Timed t(c, PS_DENSE, l, n);
            if (vel) launch_dense_apply<T>(L.g, 1, (int)n, c->uidx_u, c->ucomp_u, c->Mu, cview(v.bu), v.xu, c->s);
            else {
                VelArr<T> x{{v.xp, nullptr, nullptr}};
                VelArrC<T> b{{v.bp, nullptr, nullptr}};
                launch_dense_apply<T>(L.g, 0, (int)n, c->uidx_p, c->ucomp_p, c->Mp, b, x, c->s);
            }
        } else {
            for (int s = 0; s < c->d.nu1 + c->d.nu2; ++s) sweep<T>(c, vel, l);
        }
        return;
    }
    for (int s = 0; s < c->d.nu1; ++s) sweep<T>(c, vel, l);
    residual<T>(c, vel, l, nullptr);
    Level &C = c->lv[l + 1];
    View<T> w = view<T>(C);
    const int rsite = sizeof(T) == 4 ? PS_RESTRICT32 : PS_RESTRICT64;
    if (vel) {
        Timed t(c, rsite, l + 1, C.nu);
        launch_restrict<T>(L.g, C.g, D, vm, ROLE_V, false, cview(v.ru), w.bu, (T)1, c->s, &w.xu);
    } else {
        VelArrC<T> rf{{v.rp, nullptr, nullptr}};
        VelArr<T> bc{{w.bp, nullptr, nullptr}};
        VelArr<T> xc{{w.xp, nullptr, nullptr}};
        Timed t(c, rsite, l + 1, C.np);
        launch_restrict<T>(L.g, C.g, 1, pm, ROLE_P, false, rf, bc, (T)1, c->s, &xc);
    }
    vcycle<T>(c, vel, l + 1);
    // the one-launch sweep alternates a level's iterate buffers: look them up again
    v = view<T>(L);
    w = view<T>(C);
    const int psite = sizeof(T) == 4 ? PS_PROLONG32 : PS_PROLONG64;
    if (vel) {
        Timed t(c, psite, l, L.nu);
        launch_prolong_add<T>(C.g, L.g, D, vm, ROLE_V, cview(w.xu), v.xu, c->s);
    } else {
        VelArrC<T> xc{{w.xp, nullptr, nullptr}};
        VelArr<T> xf{{v.xp, nullptr, nullptr}};
        Timed t(c, psite, l, L.np);
        launch_prolong_add<T>(C.g, L.g, 1, pm, ROLE_P, xc, xf, c->s);
    }
    for (int s = 0; s < c->d.nu2; ++s) sweep<T>(c, vel, l);
}

// the reduced scalar back on the host
ibb_status fetch_scalar(ibb_ctx *c, double *out)
{
    HIPCHK(hipMemcpyAsync(out, c->scalar, sizeof(double), hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipStreamSynchronize(c->s));
    return IBB_OK;
}

ibb_status read_scalar(ibb_ctx *c, int nparts, double *out)
{
    {
        Timed t(c, PS_OUTER, 0, nparts);
        launch_reduce_final(c->partial, nparts, c->scalar, c->s);
    }
    return fetch_scalar(c, out);
}

// Capture launch() -- kernels only, no memset and no copy -- into *slot
// (once), on the private stream: the launch helpers use c->s, which points
// there while the capture runs.
template <typename F>
ibb_status ensure_graph(ibb_ctx *c, hipGraphExec_t *slot, F launch)
{
    if (*slot) return IBB_OK;
    if (!c->cap) HIPCHK(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    hipStream_t user = c->s;
    HIPCHK(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    c->s = c->cap;
    launch();
    c->s = user;
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamEndCapture(c->cap, &graph));
    const hipError_t e = hipGraphInstantiate(slot, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        *slot = nullptr;
        c->err = std::string("hipGraphInstantiate: ") + hipGetErrorString(e);
        return IBB_EDEVICE;
    }
    return IBB_OK;
}

// replay a captured iteration and read the squared norm it reduced
ibb_status replay_norm(ibb_ctx *c, hipGraphExec_t exec, double *rn)
{
    HIPCHK(hipGraphLaunch(exec, c->s));
    double s2;
    const ibb_status e = fetch_scalar(c, &s2);
    *rn = sqrt(s2);
    return e;
}

// ||b|| over the unknowns of level 0 (FP64)
ibb_status norm_b(ibb_ctx *c, bool vel, double *out)
{
    Level &L = c->lv[0];
    int vm[3];
    vel_masks(c->d.dim, vm);
    const int pm[3] = {0, 0, 0};
    int np;
    {
        Timed t(c, PS_OUTER, 0, vel ? L.nu : L.np);
        if (vel) np = launch_norm2<double>(L.g, c->d.dim, vm, VelArrC<double>{{L.bu[0], L.bu[1], L.bu[2]}}, c->partial, c->s);
        else np = launch_norm2<double>(L.g, 1, pm, VelArrC<double>{{L.bp, nullptr, nullptr}}, c->partial, c->s);
    }
    double s2;
    ibb_status st = read_scalar(c, np, &s2);
    *out = sqrt(s2);
    return st;
}

ibb_status resid_norm(ibb_ctx *c, bool vel, double *out)
{
    const int np = residual<double>(c, vel, 0, c->partial);
    double s2;
    ibb_status st = read_scalar(c, np, &s2);
    *out = sqrt(s2);
    return st;
}

void zero_unknowns(ibb_ctx *c, bool vel)
{
    Level &L = c->lv[0];
    const int D = c->d.dim;
    int vm[3];
    vel_masks(D, vm);
    const int pm[3] = {0, 0, 0};
    if (vel)
        launch_load_unknowns<double>(L.g, D, vm, VelArrC<double>{{nullptr, nullptr, nullptr}},
                                     VelArr<double>{{L.xu[0], L.xu[1], L.xu[2]}}, c->s);
    else
        launch_load_unknowns<double>(L.g, 1, pm, VelArrC<double>{{nullptr, nullptr, nullptr}},
                                     VelArr<double>{{L.xp, nullptr, nullptr}}, c->s);
}

struct SolveOut {
    int status = IBB_OK;
    int cycles = 0;
    int vcycles = 0;
    double relres = 0.0;
};

// component views of the GCR arrays for one system
struct GView {
    VelArr<double> b, x, r;
};

GView gcr_view(ibb_ctx *c, bool vel)
{
    GView v;
    const int nc = vel ? c->d.dim : 1;
    for (int a = 0; a < 3; ++a) {
        v.b.c[a] = a < nc ? c->gb[a] : nullptr;
        v.x.c[a] = a < nc ? c->gx[a] : nullptr;
        v.r.c[a] = a < nc ? c->gr[a] : nullptr;
    }
    return v;
}

VelArr<double> gcr_dir(ibb_ctx *c, bool vel, bool q, int j)
{
    VelArr<double> v{{nullptr, nullptr, nullptr}};
    const int nc = vel ? c->d.dim : 1;
    for (int a = 0; a < nc; ++a) v.c[a] = q ? c->gq[3 * j + a] : c->gz[3 * j + a];
    return v;
}

// dot product of two finest-level fields over the unknowns into gs[slot]
void gcr_dot(ibb_ctx *c, bool vel, const VelArr<double> &x, const VelArr<double> &y, int slot)
{
    const int np = launch_dot(c->lv[0].g, vel ? 1 : 0, cview(x), cview(y), c->partial, c->s);
    launch_reduce_final(c->partial, np, c->gs + slot, c->s);
}

// b - A x for the GCR iterate, its squared norm back on the host
// b - A x for the GCR iterate and its squared norm reduced into c->scalar
void gcr_residual_launch(ibb_ctx *c, bool vel, const GView &g)
{
    Level &L = c->lv[0];
    View<double> v = view64(L);
    const double cvp = 1.0 / (L.g.h * L.g.h), cvu = L.cvu, mass = c->d.sigma / c->d.dt;
    int np;
    if (vel) np = launch_resid_u<double>(L.g, cview(g.b), g.x, v.cu, mass, cvu, g.r, c->partial, c->s);
    else np = launch_resid_p<double>(L.g, g.b.c[0], g.x.c[0], v.cp, cvp, g.r.c[0], c->partial, c->s);
    launch_reduce_final(c->partial, np, c->scalar, c->s);
}

ibb_status gcr_residual(ibb_ctx *c, bool vel, const GView &g, double *rn)
{
    gcr_residual_launch(c, vel, g);
    double s2;
    ibb_status st = fetch_scalar(c, &s2);
    *rn = sqrt(s2);
    return st;
}

// V-cycle-preconditioned GCR(m) on the finest level (b and x in the level-0
// arrays on entry; x there on return).  Same stopping test as the V-cycle
// loop below; exact > 0 runs exactly that many iterations.  The solve is cut
// into resumable pieces so that a group can advance several such solves in
// lock step, each on its own stream: begin, then while more: launch, the
// norm back on the host, account; then finish.
struct GcrRun {
    ibb_ctx *c = nullptr;
    bool vel = false;
    int max_cycles = 0, exact = 0;
    SolveOut *o = nullptr;
    double nb = 0.0, rel = 0.0;
    int j = 0;          // position in the restart window
    bool done = false;  // stopping test met (or nothing to solve)
};

// one iteration at window position j: z = M r, q = A z made orthogonal to
// the stored q_i, x += alpha z, then the fresh residual with its squared
// norm reduced into c->scalar (kernels only)
void gcr_iteration_launches(ibb_ctx *c, bool vel, int j)
{
    const bool refined = c->d.precision == IBB_FP32_REFINED;
    const int m = c->d.krylov_restart;
    int vm[3];
    vel_masks(c->d.dim, vm);
    const int pm[3] = {0, 0, 0};
    const int *masks = vel ? vm : pm;
    const int nc = vel ? c->d.dim : 1;
    Level &L0 = c->lv[0];
    View<double> v = view64(L0);
    View<float> w = view32(L0);
    VelArr<double> bl = vel ? v.bu : VelArr<double>{{v.bp, nullptr, nullptr}};
    VelArr<double> xl = vel ? v.xu : VelArr<double>{{v.xp, nullptr, nullptr}};
    VelArr<float> bl32 = vel ? w.bu : VelArr<float>{{w.bp, nullptr, nullptr}};
    VelArr<float> xl32 = vel ? w.xu : VelArr<float>{{w.xp, nullptr, nullptr}};
    const GView g = gcr_view(c, vel);
    const double cvp = 1.0 / (L0.g.h * L0.g.h), cvu = L0.cvu, mass = c->d.sigma / c->d.dt;
    const int SLOT_T = m, SLOT_RQ = m + 1;
    const VelArr<double> z = gcr_dir(c, vel, false, j), q = gcr_dir(c, vel, true, j);
    // z = M r: V-cycles from zero on A z = r in the level-0 arrays
    for (int a = 0; a < nc; ++a) launch_fill<double>(z.c[a], L0.g.nel, 0.0, c->s);
    if (!refined) {
        for (int a = 0; a < nc; ++a) launch_fill<double>(xl.c[a], L0.g.nel, 0.0, c->s);
        launch_load_unknowns<double>(L0.g, nc, masks, cview(g.r), bl, c->s);
        vcycle<double>(c, vel, 0);
        launch_load_unknowns<double>(L0.g, nc, masks, cview(xl), z, c->s);
    } else {
        for (int a = 0; a < nc; ++a) launch_fill<float>(xl32.c[a], L0.g.nel, 0.0f, c->s);
        launch_cast_unknowns<double, float>(L0.g, nc, masks, cview(g.r), bl32, c->s);
        for (int it = 0; it < c->d.inner_cycles; ++it) vcycle<float>(c, vel, 0);
        launch_add_correction(L0.g, nc, masks, cview(xl32), z, c->s);
    }
    // q = A z, then orthogonal to the stored q_i (modified Gram-Schmidt)
    launch_apply(L0.g, vel ? 1 : 0, z, v.cp, v.cu, mass, vel ? cvu : cvp, q, c->s);
    for (int i = 0; i < j; ++i) {
        const VelArr<double> zi = gcr_dir(c, vel, false, i), qi = gcr_dir(c, vel, true, i);
        gcr_dot(c, vel, q, qi, SLOT_T);
        launch_gcr_axpy2(L0.g, vel ? 1 : 0, c->gs + SLOT_T, c->gs + i, cview(qi), cview(zi), q, z, c->s);
    }
    gcr_dot(c, vel, q, q, j);
    gcr_dot(c, vel, g.r, q, SLOT_RQ);
    launch_gcr_update(L0.g, vel ? 1 : 0, c->gs + SLOT_RQ, c->gs + j, cview(z), g.x, c->s);
    gcr_residual_launch(c, vel, g);
}

// ||b||, the solve's own copies of b and x, the first residual (syncs c->s)
ibb_status gcr_begin(GcrRun &R)
{
    ibb_ctx *c = R.c;
    const bool vel = R.vel;
    int vm[3];
    vel_masks(c->d.dim, vm);
    const int pm[3] = {0, 0, 0};
    const int *masks = vel ? vm : pm;
    const int nc = vel ? c->d.dim : 1;
    Level &L0 = c->lv[0];
    View<double> v = view64(L0);
    VelArr<double> bl = vel ? v.bu : VelArr<double>{{v.bp, nullptr, nullptr}};
    VelArr<double> xl = vel ? v.xu : VelArr<double>{{v.xp, nullptr, nullptr}};
    const GView g = gcr_view(c, vel);
    ibb_status st = norm_b(c, vel, &R.nb);
    if (st) return st;
    R.o->cycles = R.o->vcycles = 0;
    R.o->relres = 0.0;
    R.o->status = IBB_OK;
    R.j = 0;
    R.rel = 0.0;
    R.done = false;
    if (R.nb == 0.0) {
        zero_unknowns(c, vel);
        R.done = true;
        return IBB_OK;
    }
    for (int a = 0; a < nc; ++a) {
        launch_fill<double>(g.b.c[a], L0.g.nel, 0.0, c->s);
        launch_fill<double>(g.x.c[a], L0.g.nel, 0.0, c->s);
    }
    launch_load_unknowns<double>(L0.g, nc, masks, cview(bl), g.b, c->s);
    launch_load_unknowns<double>(L0.g, nc, masks, cview(xl), g.x, c->s);
    double rn;
    if ((st = gcr_residual(c, vel, g, &rn))) return st;
    R.rel = rn / R.nb;
    return IBB_OK;
}

// whether another iteration is due (the stopping test; records the outcome)
bool gcr_more(GcrRun &R)
{
    if (R.done) return false;
    SolveOut *o = R.o;
    if (R.exact > 0) {
        if (o->cycles >= R.exact) R.done = true;
    } else if (R.rel <= R.c->d.rtol) {
        R.done = true;
    } else if (!(R.rel == R.rel) || isinf(R.rel)) {
        o->status = IBB_ENUMERIC;
        R.done = true;
    } else if (o->cycles >= R.max_cycles) {
        o->status = IBB_ENOCONV;
        R.done = true;
    }
    return !R.done;
}

// launch the next iteration on c->s: a graph replay (captured once per
// window position), or kernel by kernel while kernel timing is on
ibb_status gcr_launch(GcrRun &R)
{
    ibb_ctx *c = R.c;
    const bool vel = R.vel;
    const int j = R.j;
    R.o->vcycles += c->d.precision == IBB_FP32_REFINED ? c->d.inner_cycles : 1;
    if (c->prof) {
        gcr_iteration_launches(c, vel, j);
        return IBB_OK;
    }
    std::vector<hipGraphExec_t> &gt = c->gtick[vel ? 1 : 0];
    if ((int)gt.size() < c->d.krylov_restart) gt.assign(c->d.krylov_restart, nullptr);
    ibb_status st = ensure_graph(c, &gt[j], [&]() { gcr_iteration_launches(c, vel, j); });
    if (st) return st;
    HIPCHK(hipGraphLaunch(gt[j], c->s));
    return IBB_OK;
}

void gcr_account(GcrRun &R, double rn)
{
    R.rel = rn / R.nb;
    R.o->cycles++;
    R.j = R.j + 1 == R.c->d.krylov_restart ? 0 : R.j + 1;
}

// the iterate back into the level-0 arrays, b restored
void gcr_finish(GcrRun &R)
{
    ibb_ctx *c = R.c;
    const bool vel = R.vel;
    R.o->relres = R.rel;
    if (R.nb == 0.0) return;
    int vm[3];
    vel_masks(c->d.dim, vm);
    const int pm[3] = {0, 0, 0};
    const int *masks = vel ? vm : pm;
    const int nc = vel ? c->d.dim : 1;
    Level &L0 = c->lv[0];
    View<double> v = view64(L0);
    VelArr<double> bl = vel ? v.bu : VelArr<double>{{v.bp, nullptr, nullptr}};
    VelArr<double> xl = vel ? v.xu : VelArr<double>{{v.xp, nullptr, nullptr}};
    const GView g = gcr_view(c, vel);
    launch_load_unknowns<double>(L0.g, nc, masks, cview(g.x), xl, c->s);
    launch_load_unknowns<double>(L0.g, nc, masks, cview(g.b), bl, c->s);
}

ibb_status solve_gcr(ibb_ctx *c, bool vel, int max_cycles, int exact, SolveOut *o)
{
    GcrRun R;
    R.c = c;
    R.vel = vel;
    R.max_cycles = max_cycles;
    R.exact = exact;
    R.o = o;
    ibb_status st = gcr_begin(R);
    if (st) return st;
    while (gcr_more(R)) {
        if ((st = gcr_launch(R))) return st;
        double s2;
        if ((st = fetch_scalar(c, &s2))) return st;
        gcr_account(R, sqrt(s2));
    }
    gcr_finish(R);
    return IBB_OK;
}

// V-cycles on level 0 arrays (b and x already in place)
ibb_status solve(ibb_ctx *c, bool vel, int max_cycles, int exact, SolveOut *o)
{
    if (c->d.krylov_restart > 0) return solve_gcr(c, vel, max_cycles, exact, o);
    const bool refined = c->d.precision == IBB_FP32_REFINED;
    const int D = c->d.dim;
    int vm[3];
    vel_masks(D, vm);
    const int pm[3] = {0, 0, 0};
    Level &L0 = c->lv[0];
    double nb;
    ibb_status st = norm_b(c, vel, &nb);
    if (st) return st;
    o->cycles = o->vcycles = 0;
    o->relres = 0.0;
    o->status = IBB_OK;
    if (nb == 0.0) {
        zero_unknowns(c, vel);
        return IBB_OK;
    }
    double rn;
    auto one_iteration = [&]() {
        if (!refined) {
            vcycle<double>(c, vel, 0);
            return;
        }
        // r64 already holds b - A x (from the last residual evaluation)
        const long long units = vel ? L0.nu : L0.np;
        {
            Timed t(c, PS_OUTER, 0, units);
            if (vel)
                launch_inner_start(L0.g, D, vm, VelArrC<double>{{L0.ru[0], L0.ru[1], L0.ru[2]}},
                                   VelArr<float>{{L0.bu32[0], L0.bu32[1], L0.bu32[2]}},
                                   VelArr<float>{{L0.xu32[0], L0.xu32[1], L0.xu32[2]}}, c->s);
            else
                launch_inner_start(L0.g, 1, pm, VelArrC<double>{{L0.rp, nullptr, nullptr}},
                                   VelArr<float>{{L0.bp32, nullptr, nullptr}},
                                   VelArr<float>{{L0.xp32, nullptr, nullptr}}, c->s);
        }
        for (int it = 0; it < c->d.inner_cycles; ++it) vcycle<float>(c, vel, 0);
        Timed t(c, PS_OUTER, 0, units);
        if (vel)
            launch_add_correction(L0.g, D, vm, VelArrC<float>{{L0.xu32[0], L0.xu32[1], L0.xu32[2]}},
                                  VelArr<double>{{L0.xu[0], L0.xu[1], L0.xu[2]}}, c->s);
        else
            launch_add_correction(L0.g, 1, pm, VelArrC<float>{{L0.xp32, nullptr, nullptr}},
                                  VelArr<double>{{L0.xp, nullptr, nullptr}}, c->s);
    };
    // Without kernel timing an iteration is one graph launch: the same
    // kernels in the same order as the launches below, so the same bits.
    const bool graph = !c->prof;
    if (graph) {
        st = ensure_graph(c, &c->tick[vel ? 1 : 0], [&]() {
            one_iteration();
            const int np = residual<double>(c, vel, 0, c->partial);
            launch_reduce_final(c->partial, np, c->scalar, c->s);
        });
        if (st) return st;
    }
    auto iterate = [&](double *r) -> ibb_status {
        o->vcycles += refined ? c->d.inner_cycles : 1;
        if (!graph) {
            one_iteration();
            return resid_norm(c, vel, r);
        }
        return replay_norm(c, c->tick[vel ? 1 : 0], r);
    };
    if ((st = resid_norm(c, vel, &rn))) return st;
    double rel = rn / nb;
    if (exact > 0) {
        for (int k = 0; k < exact; ++k) {
            if ((st = iterate(&rn))) return st;
            o->cycles++;
        }
        o->relres = rn / nb;
        return IBB_OK;
    }
    while (!(rel <= c->d.rtol)) {
        if (!(rel == rel) || isinf(rel)) { o->status = IBB_ENUMERIC; break; }
        if (o->cycles >= max_cycles) { o->status = IBB_ENOCONV; break; }
        if ((st = iterate(&rn))) return st;
        o->cycles++;
        prof_flush(c);
        rel = rn / nb;
    }
    o->relres = rel;
    prof_flush(c);
    return IBB_OK;
}

// unknowns of level l of one system in the order comp, z, y, x: padded
// index and component
void level_unknowns(ibb_ctx *c, int l, bool vel, std::vector<long long> &idx, std::vector<int> &cmp)
{
    Level &L = c->lv[l];
    idx.clear();
    cmp.clear();
    for (int a = 0; a < (vel ? c->d.dim : 1); ++a) {
        const int vmask = vel ? face_mask(a) : 0;
        int lo[3], hi[3];
        for (int d = 0; d < 3; ++d) unk_range(L.g, d, (vmask >> d) & 1, lo[d], hi[d]);
        for (int k = lo[2]; k <= hi[2]; ++k)
            for (int j = lo[1]; j <= hi[1]; ++j)
                for (int i = lo[0]; i <= hi[0]; ++i) {
                    idx.push_back(at(L.g, i, j, k));
                    cmp.push_back(a);
                }
    }
}

// host-side table of coarsest unknowns in the order comp, z, y, x
void coarsest_tables(ibb_ctx *c, std::vector<long long> &ip, std::vector<int> &cp, std::vector<long long> &iu,
                     std::vector<int> &cu)
{
    Level &L = c->lv[c->L - 1];
    auto add = [&](int vmask, int comp, std::vector<long long> &idx, std::vector<int> &cmp) {
        int lo[3], hi[3];
        for (int d = 0; d < 3; ++d) unk_range(L.g, d, (vmask >> d) & 1, lo[d], hi[d]);
        for (int k = lo[2]; k <= hi[2]; ++k)
            for (int j = lo[1]; j <= hi[1]; ++j)
                for (int i = lo[0]; i <= hi[0]; ++i) {
                    idx.push_back(at(L.g, i, j, k));
                    cmp.push_back(comp);
                }
    };
    add(0, 0, ip, cp);
    for (int a = 0; a < c->d.dim; ++a) add(face_mask(a), a, iu, cu);
}

// spread, coarse coefficients, FP32 copies, coarsest inverses
ibb_status rebuild_coefficients(ibb_ctx *c)
{
    const ibb_desc *d = &c->d;
    const int D = d->dim;
    Level &L0 = c->lv[0];
    const long long em = c->eta_max > 0 ? c->eta_max : 1;
    // spring forces at the current positions
    for (int a = 0; a < D; ++a) launch_fill<double>(c->F + a * em, em, 0.0, c->s);
    if (c->have_springs && c->m > 0) {
        Timed t(c, PS_SPRING_FORCE, 0, c->eta);
        launch_spring_force(L0.g, c->X, em, c->eta, c->ij, c->m, c->rest, c->K, c->alive, c->inc_start, c->inc_list,
                            c->F, c->s);
    }
    // bins at width omega, then the gathers
    Bins b = c->bins;
    bins_for_width(d, d->omega, b.nb, b.bs);
    b.nbins = b.nb[0] * b.nb[1] * b.nb[2];
    launch_bin_nodes(L0.g, b, c->X, em, c->eta, c->scan_tmp, c->s);
    for (int a = 0; a < D; ++a) {
        Timed t(c, PS_SPREAD_FACE, 0, lattice_count(L0.g, face_mask(a)));
        launch_spread_face(L0.g, c->ph, b, c->X, c->F, em, a, d->omega, c->f[a], L0.rho[a], c->s);
    }
    // with constant viscosity (eq:NSdis1) no row reads the viscosity fields,
    // which keep the fluid value they were created with
    const bool visc = !d->decoupled;
    if (visc) {
        {
            Timed t(c, PS_SPREAD_VISC, 0, lattice_count(L0.g, 0));
            launch_spread_visc(L0.g, c->ph, b, c->X, em, 0, L0.muc, c->s);
        }
        for (int e = 0; e < c->E; ++e) {
            Timed t(c, PS_SPREAD_VISC, 0, lattice_count(L0.g, edge_mask(D, c->edge_axis[e])));
            launch_spread_visc(L0.g, c->ph, b, c->X, em, edge_mask(D, c->edge_axis[e]), L0.mue[c->edge_axis[e]],
                               c->s);
        }
    }
    // coarse levels: full weighting of rho, mu (times gamma)
    int fm[3], em3[3];
    vel_masks(D, fm);
    for (int e = 0; e < 3; ++e) em3[e] = e < c->E ? edge_mask(D, c->edge_axis[e]) : 0;
    const int cm[3] = {0, 0, 0};
    for (int l = 0; l < c->L; ++l) {
        Level &L = c->lv[l];
        if (l > 0) {
            Level &F = c->lv[l - 1];
            const double gm = d->gamma[l] > 0 ? d->gamma[l] : 1.0;
            launch_restrict<double>(F.g, L.g, D, fm, ROLE_C, true, VelArrC<double>{{F.rho[0], F.rho[1], F.rho[2]}},
                                    VelArr<double>{{L.rho[0], L.rho[1], L.rho[2]}}, 1.0, c->s);
            if (visc) {
                launch_restrict<double>(F.g, L.g, 1, cm, ROLE_C, true, VelArrC<double>{{F.muc, nullptr, nullptr}},
                                        VelArr<double>{{L.muc, nullptr, nullptr}}, gm, c->s);
                VelArrC<double> fe{{nullptr, nullptr, nullptr}};
                VelArr<double> ce{{nullptr, nullptr, nullptr}};
                for (int e = 0; e < c->E; ++e) {
                    fe.c[e] = F.mue[c->edge_axis[e]];
                    ce.c[e] = L.mue[c->edge_axis[e]];
                }
                launch_restrict<double>(F.g, L.g, c->E, em3, ROLE_C, true, fe, ce, gm, c->s);
            }
        }
        // beta, then the ghost layers of every coefficient, then the FP32
        // copies: one launch each, over all of the level's arrays
        launch_beta_faces(L.g, VelArrC<double>{{L.rho[0], L.rho[1], L.rho[2]}},
                          VelArr<double>{{L.beta[0], L.beta[1], L.beta[2]}}, c->s);
        CoefSet<double> set;
        set.n = 0;
        float *set32[COEF_SET];
        auto add = [&](int vmask, double *v, float *v32) {
            set.vmask[set.n] = vmask;
            set.v[set.n] = v;
            set32[set.n++] = v32;
        };
        for (int a = 0; a < D; ++a) {
            add(face_mask(a), L.rho[a], L.rho32[a]);
            add(face_mask(a), L.beta[a], L.beta32[a]);
        }
        if (visc) {
            add(0, L.muc, L.muc32);
            for (int e = 0; e < c->E; ++e)
                add(edge_mask(D, c->edge_axis[e]), L.mue[c->edge_axis[e]], L.mue32[c->edge_axis[e]]);
        }
        launch_coef_ghosts<double>(L.g, set, c->s);
        if (d->precision == IBB_FP32_REFINED) launch_to_f32(set, set32, L.g.nel, c->s);
    }
    // Galerkin operators of the viscous system, level by level from the
    // finest (Sec. "Numerical Concerns"), with their FP32 copies
    if (d->galerkin) {
        launch_fill<int>(c->gal_err, 1, 0, c->s);
        for (int l = 1; l < c->L; ++l) {
            Level &F = c->lv[l - 1], &L = c->lv[l];
            const GalOpC<double> fine = gal_op<double>(F);
            Timed t(c, PS_GAL_BUILD, l, L.nu);
            launch_gal_build(D, F.g, L.g, view64(F).cu, d->sigma / d->dt, F.cvu, l > 1 ? &fine : nullptr,
                             GalOp<double>{{L.gv[0], L.gv[1], L.gv[2]}}, c->gal_err, c->s);
            if (d->precision == IBB_FP32_REFINED)
                launch_gal_to_f32(D, L.g, gal_op<double>(L), GalOp<float>{{L.gv32[0], L.gv32[1], L.gv32[2]}}, c->s);
        }
        int bad = 0;
        HIPCHK(hipMemcpyAsync(&bad, c->gal_err, sizeof(int), hipMemcpyDeviceToHost, c->s));
        HIPCHK(hipStreamSynchronize(c->s));
        if (bad) return fail(c, IBB_EINVAL, "a Galerkin coarse-operator entry falls outside its stencil box");
    }
    // coarsest inverses
    Level &LC = c->lv[c->L - 1];
    const double hc2 = LC.g.h * LC.g.h;
    View<double> v = view64(LC);
    if (LC.np <= DENSE_MAX)
        launch_dense_inverse(LC.g, 0, (int)LC.np, c->uidx_p, c->ucomp_p, v.cp, v.cu, d->sigma / d->dt, 1.0 / hc2,
                             c->Atmp, c->singular_p ? 1 : 0, c->Aw, c->Mp, c->s);
    if (LC.nu <= DENSE_MAX) {
        if (LC.gal)
            launch_gal_dense_inverse(D, LC.g, (int)LC.nu, c->uidx_u, c->ucomp_u, gal_op<double>(LC), c->Aw, c->Mu,
                                     c->s);
        else
            launch_dense_inverse(LC.g, 1, (int)LC.nu, c->uidx_u, c->ucomp_u, v.cp, v.cu, d->sigma / d->dt,
                                 LC.cvu, c->Atmp, 0, c->Aw, c->Mu, c->s);
    }
    // tails on the new coefficients (and the new coarsest inverses)
    for (int s = 0; s < 2; ++s) {
        const Tail &t = c->tail[s];
        if (t.n <= 0) continue;
        const LdsPlan tp{c->tplan[s], t.level, c->tplan_bytes[s]};
        const long long nc = s ? LC.nu : LC.np;
        const int ndense = nc <= DENSE_MAX ? (int)nc : 0;
        const long long *ui = s ? c->uidx_u : c->uidx_p;
        const int *uc = s ? c->ucomp_u : c->ucomp_p;
        const double *M = s ? c->Mu : c->Mp;
        if (d->precision == IBB_FP32_REFINED)
            launch_tail_columns<float>(D, c->tab32, c->L, s, d->nu1, d->nu2, ndense, ui, uc, M, tp, t, c->s);
        else
            launch_tail_columns<double>(D, c->tab64, c->L, s, d->nu1, d->nu2, ndense, ui, uc, M, tp, t, c->s);
    }
    c->have_coefs = true;
    return IBB_OK;
}

ibb_status remove_cell_mean(ibb_ctx *c, double *v)
{
    Level &L0 = c->lv[0];
    const int np = launch_sum_cells(L0.g, v, c->partial, c->s);
    launch_reduce_final(c->partial, np, c->scalar, c->s);
    launch_add_scalar_cells(L0.g, v, c->scalar, -1.0 / (double)L0.np, c->s);
    // refresh the ghost images of the shifted field
    const int pm[3] = {0, 0, 0};
    launch_load_unknowns<double>(L0.g, 1, pm, VelArrC<double>{{v, nullptr, nullptr}}, VelArr<double>{{v, nullptr, nullptr}},
                                 c->s);
    return IBB_OK;
}

ibb_status faces_in(ibb_ctx *c, const double *src, double *const *dst)
{
    Level &L0 = c->lv[0];
    long long off = 0;
    for (int a = 0; a < c->d.dim; ++a) {
        launch_layout(L0.g, face_mask(a), src + off, dst[a], true, c->s);
        off += lattice_count(L0.g, face_mask(a));
    }
    return IBB_OK;
}

ibb_status faces_out(ibb_ctx *c, int level, double *const *src, double *dst)
{
    Level &L = c->lv[level];
    long long off = 0;
    for (int a = 0; a < c->d.dim; ++a) {
        launch_layout(L.g, face_mask(a), src[a], dst + off, false, c->s);
        off += lattice_count(L.g, face_mask(a));
    }
    return IBB_OK;
}

// ---- the pieces of a step, shared by single contexts and groups --------

// momentum right-hand side at u^n; the viscous iterate starts from u^n
void proj_viscous_rhs(ibb_ctx *c)
{
    Level &L0 = c->lv[0];
    View<double> v = view64(L0);
    int vm[3];
    vel_masks(c->d.dim, vm);
    launch_load_unknowns<double>(L0.g, c->d.dim, vm, VelArrC<double>{{c->u[0], c->u[1], c->u[2]}}, v.xu, c->s);
    launch_momentum_rhs(L0.g, c->ph, VelArrC<double>{{c->u[0], c->u[1], c->u[2]}}, v.cu,
                        VelArrC<double>{{c->f[0], c->f[1], c->f[2]}}, v.bu, c->s);
}

// pressure right-hand side from u~; the pressure iterate starts from p^n
void proj_pressure_rhs(ibb_ctx *c)
{
    Level &L0 = c->lv[0];
    View<double> v = view64(L0);
    const int pm[3] = {0, 0, 0};
    launch_pressure_div(L0.g, c->ph, cview(v.xu), VelArrC<double>{{c->u[0], c->u[1], c->u[2]}}, L0.bp, c->s);
    if (c->singular_p) remove_cell_mean(c, L0.bp);
    launch_load_unknowns<double>(L0.g, 1, pm, VelArrC<double>{{c->p, nullptr, nullptr}},
                                 VelArr<double>{{L0.xp, nullptr, nullptr}}, c->s);
}

// p^{n+1} into the state; the unknown faces of the state take
// u~ - (eps dt / sigma) beta G p
void proj_finish(ibb_ctx *c)
{
    Level &L0 = c->lv[0];
    View<double> v = view64(L0);
    if (c->singular_p) remove_cell_mean(c, L0.xp);
    launch_copy(L0.xp, c->p, L0.g.nel, c->s);
    launch_project(L0.g, c->ph, cview(v.xu), L0.xp, v.cp, VelArr<double>{{c->u[0], c->u[1], c->u[2]}}, c->s);
}

void fill_stats(ibb_ctx *c, const SolveOut &su, const SolveOut &sp, float tu, float tp, ibb_solve_stats *stats)
{
    if (!stats) return;
    stats->status_u = su.status;
    stats->status_p = sp.status;
    stats->cycles_u = su.cycles;
    stats->cycles_p = sp.cycles;
    stats->vcycles_u = su.vcycles;
    stats->vcycles_p = sp.vcycles;
    stats->relres_u = su.relres;
    stats->relres_p = sp.relres;
    stats->t_u_ms = tu;
    stats->t_p_ms = tp;
    stats->dof_u = c->lv[0].nu;
    stats->dof_p = c->lv[0].np;
}

// connected components of the alive springs into frag_label, counts into
// counters[2] (fragments) and counters[3] (detached); one host round trip per
// hook-and-shortcut round until no label moves
ibb_status frag_compute(ibb_ctx *c)
{
    const int eta = c->eta;
    const int m = c->have_springs ? c->m : 0;
    launch_frag_init(c->frag_label, eta, c->s);
    for (int round = 0; round <= eta; ++round) {
        launch_frag_round(c->ij, m, c->alive, c->frag_label, eta, c->frag_flag, c->s);
        int changed = 0;
        HIPCHK(hipMemcpyAsync(&changed, c->frag_flag, sizeof(int), hipMemcpyDeviceToHost, c->s));
        HIPCHK(hipStreamSynchronize(c->s));
        if (!changed) break;
    }
    launch_frag_count(c->frag_label, c->anchored, eta, c->frag_root, c->counters + 2, c->s);
    return IBB_OK;
}

// interpolation, node update, breakage, forces, spread and the coefficient
// hierarchy; the counters (broken this step, alive, and when tracked the
// fragments and detached fragments) are left on the device
ibb_status lag_launch(ibb_ctx *c)
{
    Level &L0 = c->lv[0];
    const long long em = c->eta_max > 0 ? c->eta_max : 1;
    {
        Timed t(c, PS_INTERP, 0, (long long)c->eta * c->d.dim);
        launch_interp(L0.g, c->d.kernel, c->d.h, VelArrC<double>{{c->u[0], c->u[1], c->u[2]}}, c->X, em, c->eta,
                      c->U, em, c->s);
    }
    launch_euler(L0.g, c->d.dt / c->d.sigma, c->U, c->X, em, c->eta, c->s);
    launch_fill<int>(c->counters, 4, 0, c->s);
    if (c->have_springs && c->m > 0)
        launch_spring_break(L0.g, c->d.break_ratio, c->X, em, c->ij, c->m, c->rest, c->alive, c->counters, c->s);
    if (c->d.track_fragments) {
        ibb_status fs = frag_compute(c);
        if (fs) return fs;
    }
    ibb_status st = rebuild_coefficients(c);
    if (st) return st;
    if (c->have_springs) launch_count_alive(c->alive, c->m, c->counters + 1, c->s);
    return IBB_OK;
}

}  // namespace

// ===========================================================================
// C interface
// ===========================================================================
extern "C" {

const char *ibb_status_string(ibb_status s)
{
    switch (s) {
    case IBB_OK: return "ok";
    case IBB_EINVAL: return "invalid argument";
    case IBB_ENOMEM: return "workspace too small";
    case IBB_ENOCONV: return "multigrid did not reach the tolerance";
    case IBB_ENUMERIC: return "non-finite residual";
    case IBB_EDEVICE: return "HIP runtime error";
    case IBB_ESTATE: return "call out of order";
    }
    return "unknown status";
}

const char *ibb_last_error(const ibb_ctx *c) { return c ? c->err.c_str() : create_err.c_str(); }

ibb_status ibb_lattice_count(const ibb_desc *desc, int kind, int axis, int64_t *count, int dims[3])
{
    if (check_desc(desc) || !count || kind < 0 || kind > 2 || axis < 0 || axis > 2) return IBB_EINVAL;
    if (kind == 1 && axis >= desc->dim) return IBB_EINVAL;
    if (kind == 2 && desc->dim == 2 && axis != 2) return IBB_EINVAL;
    Grid g = make_grid(desc, 0);
    const int vmask = kind == 0 ? 0 : (kind == 1 ? face_mask(axis) : edge_mask(desc->dim, axis));
    *count = lattice_count(g, vmask);
    if (dims)
        for (int d = 0; d < 3; ++d) dims[d] = stored_extent(g, d, (vmask >> d) & 1);
    return IBB_OK;
}

ibb_status ibb_footprint_bytes(const ibb_desc *desc, int64_t max_nodes, int64_t max_springs, size_t *bytes)
{
    if (check_desc(desc) || !bytes || max_nodes < 0 || max_springs < 0 || max_nodes > INT32_MAX / 2 ||
        max_springs > INT32_MAX / 2)
        return IBB_EINVAL;
    ibb_ctx tmp;
    setup_shapes(&tmp, desc, max_nodes, max_springs);
    *bytes = carve(&tmp, nullptr, true);
    return IBB_OK;
}

ibb_status ibb_create(const ibb_desc *desc, int64_t max_nodes, int64_t max_springs, void *workspace,
                      size_t workspace_bytes, void *stream, ibb_ctx **out)
{
    if (!out) return IBB_EINVAL;
    *out = nullptr;
    if (check_desc(desc) || !workspace || max_nodes < 0 || max_springs < 0 || max_nodes > INT32_MAX / 2 ||
        max_springs > INT32_MAX / 2)
        return IBB_EINVAL;
    wg_prepare();
    ibb_ctx *c = new ibb_ctx();
    setup_shapes(c, desc, max_nodes, max_springs);
    const size_t need = carve(c, nullptr, true);
    if (workspace_bytes < need) {
        delete c;
        return IBB_ENOMEM;
    }
    char *base = reinterpret_cast<char *>(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
    carve(c, base, false);
    c->s = reinterpret_cast<hipStream_t>(stream);
    // zero the whole workspace
    const size_t used = need - 256;
    launch_fill<unsigned char>(reinterpret_cast<unsigned char *>(base), (long long)used, 0, c->s);
    // initial coefficients: uniform fluid
    for (int l = 0; l < c->L; ++l) {
        Level &L = c->lv[l];
        for (int a = 0; a < desc->dim; ++a) launch_fill<double>(L.rho[a], L.g.nel, desc->rho0, c->s);
        launch_fill<double>(L.muc, L.g.nel, desc->mu_out, c->s);
        for (int e = 0; e < c->E; ++e) launch_fill<double>(L.mue[c->edge_axis[e]], L.g.nel, desc->mu_out, c->s);
    }
    // coarsest unknown tables
    std::vector<long long> ip, iu;
    std::vector<int> cp, cu;
    coarsest_tables(c, ip, cp, iu, cu);
    hipError_t e = hipSuccess;
    if (ip.size() <= (size_t)DENSE_MAX && !ip.empty()) {
        e = hipMemcpyAsync(c->uidx_p, ip.data(), ip.size() * sizeof(long long), hipMemcpyHostToDevice, c->s);
        if (e == hipSuccess) e = hipMemcpyAsync(c->ucomp_p, cp.data(), cp.size() * sizeof(int), hipMemcpyHostToDevice, c->s);
    }
    if (e == hipSuccess && iu.size() <= (size_t)DENSE_MAX && !iu.empty()) {
        e = hipMemcpyAsync(c->uidx_u, iu.data(), iu.size() * sizeof(long long), hipMemcpyHostToDevice, c->s);
        if (e == hipSuccess) e = hipMemcpyAsync(c->ucomp_u, cu.data(), cu.size() * sizeof(int), hipMemcpyHostToDevice, c->s);
    }
    // level tables for the one-workgroup coarse cycle
    std::vector<LevTab<double>> t64(MAXLEV);
    std::vector<LevTab<float>> t32(MAXLEV);
    std::vector<BoxDiv> bdv((size_t)MAXLEV * 4);
    for (int l = 0; l < c->L; ++l) {
        Level &L = c->lv[l];
        LevTab<double> &a = t64[l];
        LevTab<float> &b = t32[l];
        a.g = b.g = L.g;
        for (int k = 0; k < 4; ++k)
            bdv[(size_t)l * 4 + k] = box_div(unk_box(L.g, k < 3 && k < desc->dim ? face_mask(k) : 0));
        a.bd = b.bd = c->boxdiv + (size_t)l * 4;
        for (int k = 0; k < 3; ++k) {
            a.xu[k] = L.xu[k]; a.bu[k] = L.bu[k]; a.ru[k] = L.ru[k];
            a.rho[k] = L.rho[k]; a.beta[k] = L.beta[k]; a.mue[k] = L.mue[k];
            b.xu[k] = L.xu32[k]; b.bu[k] = L.bu32[k]; b.ru[k] = L.ru32[k];
            b.rho[k] = L.rho32[k]; b.beta[k] = L.beta32[k]; b.mue[k] = L.mue32[k];
        }
        a.xp = L.xp; a.bp = L.bp; a.rp = L.rp; a.muc = L.muc;
        b.xp = L.xp32; b.bp = L.bp32; b.rp = L.rp32; b.muc = L.muc32;
        const double h2 = L.g.h * L.g.h;
        a.mass = desc->sigma / desc->dt;
        a.cvu = L.cvu;
        a.cvp = 1.0 / h2;
        b.mass = (float)(desc->sigma / desc->dt);
        b.cvu = (float)L.cvu;
        b.cvp = (float)(1.0 / h2);
        a.nu = b.nu = L.nu;
        a.np = b.np = L.np;
        a.dec = b.dec = L.dec;
    }
    // tails: the unknowns of the tail level and the plan of the column
    // build, whose levels must fit this device's arena (otherwise the cycle
    // recurses as without a tail)
    std::vector<LdsLevel> tplans[2];
    std::vector<long long> tidx[2];
    std::vector<int> tcomp[2];
    for (int v = 0; v < 2 && e == hipSuccess; ++v) {
        Tail &t = c->tail[v];
        if (t.n <= 0) continue;
        plan_tail_build(c, v == 1, tplans[v]);
        if (c->tplan_bytes[v] > wg_lds_budget()) {
            t.n = 0;
            continue;
        }
        level_unknowns(c, t.level, v == 1, tidx[v], tcomp[v]);
        e = hipMemcpyAsync(const_cast<long long *>(t.idx), tidx[v].data(), tidx[v].size() * sizeof(long long),
                           hipMemcpyHostToDevice, c->s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(const_cast<int *>(t.comp), tcomp[v].data(), tcomp[v].size() * sizeof(int),
                               hipMemcpyHostToDevice, c->s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(c->tplan[v], tplans[v].data(), WG_MAXLEV * sizeof(LdsLevel), hipMemcpyHostToDevice,
                               c->s);
    }
    std::vector<LdsLevel> plans[2][2];
    for (int pr = 0; pr < 2; ++pr)
        for (int v = 0; v < 2; ++v) {
            plan_lds(c, pr, v == 1, plans[pr][v]);
            if (e == hipSuccess)
                e = hipMemcpyAsync(c->ldslev[pr][v], plans[pr][v].data(), WG_MAXLEV * sizeof(LdsLevel),
                                   hipMemcpyHostToDevice, c->s);
        }
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->boxdiv, bdv.data(), bdv.size() * sizeof(BoxDiv), hipMemcpyHostToDevice, c->s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->tab64, t64.data(), MAXLEV * sizeof(LevTab<double>), hipMemcpyHostToDevice, c->s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->tab32, t32.data(), MAXLEV * sizeof(LevTab<float>), hipMemcpyHostToDevice, c->s);
    for (int i = 0; i < 4 && e == hipSuccess; ++i) e = hipEventCreate(&c->ev[i]);
    const char *what = e == hipSuccess ? "" : "copying the level tables";
    if (e == hipSuccess && (e = hipStreamSynchronize(c->s)) != hipSuccess) what = "running the initial fills";
    if (e == hipSuccess && (e = hipGetLastError()) != hipSuccess) what = "an earlier launch";
    if (e != hipSuccess) {
        create_err = std::string("ibb_create: ") + what + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
        delete c;
        return IBB_EDEVICE;
    }
    create_err.clear();
    *out = c;
    return IBB_OK;
}

ibb_status ibb_destroy(ibb_ctx *c)
{
    if (!c) return IBB_EINVAL;
    (void)hipStreamSynchronize(c->s);
    for (int i = 0; i < 4; ++i)
        if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    for (auto &e : c->pev)
        if (e) (void)hipEventDestroy(e);
    for (auto &g : c->tick)
        if (g) (void)hipGraphExecDestroy(g);
    for (auto &v : c->gtick)
        for (auto &g : v)
            if (g) (void)hipGraphExecDestroy(g);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    delete c;
    return IBB_OK;
}

ibb_status ibb_set_params(ibb_ctx *c, const ibb_desc *desc)
{
    if (!c) return IBB_EINVAL;
    if (check_desc(desc)) return fail(c, IBB_EINVAL, "ibb_set_params: invalid descriptor");
    const ibb_desc &a = *desc, &b = c->d;
    bool same = a.dim == b.dim && a.h == b.h && a.sigma == b.sigma && a.eps == b.eps && a.inv_re == b.inv_re &&
                a.force_coef == b.force_coef && a.dt == b.dt && a.rho0 == b.rho0 && a.mu_out == b.mu_out &&
                a.omega == b.omega && a.kernel == b.kernel && a.nu1 == b.nu1 && a.nu2 == b.nu2 &&
                a.max_levels == b.max_levels && a.precision == b.precision && a.inner_cycles == b.inner_cycles &&
                a.wg_coarse_max == b.wg_coarse_max && a.krylov_restart == b.krylov_restart &&
                a.smoother_passes == b.smoother_passes && a.decoupled == b.decoupled &&
                a.coarse_tail == b.coarse_tail && a.smoother_zblock == b.smoother_zblock && a.galerkin == b.galerkin;
    for (int k = 0; k < 3; ++k)
        same = same && a.n[k] == b.n[k] && a.axis_bc[k] == b.axis_bc[k] && a.body_force[k] == b.body_force[k];
    for (int k = 0; k < 16; ++k) same = same && a.gamma[k] == b.gamma[k];
    if (!same)
        return fail(c, IBB_EINVAL,
                    "ibb_set_params: only rho_b, d0_pow_d, mu_max, break_ratio, the fragment fields, rtol and "
                    "max_cycles may change");
    c->d = a;
    c->ph.rho_b = a.rho_b;
    c->ph.d0_pow_d = a.d0_pow_d;
    c->ph.mu_max = a.mu_max;
    c->have_coefs = false;
    return IBB_OK;
}

ibb_status ibb_set_state(ibb_ctx *c, const double *u, const double *p)
{
    if (!c || !u) return fail(c, IBB_EINVAL, "ibb_set_state: null pointer");
    faces_in(c, u, c->u);
    if (p) launch_layout(c->lv[0].g, 0, p, c->p, true, c->s);
    HIPCHK(hipGetLastError());
    return IBB_OK;
}

ibb_status ibb_get_state(ibb_ctx *c, double *u, double *p)
{
    if (!c) return IBB_EINVAL;
    if (u) faces_out(c, 0, c->u, u);
    if (p) launch_layout(c->lv[0].g, 0, c->p, p, false, c->s);
    HIPCHK(hipGetLastError());
    return IBB_OK;
}

ibb_status ibb_set_nodes(ibb_ctx *c, int64_t n, const double *X)
{
    if (!c || n < 0 || n > c->eta_max || (n > 0 && !X)) return fail(c, IBB_EINVAL, "ibb_set_nodes: bad size or pointer");
    const long long em = c->eta_max > 0 ? c->eta_max : 1;
    for (int a = 0; a < c->d.dim; ++a)
        if (n > 0) HIPCHK(hipMemcpyAsync(c->X + a * em, X + a * n, n * sizeof(double), hipMemcpyDeviceToDevice, c->s));
    c->eta = (int)n;
    launch_frag_anchor(c->lv[0].g, c->X, em, (int)n, c->d.attach_axis, c->d.attach_dist, c->anchored, c->s);
    c->have_nodes = true;
    return IBB_OK;
}

ibb_status ibb_fragments(ibb_ctx *c, int32_t *label, int *n_fragments, int *n_detached)
{
    if (!c) return IBB_EINVAL;
    if (!c->have_nodes) return fail(c, IBB_ESTATE, "ibb_fragments: set the nodes first");
    launch_fill<int>(c->counters + 2, 2, 0, c->s);
    ibb_status st = frag_compute(c);
    if (st) return st;
    if (label && c->eta > 0)
        HIPCHK(hipMemcpyAsync(label, c->frag_label, c->eta * sizeof(int), hipMemcpyDeviceToDevice, c->s));
    int cnt[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(cnt, c->counters + 2, 2 * sizeof(int), hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->s));
    if (n_fragments) *n_fragments = cnt[0];
    if (n_detached) *n_detached = cnt[1];
    return IBB_OK;
}

ibb_status ibb_get_nodes(ibb_ctx *c, double *X, double *F, uint8_t *alive)
{
    if (!c) return IBB_EINVAL;
    const long long em = c->eta_max > 0 ? c->eta_max : 1;
    const long long n = c->eta;
    for (int a = 0; a < c->d.dim && n > 0; ++a) {
        if (X) HIPCHK(hipMemcpyAsync(X + a * n, c->X + a * em, n * sizeof(double), hipMemcpyDeviceToDevice, c->s));
        if (F) HIPCHK(hipMemcpyAsync(F + a * n, c->F + a * em, n * sizeof(double), hipMemcpyDeviceToDevice, c->s));
    }
    if (alive && c->m > 0) HIPCHK(hipMemcpyAsync(alive, c->alive, c->m, hipMemcpyDeviceToDevice, c->s));
    return IBB_OK;
}

ibb_status ibb_set_springs(ibb_ctx *c, int64_t m, const int32_t *ij, const double *rest, const double *K,
                           const uint8_t *alive)
{
    if (!c || m < 0 || m > c->m_max || (m > 0 && (!ij || !rest || !K)))
        return fail(c, IBB_EINVAL, "ibb_set_springs: bad size or pointer");
    if (!c->have_nodes) return fail(c, IBB_ESTATE, "ibb_set_springs: set the nodes first");
    c->m = (int)m;
    if (m > 0) {
        HIPCHK(hipMemcpyAsync(c->ij, ij, m * sizeof(int), hipMemcpyDeviceToDevice, c->s));
        HIPCHK(hipMemcpyAsync(c->ij + m, ij + m, m * sizeof(int), hipMemcpyDeviceToDevice, c->s));
        HIPCHK(hipMemcpyAsync(c->rest, rest, m * sizeof(double), hipMemcpyDeviceToDevice, c->s));
        HIPCHK(hipMemcpyAsync(c->K, K, m * sizeof(double), hipMemcpyDeviceToDevice, c->s));
        if (alive) HIPCHK(hipMemcpyAsync(c->alive, alive, m, hipMemcpyDeviceToDevice, c->s));
        else launch_fill<unsigned char>(c->alive, m, 1, c->s);
        launch_incidence_keys(c->ij, (int)m, c->inc_keys, c->s);
    }
    launch_bucket_sort(c->inc_keys, (int)(2 * m), c->eta > 0 ? c->eta : 1, c->inc_count, c->inc_start, c->inc_list,
                       (int)(m > 0 ? m : 1), c->scan_tmp, c->s);
    HIPCHK(hipGetLastError());
    c->have_springs = true;
    return IBB_OK;
}

ibb_status ibb_update_coefficients(ibb_ctx *c)
{
    if (!c) return IBB_EINVAL;
    if (!c->have_nodes) return fail(c, IBB_ESTATE, "ibb_update_coefficients: no nodes set");
    ibb_status st = rebuild_coefficients(c);
    if (st) return st;
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->s));
    return IBB_OK;
}

ibb_status ibb_projection_step(ibb_ctx *c, ibb_solve_stats *stats)
{
    if (!c) return IBB_EINVAL;
    if (!c->have_coefs) return fail(c, IBB_ESTATE, "ibb_projection_step: coefficients not built");
    // momentum right-hand side and the viscous solve, warm start u^n
    proj_viscous_rhs(c);
    HIPCHK(hipEventRecord(c->ev[0], c->s));
    SolveOut su, sp;
    ibb_status st = solve(c, true, c->d.max_cycles, 0, &su);
    if (st) return st;
    HIPCHK(hipEventRecord(c->ev[1], c->s));
    // pressure right-hand side and solve, warm start p^n
    proj_pressure_rhs(c);
    HIPCHK(hipEventRecord(c->ev[2], c->s));
    st = solve(c, false, c->d.max_cycles, 0, &sp);
    if (st) return st;
    HIPCHK(hipEventRecord(c->ev[3], c->s));
    proj_finish(c);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->s));
    float tu = 0, tp = 0;
    (void)hipEventElapsedTime(&tu, c->ev[0], c->ev[1]);
    (void)hipEventElapsedTime(&tp, c->ev[2], c->ev[3]);
    fill_stats(c, su, sp, tu, tp, stats);
    if (su.status) return fail(c, (ibb_status)su.status, "viscous solve did not converge");
    if (sp.status) return fail(c, (ibb_status)sp.status, "pressure solve did not converge");
    return IBB_OK;
}

ibb_status ibb_lagrangian_update(ibb_ctx *c, ibb_lag_stats *stats)
{
    if (!c) return IBB_EINVAL;
    if (!c->have_coefs) return fail(c, IBB_ESTATE, "ibb_lagrangian_update: coefficients not built");
    HIPCHK(hipEventRecord(c->ev[0], c->s));
    ibb_status st = lag_launch(c);
    if (st) return st;
    HIPCHK(hipEventRecord(c->ev[1], c->s));
    int cnt[4] = {0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(cnt, c->counters, 4 * sizeof(int), hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->s));
    if (stats) {
        float t = 0;
        (void)hipEventElapsedTime(&t, c->ev[0], c->ev[1]);
        stats->n_broken = cnt[0];
        stats->n_alive = cnt[1];
        stats->t_ms = t;
        stats->n_fragments = c->d.track_fragments ? cnt[2] : -1;
        stats->n_detached = c->d.track_fragments ? cnt[3] : -1;
    }
    return IBB_OK;
}

ibb_status ibb_get_fields(ibb_ctx *c, int level, double *f, double *rho, double *mu_c, double *mu_e)
{
    if (!c || level < 0 || level >= c->L || (f && level != 0)) return fail(c, IBB_EINVAL, "ibb_get_fields: bad level");
    Level &L = c->lv[level];
    if (f) faces_out(c, 0, c->f, f);
    if (rho) faces_out(c, level, L.rho, rho);
    if (mu_c) launch_layout(L.g, 0, L.muc, mu_c, false, c->s);
    if (mu_e) {
        long long off = 0;
        for (int e = 0; e < c->E; ++e) {
            const int vm = edge_mask(c->d.dim, c->edge_axis[e]);
            launch_layout(L.g, vm, L.mue[c->edge_axis[e]], mu_e + off, false, c->s);
            off += lattice_count(L.g, vm);
        }
    }
    HIPCHK(hipGetLastError());
    return IBB_OK;
}

ibb_status ibb_momentum_rhs(ibb_ctx *c, double *b)
{
    if (!c || !b) return IBB_EINVAL;
    if (!c->have_coefs) return fail(c, IBB_ESTATE, "ibb_momentum_rhs: coefficients not built");
    Level &L0 = c->lv[0];
    View<double> v = view64(L0);
    for (int a = 0; a < c->d.dim; ++a) launch_fill<double>(L0.ru[a], L0.g.nel, 0.0, c->s);
    launch_momentum_rhs(L0.g, c->ph, VelArrC<double>{{c->u[0], c->u[1], c->u[2]}}, v.cu,
                        VelArrC<double>{{c->f[0], c->f[1], c->f[2]}}, v.ru, c->s);
    faces_out(c, 0, L0.ru, b);
    HIPCHK(hipGetLastError());
    return IBB_OK;
}

ibb_status ibb_pressure_rhs(ibb_ctx *c, const double *ut, double *bp)
{
    if (!c || !ut || !bp) return IBB_EINVAL;
    Level &L0 = c->lv[0];
    faces_in(c, ut, L0.ru);
    launch_pressure_div(L0.g, c->ph, VelArrC<double>{{L0.ru[0], L0.ru[1], L0.ru[2]}},
                        VelArrC<double>{{L0.ru[0], L0.ru[1], L0.ru[2]}}, L0.rp, c->s);
    if (c->singular_p) remove_cell_mean(c, L0.rp);
    launch_layout(L0.g, 0, L0.rp, bp, false, c->s);
    HIPCHK(hipGetLastError());
    return IBB_OK;
}

ibb_status ibb_mg_solve(ibb_ctx *c, int which, const double *b, double *x, int max_cycles_override, int ncycles_exact,
                        int *cycles, double *relres)
{
    if (!c || !b || !x || (which != 0 && which != 1)) return IBB_EINVAL;
    if (!c->have_coefs) return fail(c, IBB_ESTATE, "ibb_mg_solve: coefficients not built");
    Level &L0 = c->lv[0];
    const bool vel = which == 1;
    int vm[3];
    vel_masks(c->d.dim, vm);
    const int pm[3] = {0, 0, 0};
    // the initial guess enters through the unknowns only; the caller's values
    // on fixed faces are handed back unchanged
    if (vel) {
        for (int a = 0; a < c->d.dim; ++a) launch_fill<double>(L0.bu[a], L0.g.nel, 0.0, c->s);
        faces_in(c, b, L0.bu);
        faces_in(c, x, L0.ru);
        launch_load_unknowns<double>(L0.g, c->d.dim, vm, VelArrC<double>{{L0.ru[0], L0.ru[1], L0.ru[2]}},
                                     VelArr<double>{{L0.xu[0], L0.xu[1], L0.xu[2]}}, c->s);
    } else {
        launch_layout(L0.g, 0, b, L0.bp, true, c->s);
        launch_layout(L0.g, 0, x, L0.rp, true, c->s);
        launch_load_unknowns<double>(L0.g, 1, pm, VelArrC<double>{{L0.rp, nullptr, nullptr}},
                                     VelArr<double>{{L0.xp, nullptr, nullptr}}, c->s);
    }
    SolveOut o;
    ibb_status st = solve(c, vel, max_cycles_override > 0 ? max_cycles_override : c->d.max_cycles, ncycles_exact, &o);
    if (st) return st;
    if (vel) {
        faces_in(c, x, L0.ru);
        launch_load_unknowns<double>(L0.g, c->d.dim, vm, VelArrC<double>{{L0.xu[0], L0.xu[1], L0.xu[2]}},
                                     VelArr<double>{{L0.ru[0], L0.ru[1], L0.ru[2]}}, c->s);
        faces_out(c, 0, L0.ru, x);
    } else {
        launch_layout(L0.g, 0, L0.xp, x, false, c->s);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->s));
    if (cycles) *cycles = o.cycles;
    if (relres) *relres = o.relres;
    if (o.status) return fail(c, (ibb_status)o.status, "ibb_mg_solve: no convergence");
    return IBB_OK;
}

ibb_status ibb_project(ibb_ctx *c, const double *ut, const double *p, double *u)
{
    if (!c || !ut || !p || !u) return IBB_EINVAL;
    if (!c->have_coefs) return fail(c, IBB_ESTATE, "ibb_project: coefficients not built");
    Level &L0 = c->lv[0];
    View<double> v = view64(L0);
    const int pm[3] = {0, 0, 0};
    faces_in(c, ut, L0.ru);
    launch_layout(L0.g, 0, p, L0.rp, true, c->s);
    launch_load_unknowns<double>(L0.g, 1, pm, VelArrC<double>{{L0.rp, nullptr, nullptr}},
                                 VelArr<double>{{L0.xp, nullptr, nullptr}}, c->s);
    launch_project(L0.g, c->ph, cview(v.ru), L0.xp, v.cp, v.ru, c->s);
    faces_out(c, 0, L0.ru, u);
    HIPCHK(hipGetLastError());
    return IBB_OK;
}

ibb_status ibb_interp(ibb_ctx *c, double width, int64_t n, const double *X, const double *u, double *U)
{
    if (!c || n < 0 || (n > 0 && (!X || !u || !U)) || !(width > 0)) return IBB_EINVAL;
    for (int a = 0; a < c->d.dim; ++a)
        if (c->d.axis_bc[a] == IBB_AXIS_PERIODIC && 4.0 * width > c->d.n[a] * c->d.h)
            return fail(c, IBB_EINVAL, "ibb_interp: width too large for a periodic axis");
    Level &L0 = c->lv[0];
    faces_in(c, u, L0.ru);
    launch_interp(L0.g, c->d.kernel, width, VelArrC<double>{{L0.ru[0], L0.ru[1], L0.ru[2]}}, X, n, (int)n, U, n, c->s);
    HIPCHK(hipGetLastError());
    return IBB_OK;
}

ibb_status ibb_spread(ibb_ctx *c, double width, int64_t n, const double *X, const double *F, double *out)
{
    if (!c || n < 0 || n > c->eta_max || (n > 0 && (!X || !F)) || !out || !(width > 0)) return IBB_EINVAL;
    const double wmin = c->d.omega < c->d.h ? c->d.omega : c->d.h;
    if (width < wmin) return fail(c, IBB_EINVAL, "ibb_spread: width below min(omega, h)");
    for (int a = 0; a < c->d.dim; ++a)
        if (c->d.axis_bc[a] == IBB_AXIS_PERIODIC && 4.0 * width > c->d.n[a] * c->d.h)
            return fail(c, IBB_EINVAL, "ibb_spread: width too large for a periodic axis");
    Level &L0 = c->lv[0];
    Bins b = c->bins;
    bins_for_width(&c->d, width, b.nb, b.bs);
    b.nbins = b.nb[0] * b.nb[1] * b.nb[2];
    launch_bin_nodes(L0.g, b, X, n > 0 ? n : 1, (int)n, c->scan_tmp, c->s);
    for (int a = 0; a < c->d.dim; ++a)
        launch_spread_face(L0.g, c->ph, b, X, F, n > 0 ? n : 1, a, width, L0.ru[a], nullptr, c->s);
    faces_out(c, 0, L0.ru, out);
    HIPCHK(hipGetLastError());
    return IBB_OK;
}

}  // extern "C"

namespace {

// Scratch of ibb_spread_static: the bins of the nodes and one face lattice
// of staging, IBB_SPREAD_STATIC_MAX_BYTES per GPU, held until the process
// ends.  In host code `spread_scratch` only names the symbol; kernels get the
// device address that hipGetSymbolAddress returns for the current device.
__device__ __align__(256) unsigned char spread_scratch[IBB_SPREAD_STATIC_MAX_BYTES];

constexpr int SPREAD_STATIC_MAX_DEVICES = 64;
std::mutex spread_scratch_mu;
void *spread_scratch_ptr[SPREAD_STATIC_MAX_DEVICES] = {};

// the current device's copy of the scratch array (looked up once per device)
hipError_t spread_scratch_of_current(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= SPREAD_STATIC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(spread_scratch_mu);
    if (!spread_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(spread_scratch));
        if (e != hipSuccess) return e;
        spread_scratch_ptr[dev] = p;
    }
    *out = spread_scratch_ptr[dev];
    return hipSuccess;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

ibb_status ibb_spread_static(const ibb_desc *desc, double width, int64_t n, const double *X, const double *F,
                             double *out, void *stream)
{
    ibb_ctx *c = nullptr;   // no context: HIPCHK records no message
    if (check_desc(desc) || n < 0 || n > INT32_MAX / 2 || (n > 0 && (!X || !F)) || !out || !(width > 0))
        return IBB_EINVAL;
    const double wmin = desc->omega < desc->h ? desc->omega : desc->h;
    if (width < wmin) return IBB_EINVAL;
    for (int a = 0; a < desc->dim; ++a)
        if (desc->axis_bc[a] == IBB_AXIS_PERIODIC && 4.0 * width > desc->n[a] * desc->h) return IBB_EINVAL;
    const Grid g = make_grid(desc, 0);
    Bins b{};
    bins_for_width(desc, width, b.nb, b.bs);
    b.nbins = b.nb[0] * b.nb[1] * b.nb[2];
    // the scratch layout: bin of each node, bin counts, bin starts, node ids
    // by bin, scan block sums, one padded face lattice of staging
    const size_t eta = (size_t)n;
    const size_t o_bin = 0;
    const size_t o_cnt = o_bin + align256(eta * sizeof(int));
    const size_t o_start = o_cnt + align256((size_t)b.nbins * sizeof(int));
    const size_t o_sorted = o_start + align256(((size_t)b.nbins + 1) * sizeof(int));
    const size_t o_scan = o_sorted + align256(eta * sizeof(int));
    const size_t o_stage =
        o_scan + align256((size_t)scan_scratch_ints(std::max<long long>(b.nbins, (long long)eta + 1)) * sizeof(int));
    const size_t need = o_stage + align256((size_t)g.nel * sizeof(double));
    if (need > (size_t)IBB_SPREAD_STATIC_MAX_BYTES) return IBB_ENOMEM;
    void *base = nullptr;
    HIPCHK(spread_scratch_of_current(&base));
    char *sc = static_cast<char *>(base);
    b.bin_of = reinterpret_cast<int *>(sc + o_bin);
    b.count = reinterpret_cast<int *>(sc + o_cnt);
    b.start = reinterpret_cast<int *>(sc + o_start);
    b.sorted = reinterpret_cast<int *>(sc + o_sorted);
    int *scan_tmp = reinterpret_cast<int *>(sc + o_scan);
    double *stage = reinterpret_cast<double *>(sc + o_stage);
    Phys ph{};
    ph.sigma = desc->sigma;
    ph.eps = desc->eps;
    ph.inv_re = desc->inv_re;
    ph.force_coef = desc->force_coef;
    ph.dt = desc->dt;
    ph.rho0 = desc->rho0;
    ph.rho_b = desc->rho_b;
    ph.d0_pow_d = desc->d0_pow_d;
    ph.mu_out = desc->mu_out;
    ph.mu_max = desc->mu_max;
    ph.omega = desc->omega;
    ph.kernel = desc->kernel;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // the same launches as ibb_spread; the bin counts are cleared by the sort
    // itself, and every stored face position of the staging is written
    // before it is read
    launch_bin_nodes(g, b, X, n > 0 ? n : 1, (int)n, scan_tmp, s);
    long long off = 0;
    for (int a = 0; a < desc->dim; ++a) {
        launch_spread_face(g, ph, b, X, F, n > 0 ? n : 1, a, width, stage, nullptr, s);
        launch_layout(g, face_mask(a), stage, out + off, false, s);
        off += lattice_count(g, face_mask(a));
    }
    HIPCHK(hipGetLastError());
    return IBB_OK;
}

ibb_status ibb_profile_enable(ibb_ctx *c, int enable)
{
    if (!c) return IBB_EINVAL;
    prof_flush(c);
    if (enable && c->pev.empty()) {
        c->pev.resize(2 * PROF_PAIRS);
        c->pcls.resize(PROF_PAIRS);
        c->punits.resize(PROF_PAIRS);
        for (auto &e : c->pev) HIPCHK(hipEventCreate(&e));
    }
    c->prof = enable != 0;
    c->pused = 0;
    for (int i = 0; i < IBB_PROFILE_CLASSES; ++i) {
        c->plaunch[i] = 0;
        c->pms[i] = 0.0;
        c->punit_tot[i] = 0;
    }
    return IBB_OK;
}

ibb_status ibb_profile_read(ibb_ctx *c, int kernel_class, long long *launches, double *total_ms, long long *units)
{
    if (!c || kernel_class < 0 || kernel_class >= IBB_PROFILE_CLASSES) return IBB_EINVAL;
    prof_flush(c);
    if (launches) *launches = c->plaunch[kernel_class];
    if (total_ms) *total_ms = c->pms[kernel_class];
    if (units) *units = c->punit_tot[kernel_class];
    return IBB_OK;
}

ibb_status ibb_level_info(const ibb_ctx *c, int level, int *nlevels, int n[3])
{
    if (!c) return IBB_EINVAL;
    if (nlevels) *nlevels = c->L;
    if (n) {
        if (level < 0 || level >= c->L) return IBB_EINVAL;
        for (int d = 0; d < 3; ++d) n[d] = c->lv[level].g.n[d];
    }
    return IBB_OK;
}

}  // extern "C"

// ===========================================================================
// groups: several contexts stepped together on one stream.  Every pass of
// the members' V-cycles that can share a launch does (one launch per pass,
// level and dimension), and one tick of a solve (the V-cycle or refined
// outer iteration, the residual and its norm) is captured once as a HIP
// graph and replayed; members that have converged are switched off by a
// device-side flag, so the graph never changes while the group lives.
// ===========================================================================
namespace {

enum { GK_REDUCE = 10, GK_COARSE = 11 };

struct GOp {
    int kind;       // BK_* or GK_*
    int prec;       // 0: FP64 tables, 1: FP32 tables
    int D, vel, A, colour;
    size_t off;     // first BEntry (or BCoarse) of the launch
    unsigned n;     // blocks (or items)
    int lds;        // coarse launches: LDS arena bytes
};

struct Plan {
    std::vector<BEntry> ent;
    std::vector<BCoarse> cent;
    std::vector<GOp> ops[2];   // tick of the pressure (0) and the viscous (1) solve
};

}  // namespace

struct ibb_group {
    std::vector<ibb_ctx *> m;
    hipStream_t s = nullptr;
    bool refined = false;
    int inner = 1, nu1 = 2, nu2 = 2;
    BEntry *ent = nullptr;
    BCoarse *cent = nullptr;
    int *flags = nullptr;
    double *norms = nullptr;
    int *counts = nullptr;
    Plan plan;
    hipGraphExec_t exec[2] = {};
    std::vector<int> hflags, dflags;   // wanted flags, flags on the device
    std::vector<char> active;          // members taking part in the group's calls
    hipEvent_t ev[5] = {};
    // side streams (default priority) for members solved by GCR, which
    // advance in lock step with the shared ticks, and one event each
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> sev;
    std::string err;
};

#define GCHK(expr)                                                                           \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) {                                                              \
            g->err = std::string(#expr) + ": " + hipGetErrorString(e_);                      \
            return IBB_EDEVICE;                                                              \
        }                                                                                    \
    } while (0)

namespace {

// last level a member's V-cycle runs with launched passes (the coarse part,
// from there down, runs in one workgroup per member)
int coarse_start(const ibb_ctx *c, bool vel)
{
    const int lc = vel ? c->lc_u : c->lc_p;
    return lc < c->L - 1 ? lc : c->L - 1;
}

const void *table_at(ibb_ctx *c, int prec, int l)
{
    return prec ? (const void *)(c->tab32 + l) : (const void *)(c->tab64 + l);
}

// one batched pass over the members listed in `who`, one launch per dimension
void plan_pass(Plan &P, std::vector<GOp> &ops, const std::vector<ibb_ctx *> &m, const std::vector<int> &who, int kind,
               int prec, bool vel, int A, int colour, int l, bool norm)
{
    for (int D = 2; D <= 3; ++D) {
        GOp op{kind, prec, D, vel ? 1 : 0, A, colour, P.ent.size(), 0, 0};
        for (int i : who) {
            ibb_ctx *c = m[i];
            if (c->d.dim != D) continue;
            if (kind == BK_SWEEP && vel && A >= D) continue;
            const Grid &gl = c->lv[l].g;
            const Grid &gc = l + 1 < c->L ? c->lv[l + 1].g : gl;
            const int nb = batch_blocks(kind, gl, gc, vel ? 1 : 0, A);
            BEntry e{};
            e.tab = table_at(c, prec, l);
            e.tab2 = table_at(c, 1, 0);
            e.partial = norm ? c->partial : nullptr;
            e.base = (int)op.n;
            e.nb = nb;
            e.ctx = i;
            for (int b = 0; b < nb; ++b) P.ent.push_back(e);
            op.n += nb;
        }
        if (op.n) ops.push_back(op);
    }
}

void plan_sweeps(Plan &P, std::vector<GOp> &ops, const std::vector<ibb_ctx *> &m, const std::vector<int> &who, int prec,
                 bool vel, int l)
{
    for (int A = 0; A < (vel ? 3 : 1); ++A)
        for (int colour = 0; colour < 2; ++colour) plan_pass(P, ops, m, who, BK_SWEEP, prec, vel, A, colour, l, false);
}

// one V-cycle of every member, in each member's own order of passes
void plan_vcycle(Plan &P, std::vector<GOp> &ops, const std::vector<ibb_ctx *> &m, int prec, bool vel, int nu1,
                 int nu2)
{
    const int n = (int)m.size();
    int maxl = 0;
    for (ibb_ctx *c : m) maxl = std::max(maxl, coarse_start(c, vel));
    auto members_above = [&](int l) {
        std::vector<int> w;
        for (int i = 0; i < n; ++i)
            if (l < coarse_start(m[i], vel)) w.push_back(i);
        return w;
    };
    for (int l = 0; l < maxl; ++l) {
        const std::vector<int> w = members_above(l);
        for (int s = 0; s < nu1; ++s) plan_sweeps(P, ops, m, w, prec, vel, l);
        plan_pass(P, ops, m, w, BK_RESID, prec, vel, 0, 0, l, false);
        plan_pass(P, ops, m, w, BK_RESTRICT, prec, vel, 0, 0, l, false);
    }
    for (int D = 2; D <= 3; ++D) {
        GOp op{GK_COARSE, prec, D, vel ? 1 : 0, 0, 0, P.cent.size(), 0, 0};
        for (int i = 0; i < n; ++i) {
            ibb_ctx *c = m[i];
            if (c->d.dim != D) continue;
            Level &LC = c->lv[c->L - 1];
            const long long nc = vel ? LC.nu : LC.np;
            BCoarse it{};
            it.tab = table_at(c, prec, 0);
            it.uidx = vel ? c->uidx_u : c->uidx_p;
            it.ucomp = vel ? c->ucomp_u : c->ucomp_p;
            it.M = vel ? c->Mu : c->Mp;
            it.l0 = coarse_start(c, vel);
            it.L = c->L;
            it.ndense = nc <= DENSE_MAX ? (int)nc : 0;
            it.ctx = i;
            it.lds = c->ldslev[prec][vel ? 1 : 0];
            it.lds_from = c->lds_ls[prec][vel ? 1 : 0];
            it.tail = has_tail(c, prec, vel) ? c->tail[vel ? 1 : 0] : Tail{};
            op.lds = std::max(op.lds, c->lds_bytes[prec][vel ? 1 : 0]);
            P.cent.push_back(it);
            op.n++;
        }
        if (op.n) ops.push_back(op);
    }
    for (int l = maxl - 1; l >= 0; --l) {
        const std::vector<int> w = members_above(l);
        plan_pass(P, ops, m, w, BK_PROLONG, prec, vel, 0, 0, l, false);
        for (int s = 0; s < nu2; ++s) plan_sweeps(P, ops, m, w, prec, vel, l);
    }
}

// one tick: an FP64 V-cycle (or a refined outer iteration), then the FP64
// residual with its norm
void plan_tick(Plan &P, std::vector<GOp> &ops, const std::vector<ibb_ctx *> &m, bool refined, int inner, bool vel,
               int nu1, int nu2)
{
    std::vector<int> all(m.size());
    for (size_t i = 0; i < m.size(); ++i) all[i] = (int)i;
    if (refined) {
        plan_pass(P, ops, m, all, BK_PREP, 0, vel, 0, 0, 0, false);
        for (int it = 0; it < inner; ++it) plan_vcycle(P, ops, m, 1, vel, nu1, nu2);
        plan_pass(P, ops, m, all, BK_ADD, 0, vel, 0, 0, 0, false);
    } else {
        plan_vcycle(P, ops, m, 0, vel, nu1, nu2);
    }
    plan_pass(P, ops, m, all, BK_RESID, 0, vel, 0, 0, 0, true);
    GOp red{GK_REDUCE, 0, 0, vel ? 1 : 0, 0, 0, P.ent.size(), 0, 0};
    for (size_t i = 0; i < m.size(); ++i) {
        ibb_ctx *c = m[i];
        BEntry e{};
        e.partial = c->partial;
        e.nb = batch_blocks(BK_RESID, c->lv[0].g, c->lv[0].g, vel ? 1 : 0, 0) * (vel ? c->d.dim : 1);
        e.ctx = (int)i;
        P.ent.push_back(e);
        red.n++;
    }
    ops.push_back(red);
}

void build_plan(Plan &P, const std::vector<ibb_ctx *> &m, bool refined, int inner, int nu1, int nu2)
{
    for (int vel = 0; vel < 2; ++vel) plan_tick(P, P.ops[vel], m, refined, inner, vel == 1, nu1, nu2);
}

void emit_ops(ibb_group *g, const std::vector<GOp> &ops)
{
    for (const GOp &op : ops) {
        switch (op.kind) {
        case GK_REDUCE: launch_breduce(g->ent + op.off, op.n, g->flags, g->norms, g->s); break;
        case GK_COARSE:
            if (op.prec)
                launch_bcoarse<float>(op.D, op.vel, g->cent + op.off, op.n, g->flags, g->nu1, g->nu2, op.lds, g->s);
            else
                launch_bcoarse<double>(op.D, op.vel, g->cent + op.off, op.n, g->flags, g->nu1, g->nu2, op.lds, g->s);
            break;
        default:
            if (op.prec)
                launch_bpass<float>(op.kind, op.D, op.vel, op.A, op.colour, g->ent + op.off, op.n, g->flags, g->s);
            else
                launch_bpass<double>(op.kind, op.D, op.vel, op.A, op.colour, g->ent + op.off, op.n, g->flags, g->s);
        }
    }
}

ibb_status check_members(ibb_ctx *const *ctxs, int n)
{
    if (!ctxs || n < 1) return IBB_EINVAL;
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i]) return IBB_EINVAL;
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return IBB_EINVAL;
        const ibb_desc &a = ctxs[0]->d, &b = ctxs[i]->d;
        if (a.precision != b.precision || a.nu1 != b.nu1 || a.nu2 != b.nu2) return IBB_EINVAL;
        if (a.precision == IBB_FP32_REFINED && a.inner_cycles != b.inner_cycles) return IBB_EINVAL;
        // the batched passes know the rediscretised operators only
        if (b.galerkin) return IBB_EINVAL;
    }
    return IBB_OK;
}

size_t group_bytes(const Plan &P, int n)
{
    Carver cv{nullptr, 0, true};
    cv.take<BEntry>(P.ent.size());
    cv.take<BCoarse>(P.cent.size());
    cv.take<int>(n);
    cv.take<double>(n);
    cv.take<int>(4 * (size_t)n);
    return cv.off + 256;
}

struct GroupSolve {
    std::vector<SolveOut> out;
    std::vector<double> nb, rel;
    std::vector<char> done;
};

// both norms of a member's start (||b||, then ||b - A x0||) into its slot
ibb_status group_norms(ibb_group *g, bool vel, bool resid, const std::vector<char> &skip, std::vector<double> &h)
{
    const int n = (int)g->m.size();
    for (int i = 0; i < n; ++i) {
        if (skip[i]) continue;
        ibb_ctx *c = g->m[i];
        Level &L = c->lv[0];
        int np;
        if (resid) {
            np = residual<double>(c, vel, 0, c->partial);
        } else {
            int vm[3];
            vel_masks(c->d.dim, vm);
            const int pm[3] = {0, 0, 0};
            if (vel)
                np = launch_norm2<double>(L.g, c->d.dim, vm, VelArrC<double>{{L.bu[0], L.bu[1], L.bu[2]}},
                                          c->partial, g->s);
            else
                np = launch_norm2<double>(L.g, 1, pm, VelArrC<double>{{L.bp, nullptr, nullptr}}, c->partial, g->s);
        }
        launch_reduce_final(c->partial, np, g->norms + i, g->s);
    }
    h.assign(n, 0.0);
    GCHK(hipMemcpyAsync(h.data(), g->norms, n * sizeof(double), hipMemcpyDeviceToHost, g->s));
    GCHK(hipStreamSynchronize(g->s));
    return IBB_OK;
}

// the members' solves of one system, ticked together; each member follows
// exactly the sequence of its own solve (same stopping test, same passes).
// Members solved by GCR run their own iterations, each on a side stream, in
// lock step with the shared ticks: one round launches every active member's
// next iteration and reads all norms back at once.
constexpr int GROUP_SIDE_STREAMS = 4;

// on every way out of a group solve, the group's stream waits for the work
// queued on the side streams
struct SideJoin {
    ibb_group *g;
    int n = 0;
    ~SideJoin()
    {
        for (int k = 0; k < n; ++k)
            if (hipEventRecord(g->sev[k], g->side[k]) != hipSuccess ||
                hipStreamWaitEvent(g->s, g->sev[k], 0) != hipSuccess)
                (void)hipStreamSynchronize(g->side[k]);
    }
};

ibb_status group_solve(ibb_group *g, bool vel, GroupSolve &R)
{
    const int n = (int)g->m.size();
    R.out.assign(n, SolveOut());
    R.nb.assign(n, 0.0);
    R.rel.assign(n, 0.0);
    R.done.assign(n, 0);
    std::vector<double> h;
    ibb_status st;
    // GCR members: their flags stay clear in the captured ticks
    std::vector<GcrRun> gr(n);
    std::vector<int> side(n, -1);
    int ngcr = 0;
    for (int i = 0; i < n; ++i) {
        if (!g->active[i]) R.done[i] = 1;
        else if (g->m[i]->d.krylov_restart > 0) side[i] = ngcr++ % GROUP_SIDE_STREAMS;
    }
    const int nside = ngcr < GROUP_SIDE_STREAMS ? ngcr : GROUP_SIDE_STREAMS;
    while ((int)g->side.size() < nside) {
        hipStream_t sd;
        hipEvent_t ev;
        GCHK(hipStreamCreateWithFlags(&sd, hipStreamNonBlocking));
        g->side.push_back(sd);
        GCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        g->sev.push_back(ev);
    }
    SideJoin join{g, nside};
    if (ngcr) {
        // the side streams start after the group stream's work so far
        GCHK(hipEventRecord(g->ev[4], g->s));
        for (int k = 0; k < nside; ++k) GCHK(hipStreamWaitEvent(g->side[k], g->ev[4], 0));
        for (int i = 0; i < n; ++i) {
            if (side[i] < 0) continue;
            ibb_ctx *c = g->m[i];
            c->s = g->side[side[i]];
            gr[i].c = c;
            gr[i].vel = vel;
            gr[i].max_cycles = c->d.max_cycles;
            gr[i].exact = 0;
            gr[i].o = &R.out[i];
            if ((st = gcr_begin(gr[i]))) return st;
            R.done[i] = 1;
        }
    }
    if ((st = group_norms(g, vel, false, R.done, h))) return st;
    for (int i = 0; i < n; ++i) {
        if (R.done[i]) continue;
        R.nb[i] = sqrt(h[i]);
        if (R.nb[i] == 0.0) {
            zero_unknowns(g->m[i], vel);
            R.done[i] = 1;
        }
    }
    if ((st = group_norms(g, vel, true, R.done, h))) return st;
    for (int i = 0; i < n; ++i)
        if (!R.done[i]) R.rel[i] = sqrt(h[i]) / R.nb[i];
    std::vector<char> ran(n, 0);
    for (;;) {
        bool any = false, anyg = false;
        for (int i = 0; i < n; ++i) {
            g->hflags[i] = 0;
            ran[i] = 0;
            if (side[i] >= 0) {
                if (gcr_more(gr[i])) {
                    ran[i] = 1;
                    anyg = true;
                }
                continue;
            }
            if (R.done[i]) continue;
            const double rel = R.rel[i];
            ibb_ctx *c = g->m[i];
            if (rel <= c->d.rtol) { R.done[i] = 1; continue; }
            if (!(rel == rel) || isinf(rel)) { R.out[i].status = IBB_ENUMERIC; R.done[i] = 1; continue; }
            if (R.out[i].cycles >= c->d.max_cycles) { R.out[i].status = IBB_ENOCONV; R.done[i] = 1; continue; }
            g->hflags[i] = 1;
            any = true;
        }
        if (!any && !anyg) break;
        if (any) {
            if (g->hflags != g->dflags) {
                GCHK(hipMemcpyAsync(g->flags, g->hflags.data(), n * sizeof(int), hipMemcpyHostToDevice, g->s));
                g->dflags = g->hflags;
            }
            GCHK(hipGraphLaunch(g->exec[vel ? 1 : 0], g->s));
        }
        if (anyg) {
            for (int i = 0; i < n; ++i) {
                if (!ran[i]) continue;
                ibb_ctx *c = g->m[i];
                if ((st = gcr_launch(gr[i]))) return st;
                GCHK(hipMemcpyAsync(g->norms + i, c->scalar, sizeof(double), hipMemcpyDeviceToDevice, c->s));
            }
            for (int k = 0; k < nside; ++k) {
                GCHK(hipEventRecord(g->sev[k], g->side[k]));
                GCHK(hipStreamWaitEvent(g->s, g->sev[k], 0));
            }
        }
        h.assign(n, 0.0);
        GCHK(hipMemcpyAsync(h.data(), g->norms, n * sizeof(double), hipMemcpyDeviceToHost, g->s));
        GCHK(hipStreamSynchronize(g->s));
        for (int i = 0; i < n; ++i) {
            if (ran[i]) {
                gcr_account(gr[i], sqrt(h[i]));
                continue;
            }
            if (!g->hflags[i]) continue;
            R.out[i].cycles++;
            R.out[i].vcycles += g->refined ? g->inner : 1;
            R.rel[i] = sqrt(h[i]) / R.nb[i];
        }
    }
    for (int i = 0; i < n; ++i) {
        if (side[i] < 0) continue;
        gcr_finish(gr[i]);
        R.rel[i] = gr[i].rel;
        g->m[i]->s = g->s;
    }
    for (int i = 0; i < n; ++i)
        if (side[i] < 0) R.out[i].relres = R.rel[i];
    return IBB_OK;
}

// run the members on the group's stream for the duration of a call
struct Borrow {
    ibb_group *g;
    std::vector<hipStream_t> saved;
    explicit Borrow(ibb_group *gg) : g(gg)
    {
        for (ibb_ctx *c : g->m) {
            saved.push_back(c->s);
            c->s = g->s;
        }
    }
    ~Borrow()
    {
        for (size_t i = 0; i < g->m.size(); ++i) g->m[i]->s = saved[i];
    }
};

// order the group's stream after the members' streams (enter) and the
// members' streams after the group's (leave)
ibb_status join_in(ibb_group *g)
{
    for (ibb_ctx *c : g->m) {
        GCHK(hipEventRecord(g->ev[4], c->s));
        GCHK(hipStreamWaitEvent(g->s, g->ev[4], 0));
    }
    return IBB_OK;
}

ibb_status join_out(ibb_group *g, const std::vector<hipStream_t> &streams)
{
    GCHK(hipEventRecord(g->ev[4], g->s));
    for (hipStream_t s : streams) GCHK(hipStreamWaitEvent(s, g->ev[4], 0));
    return IBB_OK;
}

}  // namespace

extern "C" {

ibb_status ibb_group_footprint_bytes(ibb_ctx *const *ctxs, int n, size_t *bytes)
{
    ibb_status st = check_members(ctxs, n);
    if (st) return st;
    if (!bytes) return IBB_EINVAL;
    std::vector<ibb_ctx *> m(ctxs, ctxs + n);
    Plan P;
    const ibb_desc &d = m[0]->d;
    build_plan(P, m, d.precision == IBB_FP32_REFINED, d.inner_cycles, d.nu1, d.nu2);
    *bytes = group_bytes(P, n);
    return IBB_OK;
}

ibb_status ibb_group_create(ibb_ctx *const *ctxs, int n, void *workspace, size_t bytes, ibb_group **out)
{
    if (!out) return IBB_EINVAL;
    *out = nullptr;
    ibb_status st = check_members(ctxs, n);
    if (st) return st;
    if (!workspace) return IBB_EINVAL;
    ibb_group *g = new ibb_group();
    g->m.assign(ctxs, ctxs + n);
    const ibb_desc &d = g->m[0]->d;
    g->refined = d.precision == IBB_FP32_REFINED;
    g->inner = d.inner_cycles > 0 ? d.inner_cycles : 1;
    g->nu1 = d.nu1;
    g->nu2 = d.nu2;
    build_plan(g->plan, g->m, g->refined, g->inner, g->nu1, g->nu2);
    if (bytes < group_bytes(g->plan, n)) {
        delete g;
        return IBB_ENOMEM;
    }
    Carver cv{(char *)workspace, 0, false};
    g->ent = cv.take<BEntry>(g->plan.ent.size());
    g->cent = cv.take<BCoarse>(g->plan.cent.size());
    g->flags = cv.take<int>(n);
    g->norms = cv.take<double>(n);
    g->counts = cv.take<int>(4 * (size_t)n);
    g->hflags.assign(n, 0);
    g->dflags.assign(n, 0);
    g->active.assign(n, 1);
    auto bail = [&](const char *what, hipError_t e) {
        fprintf(stderr, "ibb_group_create: %s: %s\n", what, hipGetErrorString(e));
        for (int v = 0; v < 2; ++v)
            if (g->exec[v]) (void)hipGraphExecDestroy(g->exec[v]);
        for (hipEvent_t &e2 : g->ev)
            if (e2) (void)hipEventDestroy(e2);
        if (g->s) (void)hipStreamDestroy(g->s);
        delete g;
        return IBB_EDEVICE;
    };
    hipError_t e = hipStreamCreateWithFlags(&g->s, hipStreamNonBlocking);
    if (e != hipSuccess) return bail("stream", e);
    for (hipEvent_t &ev : g->ev)
        if ((e = hipEventCreate(&ev)) != hipSuccess) return bail("event", e);
    // the members' pending work (their tables, coefficients) comes first
    for (ibb_ctx *c : g->m) {
        if ((e = hipEventRecord(g->ev[4], c->s)) != hipSuccess) return bail("event record", e);
        if ((e = hipStreamWaitEvent(g->s, g->ev[4], 0)) != hipSuccess) return bail("stream wait", e);
    }
    if (!g->plan.ent.empty() &&
        (e = hipMemcpyAsync(g->ent, g->plan.ent.data(), g->plan.ent.size() * sizeof(BEntry), hipMemcpyHostToDevice,
                            g->s)) != hipSuccess)
        return bail("entries", e);
    if (!g->plan.cent.empty() &&
        (e = hipMemcpyAsync(g->cent, g->plan.cent.data(), g->plan.cent.size() * sizeof(BCoarse),
                            hipMemcpyHostToDevice, g->s)) != hipSuccess)
        return bail("coarse entries", e);
    if ((e = hipMemcpyAsync(g->flags, g->dflags.data(), n * sizeof(int), hipMemcpyHostToDevice, g->s)) != hipSuccess)
        return bail("flags", e);
    if ((e = hipStreamSynchronize(g->s)) != hipSuccess) return bail("sync", e);
    for (int v = 0; v < 2; ++v) {
        hipGraph_t graph = nullptr;
        if ((e = hipStreamBeginCapture(g->s, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return bail("begin capture", e);
        emit_ops(g, g->plan.ops[v]);
        e = hipStreamEndCapture(g->s, &graph);
        if (e != hipSuccess) return bail("end capture", e);
        e = hipGraphInstantiate(&g->exec[v], graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return bail("instantiate", e);
    }
    *out = g;
    return IBB_OK;
}

ibb_status ibb_group_set_active(ibb_group *g, int member, int active)
{
    if (!g || member < 0 || member >= (int)g->m.size() || (active != 0 && active != 1)) return IBB_EINVAL;
    g->active[member] = (char)active;
    return IBB_OK;
}

ibb_status ibb_group_destroy(ibb_group *g)
{
    if (!g) return IBB_EINVAL;
    (void)hipStreamSynchronize(g->s);
    for (int v = 0; v < 2; ++v)
        if (g->exec[v]) (void)hipGraphExecDestroy(g->exec[v]);
    for (hipEvent_t &e : g->ev)
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t sd : g->side) {
        (void)hipStreamSynchronize(sd);
        (void)hipStreamDestroy(sd);
    }
    for (hipEvent_t e : g->sev)
        if (e) (void)hipEventDestroy(e);
    if (g->s) (void)hipStreamDestroy(g->s);
    delete g;
    return IBB_OK;
}

const char *ibb_group_last_error(const ibb_group *g) { return g ? g->err.c_str() : ""; }

ibb_status ibb_group_projection_step(ibb_group *g, ibb_solve_stats *per_ctx)
{
    if (!g) return IBB_EINVAL;
    const int n = (int)g->m.size();
    for (int i = 0; i < n; ++i)
        if (g->active[i] && !g->m[i]->have_coefs) {
            g->err = "ibb_group_projection_step: coefficients not built";
            return IBB_ESTATE;
        }
    ibb_status st = join_in(g);
    if (st) return st;
    GroupSolve su, sp;
    std::vector<hipStream_t> streams;
    for (ibb_ctx *c : g->m) streams.push_back(c->s);
    {
        Borrow b(g);
        for (int i = 0; i < n; ++i)
            if (g->active[i]) proj_viscous_rhs(g->m[i]);
        GCHK(hipEventRecord(g->ev[0], g->s));
        if ((st = group_solve(g, true, su))) return st;
        GCHK(hipEventRecord(g->ev[1], g->s));
        for (int i = 0; i < n; ++i)
            if (g->active[i]) proj_pressure_rhs(g->m[i]);
        GCHK(hipEventRecord(g->ev[2], g->s));
        if ((st = group_solve(g, false, sp))) return st;
        GCHK(hipEventRecord(g->ev[3], g->s));
        for (int i = 0; i < n; ++i)
            if (g->active[i]) proj_finish(g->m[i]);
        GCHK(hipGetLastError());
        GCHK(hipStreamSynchronize(g->s));
    }
    if ((st = join_out(g, streams))) return st;
    float tu = 0, tp = 0;
    (void)hipEventElapsedTime(&tu, g->ev[0], g->ev[1]);
    (void)hipEventElapsedTime(&tp, g->ev[2], g->ev[3]);
    ibb_status worst = IBB_OK;
    for (int i = 0; i < n; ++i) {
        if (!g->active[i]) {
            if (per_ctx) memset(per_ctx + i, 0, sizeof(ibb_solve_stats));
            continue;
        }
        fill_stats(g->m[i], su.out[i], sp.out[i], tu, tp, per_ctx ? per_ctx + i : nullptr);
        if (!worst && su.out[i].status) worst = (ibb_status)su.out[i].status;
        if (!worst && sp.out[i].status) worst = (ibb_status)sp.out[i].status;
    }
    if (worst) g->err = "a member's solve did not converge (see its statistics)";
    return worst;
}

ibb_status ibb_group_lagrangian_update(ibb_group *g, ibb_lag_stats *per_ctx)
{
    if (!g) return IBB_EINVAL;
    const int n = (int)g->m.size();
    for (int i = 0; i < n; ++i)
        if (g->active[i] && !g->m[i]->have_coefs) {
            g->err = "ibb_group_lagrangian_update: coefficients not built";
            return IBB_ESTATE;
        }
    ibb_status st = join_in(g);
    if (st) return st;
    std::vector<hipStream_t> streams;
    for (ibb_ctx *c : g->m) streams.push_back(c->s);
    std::vector<int> cnt(4 * (size_t)n, 0);
    {
        Borrow b(g);
        GCHK(hipEventRecord(g->ev[0], g->s));
        for (int i = 0; i < n; ++i) {
            ibb_ctx *c = g->m[i];
            if (!g->active[i]) continue;
            if ((st = lag_launch(c))) {
                g->err = c->err;
                return st;
            }
            GCHK(hipMemcpyAsync(g->counts + 4 * i, c->counters, 4 * sizeof(int), hipMemcpyDeviceToDevice, g->s));
        }
        GCHK(hipEventRecord(g->ev[1], g->s));
        GCHK(hipMemcpyAsync(cnt.data(), g->counts, 4 * n * sizeof(int), hipMemcpyDeviceToHost, g->s));
        GCHK(hipGetLastError());
        GCHK(hipStreamSynchronize(g->s));
    }
    if ((st = join_out(g, streams))) return st;
    float t = 0;
    (void)hipEventElapsedTime(&t, g->ev[0], g->ev[1]);
    if (per_ctx)
        for (int i = 0; i < n; ++i) {
            per_ctx[i].n_broken = cnt[4 * i];
            per_ctx[i].n_alive = cnt[4 * i + 1];
            per_ctx[i].t_ms = t;
            per_ctx[i].n_fragments = g->m[i]->d.track_fragments ? cnt[4 * i + 2] : -1;
            per_ctx[i].n_detached = g->m[i]->d.track_fragments ? cnt[4 * i + 3] : -1;
        }
    return IBB_OK;
}

}  // extern "C"
