// Galerkin coarse operators of the viscous system.  Sec. "Numerical
// Concerns" reports slow multigrid convergence at large mu_max with
// rediscretised coarse operators and names, as its second remedy, coarse
// operators that satisfy the Galerkin condition:
//     A_{l+1} = R_l A_l P_l,
// R_l the full-weighting restriction and P_l the linear prolongation of the
// V-cycle (Sec. "Multigrid"), with the same boundary rules as the transfer
// kernels.  This file builds those operators on the device, in the slot
// layout of kernels.h, and provides what a V-cycle needs on such a level:
// the smoother, the residual and the coarsest inverse.
//
// Smoother: R A P couples points of one colour, so a red-black pass updates
// every point of its (component, colour) set from the values the set held
// before the pass (Jacobi within the set, Gauss-Seidel from set to set); on
// a rediscretised level that is exactly the red-black Gauss-Seidel sweep.
#include "common.h"
#include "kernels.h"

#pragma clang fp contract(on)

namespace ibmg {

namespace {

constexpr int GAL_BUILD_THREADS = 64;

// one term of a finest-level row: column (component, entry) and its weight
struct GTerm {
    long long idx;
    double v;
    int comp;
};

// The terms of row (A, i, j, k) of the finest viscous operator
// A_u = (sigma rho / dt) I - Re^-1 D.(mu (D u + D u^T)) (eq:NSdis1-1,
// eq:divergencePartial): the same references, reflections and coefficient
// sums as the smoother's row, written as (column, weight) pairs; a
// reference that reflects onto the row itself stays a separate term.
template <int D, int A>
__device__ inline int u_terms(const Grid &g, const CoefU<double> &cf, double mass, double cvisc, int i, int j, int k,
                              GTerm *t)
{
    const int q[3] = {i, j, k};
    const long long f = at(g, i, j, k);
    const int ma = face_mask(A);
    int qa_m[3] = {i, j, k}, qa_p[3] = {i, j, k};
    qa_m[A] -= 1;
    qa_p[A] += 1;
    int n = 0;
    auto add = [&](Ref r, int comp, double v) {
        if (r.s == 0) return;
        t[n].idx = r.idx;
        t[n].comp = comp;
        t[n].v = r.s > 0 ? v : -v;
        ++n;
    };
    const double cp = 2.0 * ld(cf.muc, ref_at(g, 0, ROLE_C, i, j, k));
    const double cm = 2.0 * ld(cf.muc, ref_at(g, 0, ROLE_C, qa_m[0], qa_m[1], qa_m[2]));
    double dsum = cp + cm;
    add(ref_at(g, ma, ROLE_V, qa_p[0], qa_p[1], qa_p[2]), A, -cvisc * cp);
    add(ref_at(g, ma, ROLE_V, qa_m[0], qa_m[1], qa_m[2]), A, -cvisc * cm);
#pragma unroll
    for (int bi = 0; bi < D - 1; ++bi) {
        const int B = bi < A ? bi : bi + 1;
        const int c = 3 - A - B;
        const int mb = face_mask(B), mem = edge_mask(D, c);
        int qb_p[3] = {q[0], q[1], q[2]}, qb_m[3] = {q[0], q[1], q[2]};
        qb_p[B] += 1;
        qb_m[B] -= 1;
        int qbp_am[3] = {qb_p[0], qb_p[1], qb_p[2]};
        qbp_am[A] -= 1;
        const double mp = ld(cf.mue[c], ref_at(g, mem, ROLE_C, qb_p[0], qb_p[1], qb_p[2]));
        const double mm = ld(cf.mue[c], ref_at(g, mem, ROLE_C, i, j, k));
        dsum += mp + mm;
        add(ref_at(g, ma, ROLE_V, qb_p[0], qb_p[1], qb_p[2]), A, -cvisc * mp);
        add(ref_at(g, ma, ROLE_V, qb_m[0], qb_m[1], qb_m[2]), A, -cvisc * mm);
        add(ref_at(g, mb, ROLE_V, qb_p[0], qb_p[1], qb_p[2]), B, -cvisc * mp);
        add(ref_at(g, mb, ROLE_V, qbp_am[0], qbp_am[1], qbp_am[2]), B, cvisc * mp);
        add(ref_at(g, mb, ROLE_V, i, j, k), B, cvisc * mm);
        add(ref_at(g, mb, ROLE_V, qa_m[0], qa_m[1], qa_m[2]), B, -cvisc * mm);
    }
    t[n].idx = f;
    t[n].comp = A;
    t[n].v = mass * cf.rho[A][f] + cvisc * dsum;
    return n + 1;
}

template <int D>
__device__ inline int u_terms_any(int a, const Grid &g, const CoefU<double> &cf, double mass, double cvisc, int i,
                                  int j, int k, GTerm *t)
{
    if (a == 0) return u_terms<D, 0>(g, cf, mass, cvisc, i, j, k, t);
    if (D == 3 && a == 2) return u_terms<D, D == 3 ? 2 : 0>(g, cf, mass, cvisc, i, j, k, t);
    return u_terms<D, 1>(g, cf, mass, cvisc, i, j, k, t);
}

// offset of column index J from row index I along an axis, inside the box
// range [lo, lo + n); on a periodic axis (period > 0) the offset of least
// magnitude congruent to J - I, the more negative one on a tie
__device__ inline bool gal_delta(int diff, int lo, int n, int period, int &delta)
{
    if (period == 0) {
        if (diff < lo || diff >= lo + n) return false;
        delta = diff;
        return true;
    }
    bool found = false;
    int best = 0;
    for (int t = lo; t < lo + n; ++t) {
        const int m = ((t - diff) % period + period) % period;
        if (m == 0 && (!found || abs(t) < abs(best))) {
            best = t;
            found = true;
        }
    }
    delta = best;
    return found;
}

// entry of the unknown of component b at offset dl from q (periodic axes
// wrap); false when no unknown sits there
__device__ inline bool gal_col(const Grid &g, int b, const int q[3], const int dl[3], long long &e)
{
    int p[3] = {0, 0, 0};
    for (int d = 0; d < g.D; ++d) {
        int t = q[d] + dl[d];
        if (g.bc[d] == AX_PERIODIC) {
            t = ((t % g.n[d]) + g.n[d]) % g.n[d];
        } else {
            int lo, hi;
            unk_range(g, d, d == b, lo, hi);
            if (t < lo || t > hi) return false;
        }
        p[d] = t;
    }
    e = at(g, p[0], p[1], p[2]);
    return true;
}

// Rows of component a of the coarse operator, column component b: one
// thread per row accumulates, over every path row -> restriction tap f ->
// fine entry (f, g) -> prolongation tap J, the product R(I, f) A(f, g)
// P(g, J) into its slot for J (LDS, one column per thread), then stores
// the box.  The order of the paths is fixed, so the sums are repeatable.
template <int D, bool FROM0>
__global__ void __launch_bounds__(GAL_BUILD_THREADS) k_gal_build(Grid gf, Grid gc, VelBox rows, CoefU<double> cu,
                                                                 double mass, double cvisc, GalOpC<double> fine,
                                                                 GalOp<double> out, int *err)
{
    extern __shared__ double gacc[];   // [GAL_MAX_BOX][GAL_BUILD_THREADS]
    const int a = blockIdx.y / D, b = blockIdx.y % D;
    int I, J, K;
    if (!box_pos(rows.b[a], blockIdx.x * blockDim.x + threadIdx.x, I, J, K)) return;
    const int Q[3] = {I, J, K};
    const GalBox bx = gal_box(D, a, b);
    const int ns = bx.n[0] * bx.n[1] * bx.n[2];
    double *acc = gacc + threadIdx.x;
    for (int s = 0; s < ns; ++s) acc[s * GAL_BUILD_THREADS] = 0.0;
    // restriction taps on the fine grid, resolved as the transfer kernels do
    int fq[3][4], nf[3];
    double fw[3][4];
    for (int d = 0; d < 3; ++d) {
        if (d >= D) {
            nf[d] = 1;
            fq[d][0] = 0;
            fw[d][0] = 1.0;
            continue;
        }
        int raw[4];
        double w[4];
        nf[d] = rst_weights(d == a, Q[d], raw, w);
        for (int t = 0; t < nf[d]; ++t) {
            int q = raw[t], sg = 1;
            const bool live = resolve(gf, d, d == a, ROLE_V, q, sg);
            fq[d][t] = live ? q : 0;
            fw[d][t] = live ? (sg > 0 ? w[t] : -w[t]) : 0.0;
        }
    }
    int bad = 0;
    // add rv P(g, .) for the fine unknown g of component b at (gi, gj, gk)
    auto scatter = [&](int gi, int gj, int gk, double rv) {
        const int G3[3] = {gi, gj, gk};
        int cq[3][2];
        double cw[3][2];
        for (int d = 0; d < 3; ++d) {
            if (d >= D) {
                cq[d][0] = cq[d][1] = 0;
                cw[d][0] = 1.0;
                cw[d][1] = 0.0;
                continue;
            }
            int raw[2];
            double w[2];
            const int n = prl_weights(d == b, G3[d], raw, w);
            if (n == 1) {
                raw[1] = raw[0];
                w[1] = 0.0;
            }
            for (int t = 0; t < 2; ++t) {
                int q = raw[t], sg = 1;
                const bool live = resolve(gc, d, d == b, ROLE_V, q, sg);
                cq[d][t] = live ? q : 0;
                cw[d][t] = live ? (sg > 0 ? w[t] : -w[t]) : 0.0;
            }
        }
        for (int c = 0; c < 2; ++c)
            for (int bb = 0; bb < 2; ++bb)
                for (int aa = 0; aa < 2; ++aa) {
                    const double p = cw[0][aa] * cw[1][bb] * cw[2][c];
                    if (p == 0.0) continue;
                    const int Jq[3] = {cq[0][aa], cq[1][bb], cq[2][c]};
                    int dl[3] = {0, 0, 0}, ok = 1;
                    for (int d = 0; d < D; ++d)
                        ok &= gal_delta(Jq[d] - Q[d], bx.lo[d], bx.n[d], gc.bc[d] == AX_PERIODIC ? gc.n[d] : 0,
                                        dl[d]);
                    if (!ok) {
                        bad = 1;
                        continue;
                    }
                    const int s = (dl[0] - bx.lo[0]) + bx.n[0] * ((dl[1] - bx.lo[1]) + bx.n[1] * (dl[2] - bx.lo[2]));
                    acc[s * GAL_BUILD_THREADS] += rv * p;
                }
    };
    for (int c = 0; c < nf[2]; ++c)
        for (int bb = 0; bb < nf[1]; ++bb)
            for (int aa = 0; aa < nf[0]; ++aa) {
                const double r = fw[0][aa] * fw[1][bb] * fw[2][c];
                if (r == 0.0) continue;
                const int F3[3] = {fq[0][aa], fq[1][bb], fq[2][c]};
                if (FROM0) {
                    GTerm t[1 + 2 + 6 * (D - 1)];
                    const int n = u_terms_any<D>(a, gf, cu, mass, cvisc, F3[0], F3[1], F3[2], t);
                    for (int m = 0; m < n; ++m) {
                        if (t[m].comp != b) continue;
                        int gi, gj, gk;
                        decode(gf, t[m].idx, gi, gj, gk);
                        scatter(gi, gj, gk, r * t[m].v);
                    }
                } else {
                    const GalBox fb = gal_box(D, a, b);
                    const long long ef = at(gf, F3[0], F3[1], F3[2]);
                    const double *__restrict__ v = fine.v[a] + (long long)gal_first_slot(D, a, b) * gf.nel;
                    int s = 0;
                    for (int dz = 0; dz < fb.n[2]; ++dz)
                        for (int dy = 0; dy < fb.n[1]; ++dy)
                            for (int dx = 0; dx < fb.n[0]; ++dx, ++s) {
                                const double w = v[(long long)s * gf.nel + ef];
                                if (w == 0.0) continue;
                                const int dl[3] = {fb.lo[0] + dx, fb.lo[1] + dy, fb.lo[2] + dz};
                                long long eg;
                                if (!gal_col(gf, b, F3, dl, eg)) continue;
                                int gi, gj, gk;
                                decode(gf, eg, gi, gj, gk);
                                scatter(gi, gj, gk, r * w);
                            }
                }
            }
    if (bad) atomicOr(err, 1);
    double *__restrict__ o = out.v[a] + (long long)gal_first_slot(D, a, b) * gc.nel + at(gc, I, J, K);
    for (int s = 0; s < ns; ++s) o[(long long)s * gc.nel] = acc[s * GAL_BUILD_THREADS];
}

__global__ void __launch_bounds__(256) k_gal_cast(const double *__restrict__ src, float *dst, long long n)
{
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x)
        dst[t] = (float)src[t];
}

// Where the offsets -2 .. 2 from a row's position lead along each axis,
// for a cell-centred (c = 0) and a vertex-centred (c = 1) column lattice:
// the (wrapped) coordinate of the unknown there, or, where no unknown sits,
// a coordinate of the array's ghost or fixed-face layer (never an unknown).
// The build leaves every slot whose column is no unknown at zero, so such a
// slot adds 0 times a finite value and the row needs no test per entry.
struct AxisReach {
    int p[3][2][5];
};

__device__ inline AxisReach axis_reach(const Grid &g, const int q[3])
{
    AxisReach r;
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int o = 0; o < 5; ++o) {
                if (d >= g.D) {
                    r.p[d][c][o] = 0;   // only offset 0 is used
                    continue;
                }
                int t = q[d] + o - 2;
                if (g.bc[d] == AX_PERIODIC) {
                    t = t < 0 ? t + g.n[d] : (t >= g.n[d] ? t - g.n[d] : t);
                    t = t < 0 ? t + g.n[d] : (t >= g.n[d] ? t - g.n[d] : t);   // periods of 1 or 2
                } else {
                    int lo, hi;
                    unk_range(g, d, c, lo, hi);
                    if (t < lo) t = t < -1 ? -1 : t;
                    else if (t > hi) t = t > g.n[d] + 1 ? g.n[d] + 1 : t;
                }
                r.p[d][c][o] = t;
            }
    return r;
}

// acc += sum over the box of column component C of w * x[column] (the
// diagonal, offset 0 of the row's own component, goes to dg and is left out
// of acc when SKIP); the box has compile-time extents, so the loop unrolls
// and every load of the row issues independently
template <typename T, int D, int A, int C, bool SKIP>
__device__ inline void gal_row_box(const Grid &g, long long e, const AxisReach &rch, const T *__restrict__ v,
                                   const T *__restrict__ xc, T &acc, T &dg)
{
    constexpr GalBox bx = gal_box(D, A, C);
    constexpr int first = gal_first_slot(D, A, C);
#pragma unroll
    for (int dz = 0; dz < bx.n[2]; ++dz)
#pragma unroll
        for (int dy = 0; dy < bx.n[1]; ++dy)
#pragma unroll
            for (int dx = 0; dx < bx.n[0]; ++dx) {
                const int s = first + dx + bx.n[0] * (dy + bx.n[1] * dz);
                const int ox = bx.lo[0] + dx, oy = bx.lo[1] + dy, oz = bx.lo[2] + dz;
                const T w = v[(long long)s * g.nel + e];
                if (C == A && ox == 0 && oy == 0 && oz == 0) {
                    dg = w;
                    if (SKIP) continue;
                }
                const int px = rch.p[0][C == 0][ox + 2];
                const int py = rch.p[1][C == 1][oy + 2];
                const int pz = rch.p[2][C == 2][oz + 2];
                acc += w * xc[at(g, px, py, pz)];
            }
}

// sum over the row's slots of w * x[column], the diagonal left out when
// SKIP (the smoother) and returned in dg
template <typename T, int D, int A, bool SKIP>
__device__ inline T gal_row(const Grid &g, const int q[3], long long e, const T *__restrict__ v, const VelArrC<T> &x,
                            T &dg)
{
    const AxisReach rch = axis_reach(g, q);
    T acc = T(0);
    gal_row_box<T, D, A, 0, SKIP>(g, e, rch, v, x.c[0], acc, dg);
    gal_row_box<T, D, A, 1, SKIP>(g, e, rch, v, x.c[1], acc, dg);
    if (D == 3) gal_row_box<T, D, A, D == 3 ? 2 : 1, SKIP>(g, e, rch, v, x.c[D == 3 ? 2 : 1], acc, dg);
    return acc;
}

template <typename T, int D, int A>
__global__ void __launch_bounds__(256) k_gal_smooth(Grid g, Box box, int colour, GalOpC<T> op,
                                                    const T *__restrict__ b, VelArrC<T> x, T *y)
{
    int i, j, k;
    if (!box_pos(box, blockIdx.x * blockDim.x + threadIdx.x, i, j, k)) return;
    const long long e = at(g, i, j, k);
    if (((i + j + k) & 1) != colour) {
        y[e] = x.c[A][e];
        return;
    }
    const int q[3] = {i, j, k};
    T dg = T(1);
    const T off = gal_row<T, D, A, true>(g, q, e, op.v[A], x, dg);
    y[e] = (b[e] - off) / dg;
}

template <typename T, int D, int A>
__device__ inline void gal_resid_point(const Grid &g, const Box &box, int t, const GalOpC<T> &op, const VelArrC<T> &b,
                                       const VelArrC<T> &x, const VelArr<T> &r)
{
    int i, j, k;
    if (!box_pos(box, t, i, j, k)) return;
    const long long e = at(g, i, j, k);
    const int q[3] = {i, j, k};
    T dg;
    const T ax = gal_row<T, D, A, false>(g, q, e, op.v[A], x, dg);
    r.c[A][e] = b.c[A][e] - ax;
}

template <typename T, int D>
__global__ void __launch_bounds__(256) k_gal_resid(Grid g, VelBox boxes, GalOpC<T> op, VelArrC<T> b, VelArrC<T> x,
                                                   VelArr<T> r)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.y == 0) gal_resid_point<T, D, 0>(g, boxes.b[0], t, op, b, x, r);
    else if (blockIdx.y == 1) gal_resid_point<T, D, 1>(g, boxes.b[1], t, op, b, x, r);
    else gal_resid_point<T, D, D == 3 ? 2 : 1>(g, boxes.b[D == 3 ? 2 : 1], t, op, b, x, r);
}

// row r of the coarsest operator as a dense row over the listed unknowns
template <int D>
__global__ void __launch_bounds__(64) k_gal_dense_assemble(Grid g, int n, const long long *__restrict__ uidx,
                                                           const int *__restrict__ ucomp, GalOpC<double> op,
                                                           double *Aw)
{
    const int r = threadIdx.x;
    if (r >= n) return;
    for (int j = 0; j < n; ++j) Aw[r * n + j] = 0.0;
    const int a = ucomp[r];
    const long long e = uidx[r];
    int q[3];
    decode(g, e, q[0], q[1], q[2]);
    int s = 0;
    for (int c = 0; c < D; ++c) {
        const GalBox bx = gal_box(D, a, c);
        const double *__restrict__ v = op.v[a];
        for (int dz = 0; dz < bx.n[2]; ++dz)
            for (int dy = 0; dy < bx.n[1]; ++dy)
                for (int dx = 0; dx < bx.n[0]; ++dx, ++s) {
                    const double w = v[(long long)s * g.nel + e];
                    if (w == 0.0) continue;
                    const int dl[3] = {bx.lo[0] + dx, bx.lo[1] + dy, bx.lo[2] + dz};
                    long long col;
                    if (!gal_col(g, c, q, dl, col)) continue;
                    for (int j = 0; j < n; ++j)
                        if (uidx[j] == col && ucomp[j] == c) {
                            Aw[r * n + j] += w;
                            break;
                        }
                }
    }
}

unsigned blocks_of(long long n, int threads) { return (unsigned)((n + threads - 1) / threads); }

}  // namespace

void launch_gal_build(int D, const Grid &gf, const Grid &gc, const CoefU<double> &cu, double mass, double cvisc,
                      const GalOpC<double> *fine, const GalOp<double> &out, int *err, hipStream_t s)
{
    VelBox rows;
    long long most = 0;
    for (int a = 0; a < 3; ++a) {
        rows.b[a] = a < D ? unk_box(gc, face_mask(a)) : Box{{0, 0, 0}, {0, 0, 0}};
        const long long n = (long long)rows.b[a].ext[0] * rows.b[a].ext[1] * rows.b[a].ext[2];
        most = n > most ? n : most;
    }
    const dim3 grid(blocks_of(most, GAL_BUILD_THREADS), D * D);
    const unsigned shm = GAL_MAX_BOX * GAL_BUILD_THREADS * sizeof(double);
    const GalOpC<double> f = fine ? *fine : GalOpC<double>{{nullptr, nullptr, nullptr}};
    if (D == 3) {
        if (fine) launch_timed_shm(k_gal_build<3, false>, grid, dim3(GAL_BUILD_THREADS), shm, s, gf, gc, rows, cu, mass,
                                   cvisc, f, out, err);
        else launch_timed_shm(k_gal_build<3, true>, grid, dim3(GAL_BUILD_THREADS), shm, s, gf, gc, rows, cu, mass,
                              cvisc, f, out, err);
    } else {
        if (fine) launch_timed_shm(k_gal_build<2, false>, grid, dim3(GAL_BUILD_THREADS), shm, s, gf, gc, rows, cu, mass,
                                   cvisc, f, out, err);
        else launch_timed_shm(k_gal_build<2, true>, grid, dim3(GAL_BUILD_THREADS), shm, s, gf, gc, rows, cu, mass,
                              cvisc, f, out, err);
    }
}

void launch_gal_to_f32(int D, const Grid &g, const GalOpC<double> &src, const GalOp<float> &dst, hipStream_t s)
{
    for (int a = 0; a < D; ++a) {
        const long long n = (long long)gal_row_slots(D, a) * g.nel;
        unsigned nb = blocks_of(n, 256);
        if (nb > 4096) nb = 4096;
        hipLaunchKernelGGL(k_gal_cast, dim3(nb), dim3(256), 0, s, src.v[a], dst.v[a], n);
    }
}

template <typename T>
void launch_gal_smooth(int D, const Grid &g, int a, int colour, const GalOpC<T> &op, const T *b, const VelArrC<T> &x,
                       T *y, hipStream_t s)
{
    const Box box = unk_box(g, face_mask(a));
    const long long n = (long long)box.ext[0] * box.ext[1] * box.ext[2];
    if (n <= 0) return;
    const dim3 grid(blocks_of(n, 256));
    if (D == 3) {
        if (a == 0) launch_timed(k_gal_smooth<T, 3, 0>, grid, dim3(256), s, g, box, colour, op, b, x, y);
        else if (a == 1) launch_timed(k_gal_smooth<T, 3, 1>, grid, dim3(256), s, g, box, colour, op, b, x, y);
        else launch_timed(k_gal_smooth<T, 3, 2>, grid, dim3(256), s, g, box, colour, op, b, x, y);
    } else {
        if (a == 0) launch_timed(k_gal_smooth<T, 2, 0>, grid, dim3(256), s, g, box, colour, op, b, x, y);
        else launch_timed(k_gal_smooth<T, 2, 1>, grid, dim3(256), s, g, box, colour, op, b, x, y);
    }
}

template <typename T>
void launch_gal_resid(int D, const Grid &g, const GalOpC<T> &op, const VelArrC<T> &b, const VelArrC<T> &x,
                      const VelArr<T> &r, hipStream_t s)
{
    VelBox boxes;
    long long most = 0;
    for (int a = 0; a < 3; ++a) {
        boxes.b[a] = a < D ? unk_box(g, face_mask(a)) : Box{{0, 0, 0}, {0, 0, 0}};
        const long long n = (long long)boxes.b[a].ext[0] * boxes.b[a].ext[1] * boxes.b[a].ext[2];
        most = n > most ? n : most;
    }
    if (most <= 0) return;
    const dim3 grid(blocks_of(most, 256), D);
    if (D == 3) launch_timed(k_gal_resid<T, 3>, grid, dim3(256), s, g, boxes, op, b, x, r);
    else launch_timed(k_gal_resid<T, 2>, grid, dim3(256), s, g, boxes, op, b, x, r);
}

void launch_gal_dense_inverse(int D, const Grid &g, int n, const long long *uidx, const int *ucomp,
                              const GalOpC<double> &op, double *Aw, double *M, hipStream_t s)
{
    if (n <= 0 || n > DENSE_LDS) return;
    if (D == 3) hipLaunchKernelGGL(k_gal_dense_assemble<3>, dim3(1), dim3(64), 0, s, g, n, uidx, ucomp, op, Aw);
    else hipLaunchKernelGGL(k_gal_dense_assemble<2>, dim3(1), dim3(64), 0, s, g, n, uidx, ucomp, op, Aw);
    launch_dense_gj(n, 0, Aw, M, s);
}

template void launch_gal_smooth<double>(int, const Grid &, int, int, const GalOpC<double> &, const double *,
                                        const VelArrC<double> &, double *, hipStream_t);
template void launch_gal_smooth<float>(int, const Grid &, int, int, const GalOpC<float> &, const float *,
                                       const VelArrC<float> &, float *, hipStream_t);
template void launch_gal_resid<double>(int, const Grid &, const GalOpC<double> &, const VelArrC<double> &,
                                       const VelArrC<double> &, const VelArr<double> &, hipStream_t);
template void launch_gal_resid<float>(int, const Grid &, const GalOpC<float> &, const VelArrC<float> &,
                                      const VelArrC<float> &, const VelArr<float> &, hipStream_t);

}  // namespace ibmg
