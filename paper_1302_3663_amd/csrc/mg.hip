// Multigrid kernels for the pressure system A_p = -D(beta G) (eq:NSdis4,
// eq:divergenceGrad) and the viscous system
// A_u = (sigma rho / dt) I - Re^-1 D.(mu (D u + D u^T)) (eq:NSdis1-1,
// eq:divergencePartial) on the staggered grid: red-black Gauss-Seidel
// (component by component, red then black), residual with a fused squared
// norm, full-weighting restriction, linear prolongation, and the direct
// solve on the coarsest level (Sec. "Multigrid").
//
// Every kernel is templated on the arithmetic type T (double, or float for
// the inner cycles of the refined solver).  A point more than one cell away
// from every boundary reads its neighbours at fixed offsets; points near a
// boundary resolve each neighbour through the boundary rules of common.h.
//
// Multiply-adds are fused only inside one source expression, never across
// statements, so a row computes the same bits in every kernel that inlines
// it (the launched passes and the one-workgroup coarse cycle).
#include <algorithm>

#include <hip/hip_ext.h>

#include "common.h"
#include "kernels.h"

#pragma clang fp contract(on)

namespace ibmg {

// ---------------------------------------------------------------------------
// rows of the two operators: (A x) at one unknown and the diagonal entry.
// Templated on the dimension D and (viscous) the component A so that every
// loop unrolls and all loads of a row issue together.
// ---------------------------------------------------------------------------
__device__ inline int self_sign(Ref r, long long c) { return (r.s != 0 && r.idx == c) ? r.s : 0; }

// the bi-th axis other than A
template <int A>
__device__ constexpr int other_axis(int bi) { return bi < A ? bi : bi + 1; }

template <typename T, int D>
__device__ inline void p_row_fast(const Grid &g, const T *__restrict__ x, const CoefP<T> &cf, T cvisc, int c, T &Ax,
                                  T &dg)
{
    const int st[3] = {1, g.NX, (int)g.NXY};
    T xn[2 * D], bt[2 * D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        xn[2 * a] = x[c + st[a]];
        xn[2 * a + 1] = x[c - st[a]];
        bt[2 * a] = cf.beta[a][c + st[a]];
        bt[2 * a + 1] = cf.beta[a][c];
    }
    const T xc = x[c];
    T acc = 0, d = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        acc += bt[2 * a] * (xc - xn[2 * a]) + bt[2 * a + 1] * (xc - xn[2 * a + 1]);
        d += bt[2 * a] + bt[2 * a + 1];
    }
    Ax = acc * cvisc;
    dg = d * cvisc;
}

template <typename T, int D>
__device__ inline void p_row_slow(const Grid &g, const T *__restrict__ x, const CoefP<T> &cf, T cvisc, int i, int j,
                                  int k, T &Ax, T &dg)
{
    const long long c = at(g, i, j, k);
    Ref rb[2 * D], rx[2 * D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        int qp[3] = {i, j, k}, qm[3] = {i, j, k};
        qp[a] += 1;
        qm[a] -= 1;
        rb[2 * a] = ref_at(g, face_mask(a), ROLE_C, qp[0], qp[1], qp[2]);
        rb[2 * a + 1] = ref_at(g, face_mask(a), ROLE_C, i, j, k);
        rx[2 * a] = ref_at(g, 0, ROLE_P, qp[0], qp[1], qp[2]);
        rx[2 * a + 1] = ref_at(g, 0, ROLE_P, qm[0], qm[1], qm[2]);
    }
    T bt[2 * D], xn[2 * D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        bt[2 * a] = ld(cf.beta[a], rb[2 * a]);
        bt[2 * a + 1] = ld(cf.beta[a], rb[2 * a + 1]);
        xn[2 * a] = ld(x, rx[2 * a]);
        xn[2 * a + 1] = ld(x, rx[2 * a + 1]);
    }
    const T xc = x[c];
    T acc = 0, d = 0;
#pragma unroll
    for (int t = 0; t < 2 * D; ++t) {
        acc += bt[t] * (xc - xn[t]);
        d += bt[t] * T(1 - self_sign(rx[t], c));
    }
    Ax = acc * cvisc;
    dg = d * cvisc;
}

// Constant viscosity, eq:NSdis1: the 2D + 1 point Laplacian of component A
// alone with unit coefficients (the viscosity is folded into cvisc), every
// neighbour resolved through the boundary rules.
template <typename T, int D, int A>
__device__ inline void u_row_slow_dec(const Grid &g, const T *__restrict__ ua, const T *__restrict__ rho, T mass,
                                      T cvisc, int i, int j, int k, T &Ax, T &dg)
{
    const long long f = at(g, i, j, k);
    const int ma = face_mask(A);
    Ref rp[D], rm[D];
#pragma unroll
    for (int b = 0; b < D; ++b) {
        int qp[3] = {i, j, k}, qm[3] = {i, j, k};
        qp[b] += 1;
        qm[b] -= 1;
        rp[b] = ref_at(g, ma, ROLE_V, qp[0], qp[1], qp[2]);
        rm[b] = ref_at(g, ma, ROLE_V, qm[0], qm[1], qm[2]);
    }
    const T xf = ua[f];
    T acc = 0, d = 0;
#pragma unroll
    for (int b = 0; b < D; ++b) {
        acc += (ld(ua, rp[b]) - xf) - (xf - ld(ua, rm[b]));
        d += T(1 - self_sign(rp[b], f)) + T(1 - self_sign(rm[b], f));
    }
    const T m = mass * rho[f];
    Ax = m * xf - cvisc * acc;
    dg = m + cvisc * d;
}

template <typename T, int D, int A>
__device__ inline void u_row_slow(const Grid &g, const VelArr<T> &x, const CoefU<T> &cf, T mass, T cvisc, int i, int j,
                                  int k, T &Ax, T &dg)
{
    if (cf.dec) {
        u_row_slow_dec<T, D, A>(g, x.c[A], cf.rho[A], mass, cvisc, i, j, k, Ax, dg);
        return;
    }
    const int q[3] = {i, j, k};
    const long long f = at(g, i, j, k);
    const int ma = face_mask(A);
    int qa_m[3] = {i, j, k}, qa_p[3] = {i, j, k};
    qa_m[A] -= 1;
    qa_p[A] += 1;
    // resolve every reference first (arithmetic only)
    const Ref rcp = ref_at(g, 0, ROLE_C, i, j, k);
    const Ref rcm = ref_at(g, 0, ROLE_C, qa_m[0], qa_m[1], qa_m[2]);
    const Ref rvp = ref_at(g, ma, ROLE_V, qa_p[0], qa_p[1], qa_p[2]);
    const Ref rvm = ref_at(g, ma, ROLE_V, qa_m[0], qa_m[1], qa_m[2]);
    Ref rmp[D - 1], rmm[D - 1], rap[D - 1], ram[D - 1], r0[D - 1], r1[D - 1], r2[D - 1], r3[D - 1];
#pragma unroll
    for (int bi = 0; bi < D - 1; ++bi) {
        const int B = other_axis<A>(bi);
        const int c = 3 - A - B;
        const int mb = face_mask(B), mem = edge_mask(D, c);
        int qb_p[3] = {q[0], q[1], q[2]}, qb_m[3] = {q[0], q[1], q[2]};
        qb_p[B] += 1;
        qb_m[B] -= 1;
        int qbp_am[3] = {qb_p[0], qb_p[1], qb_p[2]};
        qbp_am[A] -= 1;
        rmp[bi] = ref_at(g, mem, ROLE_C, qb_p[0], qb_p[1], qb_p[2]);
        rmm[bi] = ref_at(g, mem, ROLE_C, i, j, k);
        rap[bi] = ref_at(g, ma, ROLE_V, qb_p[0], qb_p[1], qb_p[2]);
        ram[bi] = ref_at(g, ma, ROLE_V, qb_m[0], qb_m[1], qb_m[2]);
        r0[bi] = ref_at(g, mb, ROLE_V, qb_p[0], qb_p[1], qb_p[2]);
        r1[bi] = ref_at(g, mb, ROLE_V, qbp_am[0], qbp_am[1], qbp_am[2]);
        r2[bi] = ref_at(g, mb, ROLE_V, i, j, k);
        r3[bi] = ref_at(g, mb, ROLE_V, qa_m[0], qa_m[1], qa_m[2]);
    }
    // then every load
    const T *__restrict__ ua = x.c[A];
    const T xf = ua[f];
    const T rho = cf.rho[A][f];
    const T cp = T(2) * ld(cf.muc, rcp), cm = T(2) * ld(cf.muc, rcm);
    const T vp = ld(ua, rvp), vm = ld(ua, rvm);
    T mp[D - 1], mm[D - 1], ap[D - 1], am[D - 1], b0[D - 1], b1[D - 1], b2[D - 1], b3[D - 1];
#pragma unroll
    for (int bi = 0; bi < D - 1; ++bi) {
        const int B = other_axis<A>(bi);
        const T *__restrict__ ub = x.c[B];
        const T *__restrict__ me = cf.mue[3 - A - B];
        mp[bi] = ld(me, rmp[bi]);
        mm[bi] = ld(me, rmm[bi]);
        ap[bi] = ld(ua, rap[bi]);
        am[bi] = ld(ua, ram[bi]);
        b0[bi] = ld(ub, r0[bi]);
        b1[bi] = ld(ub, r1[bi]);
        b2[bi] = ld(ub, r2[bi]);
        b3[bi] = ld(ub, r3[bi]);
    }
    T acc = cp * (vp - xf) - cm * (xf - vm);
    T d = cp * T(1 - self_sign(rvp, f)) + cm * T(1 - self_sign(rvm, f));
#pragma unroll
    for (int bi = 0; bi < D - 1; ++bi) {
        acc += mp[bi] * ((ap[bi] - xf) + (b0[bi] - b1[bi])) - mm[bi] * ((xf - am[bi]) + (b2[bi] - b3[bi]));
        d += mp[bi] * T(1 - self_sign(rap[bi], f)) + mm[bi] * T(1 - self_sign(ram[bi], f));
    }
    const T m = mass * rho;
    Ax = m * xf - cvisc * acc;
    dg = m + cvisc * d;
}

// Rows read through the ghost layer: every neighbour sits at a fixed
// offset.  Where the ghost across a boundary mirrors the point itself, the
// diagonal gains the reflection: coefficient x (1 - sign) instead of the
// coefficient alone.
template <typename T, int D>
__device__ inline void p_row(const Grid &g, const T *__restrict__ x, const CoefP<T> &cf, T cvisc, int i, int j, int k,
                             T &Ax, T &dg)
{
    const int c = (int)at(g, i, j, k);
    const int st[3] = {1, g.NX, (int)g.NXY};
    T xn[2 * D], bt[2 * D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        xn[2 * a] = x[c + st[a]];
        xn[2 * a + 1] = x[c - st[a]];
        bt[2 * a] = cf.beta[a][c + st[a]];
        bt[2 * a + 1] = cf.beta[a][c];
    }
    const T xc = x[c];
    const int q[3] = {i, j, k};
    T acc = 0, d = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        acc += bt[2 * a] * (xc - xn[2 * a]) + bt[2 * a + 1] * (xc - xn[2 * a + 1]);
        d += bt[2 * a] + bt[2 * a + 1];
        if (g.bc[a] != AX_PERIODIC) {
            if (q[a] == 0) d -= bt[2 * a + 1];                                         // even mirror
            if (q[a] == g.n[a] - 1) d += g.bc[a] == AX_INOUT ? bt[2 * a] : -bt[2 * a];  // odd at the outflow
        }
    }
    Ax = acc * cvisc;
    dg = d * cvisc;
}

// Constant viscosity through the ghost layer: component A alone, unit
// coefficients; a mirrored self-reference adds to the diagonal as in u_row.
// (r: the density at the face, read by the caller)
template <typename T, int D, int A>
__device__ inline void u_row_dec_r(const Grid &g, const T *__restrict__ ua, T r, T mass, T cvisc, int i, int j, int k,
                                   T &Ax, T &dg)
{
    const int f = (int)at(g, i, j, k);
    const int st[3] = {1, g.NX, (int)g.NXY};
    T vp[D], vm[D];
#pragma unroll
    for (int b = 0; b < D; ++b) {
        vp[b] = ua[f + st[b]];
        vm[b] = ua[f - st[b]];
    }
    const T xf = ua[f];
    const int q[3] = {i, j, k};
    T acc = 0, d = T(2 * D);
#pragma unroll
    for (int b = 0; b < D; ++b) {
        acc += (vp[b] - xf) - (xf - vm[b]);
        if (b != A && g.bc[b] != AX_PERIODIC) {
            if (q[b] == 0) d += T(1);                                              // odd mirror
            if (q[b] == g.n[b] - 1) d += g.bc[b] == AX_WALLS ? T(1) : T(-1);        // even at the outflow
        }
    }
    const T m = mass * r;
    Ax = m * xf - cvisc * acc;
    dg = m + cvisc * d;
}

template <typename T, int D, int A>
__device__ inline void u_row_dec(const Grid &g, const T *__restrict__ ua, const T *__restrict__ rho, T mass, T cvisc,
                                 int i, int j, int k, T &Ax, T &dg)
{
    u_row_dec_r<T, D, A>(g, ua, rho[at(g, i, j, k)], mass, cvisc, i, j, k, Ax, dg);
}

// u_a at the row's point and its axis neighbours, read from the uniform
// array at fixed offsets
template <typename T>
struct UaFlat {
    const T *__restrict__ p;
    int f;
    int st[3];
    __device__ T here() const { return p[f]; }
    __device__ T nb(int ax, int s) const { return p[f + s * st[ax]]; }
};

// The coupled viscous row (eq:NSdis1-1 with eq:divergencePartial) at uniform
// entry f, lattice position (i, j, k), with u_a read through `ua` (the
// uniform array, or a window of it) and every other field through f.  One
// body for every reader, so that all of them compute the same bits.
template <typename T, int D, int A, typename UA, typename XV>
__device__ inline void u_row_core(const Grid &g, const UA &ua, const XV &x, const CoefU<T> &cf, T rho, T mass, T cvisc,
                                  int f, int i, int j, int k, T &Ax, T &dg)
{
    const int st[3] = {1, g.NX, (int)g.NXY};
    const int sa = st[A];
    const T xf = ua.here();
    const T cp = T(2) * cf.muc[f], cm = T(2) * cf.muc[f - sa];
    const T vp = ua.nb(A, 1), vm = ua.nb(A, -1);
    T mp[D - 1], mm[D - 1], ap[D - 1], am[D - 1], b0[D - 1], b1[D - 1], b2[D - 1], b3[D - 1];
#pragma unroll
    for (int bi = 0; bi < D - 1; ++bi) {
        const int B = other_axis<A>(bi);
        const int sb = st[B];
        const T *__restrict__ ub = x.c[B];
        const T *__restrict__ me = cf.mue[3 - A - B];
        mp[bi] = me[f + sb];
        mm[bi] = me[f];
        ap[bi] = ua.nb(B, 1);
        am[bi] = ua.nb(B, -1);
        b0[bi] = ub[f + sb];
        b1[bi] = ub[f + sb - sa];
        b2[bi] = ub[f];
        b3[bi] = ub[f - sa];
    }
    const int q[3] = {i, j, k};
    T acc = cp * (vp - xf) - cm * (xf - vm);
    T d = cp + cm;
#pragma unroll
    for (int bi = 0; bi < D - 1; ++bi) {
        const int B = other_axis<A>(bi);
        acc += mp[bi] * ((ap[bi] - xf) + (b0[bi] - b1[bi])) - mm[bi] * ((xf - am[bi]) + (b2[bi] - b3[bi]));
        d += mp[bi] + mm[bi];
        if (g.bc[B] != AX_PERIODIC) {
            if (q[B] == 0) d += mm[bi];                                                  // odd mirror
            if (q[B] == g.n[B] - 1) d += g.bc[B] == AX_WALLS ? mp[bi] : -mp[bi];          // even at the outflow
        }
    }
    const T m = mass * rho;
    Ax = m * xf - cvisc * acc;
    dg = m + cvisc * d;
}

template <typename T, int D, int A>
__device__ inline void u_row(const Grid &g, const VelArr<T> &x, const CoefU<T> &cf, T mass, T cvisc, int i, int j,
                             int k, T &Ax, T &dg)
{
    const int f = (int)at(g, i, j, k);
    // read before the branch, which both forms take it in
    const T rho = cf.rho[A][f];
    if (cf.dec) {
        u_row_dec_r<T, D, A>(g, x.c[A], rho, mass, cvisc, i, j, k, Ax, dg);
        return;
    }
    const UaFlat<T> ua{x.c[A], f, {1, g.NX, (int)g.NXY}};
    u_row_core<T, D, A>(g, ua, x, cf, rho, mass, cvisc, f, i, j, k, Ax, dg);
}

// runtime-dimension entry points (coarsest dense assembly)
template <typename T>
__device__ inline void p_row_slow_any(const Grid &g, const T *x, const CoefP<T> &cf, T cvisc, int i, int j, int k, T &Ax,
                                      T &dg)
{
    if (g.D == 3) p_row_slow<T, 3>(g, x, cf, cvisc, i, j, k, Ax, dg);
    else p_row_slow<T, 2>(g, x, cf, cvisc, i, j, k, Ax, dg);
}

template <typename T>
__device__ inline void u_row_slow_any(const Grid &g, const VelArr<T> &x, const CoefU<T> &cf, T mass, T cvisc, int a,
                                      int i, int j, int k, T &Ax, T &dg)
{
    if (g.D == 3) {
        if (a == 0) u_row_slow<T, 3, 0>(g, x, cf, mass, cvisc, i, j, k, Ax, dg);
        else if (a == 1) u_row_slow<T, 3, 1>(g, x, cf, mass, cvisc, i, j, k, Ax, dg);
        else u_row_slow<T, 3, 2>(g, x, cf, mass, cvisc, i, j, k, Ax, dg);
    } else {
        if (a == 0) u_row_slow<T, 2, 0>(g, x, cf, mass, cvisc, i, j, k, Ax, dg);
        else u_row_slow<T, 2, 1>(g, x, cf, mass, cvisc, i, j, k, Ax, dg);
    }
}

// ---------------------------------------------------------------------------
// Workgroups go to the chip's 8 XCDs in turn (workgroup b to XCD b mod 8),
// and each XCD has its own L2.  Renumbered so that each XCD works through one
// contiguous range of the index space, the rows and planes that neighbouring
// points share stay in one L2.  A bijection of [0, gridDim.x); remap = 0
// keeps the hardware order.  Measured on the smoothers: 10% faster on arrays
// of 4.4 M entries, 5-7% slower on 34.5 M, where a plane's reuse window no
// longer fits an XCD's L2 and the shared last-level cache did better with
// every XCD on neighbouring rows; hence the size limit below.
// ---------------------------------------------------------------------------
constexpr long long XCD_REMAP_MAX_NEL = 16ll << 20;

__device__ inline unsigned xcd_block(int remap)
{
    constexpr unsigned NXCD = 8;
    const unsigned nb = gridDim.x, b = blockIdx.x;
    if (!remap) return b;
    const unsigned q = nb / NXCD, r = nb % NXCD, x = b % NXCD;
    return x * q + (x < r ? x : r) + b / NXCD;
}

// ---------------------------------------------------------------------------
// smoothers: one colour of one component; the updated value is also written
// to its ghost images so that later passes read it at fixed offsets.  Each
// point reads its own x and b before its row, so that all of its loads are
// in flight together (read after the row, they cost a second round trip).
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ void __launch_bounds__(256) k_smooth_p(Grid g, Box box, const T *__restrict__ b, T *x, CoefP<T> cf, T cvisc,
                                                  int colour, int remap)
{
    int i, j, k;
    if (!box_colour_pos(box, colour, xcd_block(remap) * blockDim.x + threadIdx.x, i, j, k)) return;
    const long long c = at(g, i, j, k);
    const T bc = b[c], xc = x[c];
    T Ax, dg;
    p_row<T, D>(g, x, cf, cvisc, i, j, k, Ax, dg);
    const T xn = xc + (bc - Ax) / dg;
    x[c] = xn;
    write_images(g, 0, ROLE_P, x, i, j, k, xn);
}

template <typename T, int D, int A>
__global__ void __launch_bounds__(256) k_smooth_u(Grid g, Box box, const T *__restrict__ b, VelArr<T> x, CoefU<T> cf,
                                                  T mass, T cvisc, int colour, int remap)
{
    int i, j, k;
    if (!box_colour_pos(box, colour, xcd_block(remap) * blockDim.x + threadIdx.x, i, j, k)) return;
    const long long f = at(g, i, j, k);
    const T bf = b[f], xf = x.c[A][f];
    T Ax, dg;
    u_row<T, D, A>(g, x, cf, mass, cvisc, i, j, k, Ax, dg);
    const T xn = xf + (bf - Ax) / dg;
    x.c[A][f] = xn;
    write_images(g, face_mask(A), ROLE_V, x.c[A], i, j, k, xn);
}

// The same colour passes (3D), z-blocked: a workgroup owns a band of `rows`
// rows of one colour in each plane of a run of ZB_PLANES consecutive planes
// and walks those planes in order, so that the planes a point reads above
// and below were read by the same workgroup one step before (hits in its
// caches) rather than fetched again by other workgroups at other times.  The
// points of one colour are independent, so this order gives the same bits
// as the flat launch.
constexpr int ZB_PLANES = 16;

template <typename T>
__global__ void __launch_bounds__(256) k_smooth_p_zb(Grid g, Box box, const T *__restrict__ b, T *x, CoefP<T> cf,
                                                     T cvisc, int colour, int rows, int nbands)
{
    const int half = (box.ext[0] + 1) >> 1;
    const int j0 = (blockIdx.x % nbands) * rows, kz0 = (blockIdx.x / nbands) * ZB_PLANES;
    const int npts = half * min(rows, box.ext[1] - j0);
    const int kz1 = min(kz0 + ZB_PLANES, box.ext[2]);
    for (int kz = kz0; kz < kz1; ++kz) {
        const int k = box.lo[2] + kz;
        for (int t = threadIdx.x; t < npts; t += blockDim.x) {
            const int j = box.lo[1] + j0 + t / half;
            const int i = box.lo[0] + 2 * (t % half) + ((box.lo[0] + j + k + colour) & 1);
            if (i >= box.lo[0] + box.ext[0]) continue;
            const long long c = at(g, i, j, k);
            const T bc = b[c], xc = x[c];
            T Ax, dg;
            p_row<T, 3>(g, x, cf, cvisc, i, j, k, Ax, dg);
            const T xn = xc + (bc - Ax) / dg;
            x[c] = xn;
            write_images(g, 0, ROLE_P, x, i, j, k, xn);
        }
    }
}

template <typename T, int A>
__global__ void __launch_bounds__(256) k_smooth_u_zb(Grid g, Box box, const T *__restrict__ b, VelArr<T> x, CoefU<T> cf,
                                                     T mass, T cvisc, int colour, int rows, int nbands)
{
    const int half = (box.ext[0] + 1) >> 1;
    const int j0 = (blockIdx.x % nbands) * rows, kz0 = (blockIdx.x / nbands) * ZB_PLANES;
    const int npts = half * min(rows, box.ext[1] - j0);
    const int kz1 = min(kz0 + ZB_PLANES, box.ext[2]);
    for (int kz = kz0; kz < kz1; ++kz) {
        const int k = box.lo[2] + kz;
        for (int t = threadIdx.x; t < npts; t += blockDim.x) {
            const int j = box.lo[1] + j0 + t / half;
            const int i = box.lo[0] + 2 * (t % half) + ((box.lo[0] + j + k + colour) & 1);
            if (i >= box.lo[0] + box.ext[0]) continue;
            const long long f = at(g, i, j, k);
            const T bf = b[f], xf = x.c[A][f];
            T Ax, dg;
            u_row<T, 3, A>(g, x, cf, mass, cvisc, i, j, k, Ax, dg);
            const T xn = xf + (bf - Ax) / dg;
            x.c[A][f] = xn;
            write_images(g, face_mask(A), ROLE_V, x.c[A], i, j, k, xn);
        }
    }
}

// one colour of every component of the constant-viscosity system (eq:NSdis1)
// in one launch: the components do not couple, so this is the sweep of the
// components one after another.  blockIdx.y is the component.
template <typename T, int D>
__global__ void __launch_bounds__(256) k_smooth_u_dec(Grid g, VelBox boxes, VelArrC<T> b, VelArr<T> x, CoefU<T> cf,
                                                      T mass, T cvisc, int colour, int remap)
{
    const int a = blockIdx.y;
    int i, j, k;
    if (!box_colour_pos(boxes.b[a], colour, xcd_block(remap) * blockDim.x + threadIdx.x, i, j, k)) return;
    const long long f = at(g, i, j, k);
    T *xa = x.c[a];
    const T bf = b.c[a][f], xf = xa[f];
    T Ax, dg;
    if (a == 0) u_row_dec<T, D, 0>(g, x.c[0], cf.rho[0], mass, cvisc, i, j, k, Ax, dg);
    else if (a == 1) u_row_dec<T, D, 1>(g, x.c[1], cf.rho[1], mass, cvisc, i, j, k, Ax, dg);
    else u_row_dec<T, D, (D == 3 ? 2 : 1)>(g, x.c[2], cf.rho[2], mass, cvisc, i, j, k, Ax, dg);
    const T xn = xf + (bf - Ax) / dg;
    xa[f] = xn;
    write_images(g, face_mask(a), ROLE_V, xa, i, j, k, xn);
}

// ---------------------------------------------------------------------------
// One full red-black sweep of one component in one launch.  Each workgroup
// owns a tile of the component's unknowns and stages a window of the tile
// plus two points on every side in LDS: the red points of the tile and of
// the ring around it are updated from the old black values, then the black
// points of the tile from those reds.  The red ring is computed again by
// the neighbouring tiles with the same arithmetic.  The result goes to a
// second buffer (x_out), so that no workgroup reads a value another one has
// already updated.  Along periodic axes the window holds the wrapped points
// themselves; along the other axes it holds the ghost images, which a red
// update refreshes inside the window.
// ---------------------------------------------------------------------------
template <typename T, int D>
struct RBTile {
    static constexpr int H = 2;
    static constexpr int TX = D == 3 ? 8 : 16, TY = D == 3 ? 8 : 16, TZ = D == 3 ? (sizeof(T) == 8 ? 4 : 8) : 1;
    static constexpr int WX = TX + 2 * H, WY = TY + 2 * H, WZ = D == 3 ? TZ + 2 * H : 1;
    static constexpr int W = WX * WY * WZ;
};

// write v (times the sign) to the ghost images of (i, j, k) along the
// non-periodic axes that fall inside the window [o, o + W)
template <typename T, int D>
__device__ inline void write_images_window(const Grid &g, int vmask, int role, T *x, int i, int j, int k, T v,
                                           const int o[3], const int w[3])
{
    const int q[3] = {i, j, k};
    AxisImages im[3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
        im[d] = d < D && g.bc[d] != AX_PERIODIC ? images_of(g, d, (vmask >> d) & 1, role, q[d])
                                               : AxisImages{{0, 0}, {0, 0}};
    if ((im[0].s[0] | im[0].s[1] | im[1].s[0] | im[1].s[1] | im[2].s[0] | im[2].s[1]) == 0) return;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (a == 0 && b == 0 && c == 0) continue;
                const int sa = a ? im[0].s[a - 1] : 1;
                const int sb = b ? im[1].s[b - 1] : 1;
                const int sc = c ? im[2].s[c - 1] : 1;
                if (sa == 0 || sb == 0 || sc == 0) continue;
                const int qa = a ? im[0].q[a - 1] : i;
                const int qb = b ? im[1].q[b - 1] : j;
                const int qc = c ? im[2].q[c - 1] : k;
                if (qa < o[0] || qa >= o[0] + w[0] || qb < o[1] || qb >= o[1] + w[1]) continue;
                if (D == 3 && (qc < o[2] || qc >= o[2] + w[2])) continue;
                x[at(g, qa, qb, qc)] = sa * sb * sc > 0 ? v : -v;
            }
}

template <typename T, int D, int VEL, int A>
__global__ void __launch_bounds__(256) k_smooth_rb(Grid g, Box box, VelArrC<T> xin, const T *__restrict__ b,
                                                   CoefU<T> cu, CoefP<T> cp, T mass, T cvisc, T *xout)
{
    using TL = RBTile<T, D>;
    constexpr int NARR = VEL ? 2 * D + 2 : D + 2;
    constexpr int BS = 256;
    __shared__ T w[NARR][TL::W];
    const int vmask = VEL ? face_mask(A) : 0;
    const int role = VEL ? ROLE_V : ROLE_P;
    // this workgroup's tile and window origin (extended lattice coordinates)
    const int ntx = (box.ext[0] + TL::TX - 1) / TL::TX, nty = (box.ext[1] + TL::TY - 1) / TL::TY;
    const int tid = blockIdx.x;
    const int t0 = tid % ntx, t1 = (tid / ntx) % nty, t2 = tid / (ntx * nty);
    const int lo[3] = {box.lo[0] + t0 * TL::TX, box.lo[1] + t1 * TL::TY, D == 3 ? box.lo[2] + t2 * TL::TZ : 0};
    const int o[3] = {lo[0] - TL::H, lo[1] - TL::H, D == 3 ? lo[2] - TL::H : 0};
    const int wd[3] = {TL::WX, TL::WY, TL::WZ};
    // the window as a grid: same axes and boundary kinds, window strides
    Grid gw = g;
    gw.NX = TL::WX;
    gw.NY = TL::WY;
    gw.NXY = (long long)TL::WX * TL::WY;
    const long long shift = at(gw, o[0], o[1], o[2]);
    // source arrays of the window, in the order of w
    const T *src[NARR];
    if (VEL) {
        src[0] = xin.c[A];
#pragma unroll
        for (int bi = 0; bi < D - 1; ++bi) {
            const int B = other_axis<A>(bi);
            src[1 + bi] = xin.c[B];
            src[D + 3 + bi] = cu.mue[3 - A - B];
        }
        src[D] = b;
        src[D + 1] = cu.rho[A];
        src[D + 2] = cu.muc;
    } else {
        src[0] = xin.c[0];
        src[1] = b;
#pragma unroll
        for (int a = 0; a < D; ++a) src[2 + a] = cp.beta[a];
    }
    // stage the window: every load issued before the first store
    constexpr int PER = (TL::W + BS - 1) / BS;
    int eidx[PER];
#pragma unroll
    for (int it = 0; it < PER; ++it) {
        const int sidx = threadIdx.x + it * BS;
        int q[3] = {o[0] + sidx % TL::WX, o[1] + (sidx / TL::WX) % TL::WY, D == 3 ? o[2] + sidx / (TL::WX * TL::WY) : 0};
        bool ok = sidx < TL::W;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            if (g.bc[d] == AX_PERIODIC) {
                if (q[d] < 0) q[d] += g.n[d];
                while (q[d] >= g.n[d]) q[d] -= g.n[d];
            } else if (q[d] < -1 || q[d] > g.n[d] + 1) {
                ok = false;
            }
        }
        eidx[it] = ok ? (int)at(g, q[0], q[1], q[2]) : -1;
    }
    T v[NARR][PER];
#pragma unroll
    for (int m = 0; m < NARR; ++m)
#pragma unroll
        for (int it = 0; it < PER; ++it) {
            const T x = src[m][eidx[it] >= 0 ? eidx[it] : 0];
            v[m][it] = eidx[it] >= 0 ? x : T(0);
        }
#pragma unroll
    for (int m = 0; m < NARR; ++m)
#pragma unroll
        for (int it = 0; it < PER; ++it) {
            const int sidx = threadIdx.x + it * BS;
            if (sidx < TL::W) w[m][sidx] = v[m][it];
        }
    __syncthreads();
    // window views shifted so that at(gw, i, j, k) indexes them
    VelArr<T> xw{{nullptr, nullptr, nullptr}};
    CoefU<T> cw = cu;
    CoefP<T> pw = cp;
    T *bw;
    if (VEL) {
        xw.c[A] = &w[0][0] - shift;
#pragma unroll
        for (int bi = 0; bi < D - 1; ++bi) {
            const int B = other_axis<A>(bi);
            xw.c[B] = &w[1 + bi][0] - shift;
            cw.mue[3 - A - B] = &w[D + 3 + bi][0] - shift;
        }
        bw = &w[D][0] - shift;
        cw.rho[A] = &w[D + 1][0] - shift;
        cw.muc = &w[D + 2][0] - shift;
    } else {
        xw.c[0] = &w[0][0] - shift;
        bw = &w[1][0] - shift;
#pragma unroll
        for (int a = 0; a < D; ++a) pw.beta[a] = &w[2 + a][0] - shift;
    }
    T *xa = xw.c[VEL ? A : 0];
    int ulo[3], uhi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) unk_range(g, d, (vmask >> d) & 1, ulo[d], uhi[d]);
    // red: the tile and the ring around it, enumerated by colour
    constexpr int RX = TL::TX + 2, RY = TL::TY + 2, RZ = D == 3 ? TL::TZ + 2 : 1, RH = RX / 2;
    for (int t = threadIdx.x; t < RH * RY * RZ; t += BS) {
        const int ih = t % RH, r = t / RH;
        const int q1 = lo[1] - 1 + r % RY, q2 = D == 3 ? lo[2] - 1 + r / RY : 0;
        const int q0 = lo[0] - 1 + 2 * ih + ((lo[0] - 1 + q1 + q2) & 1);
        const int qq[3] = {q0, q1, q2};
        bool unknown = true;
#pragma unroll
        for (int d = 0; d < D; ++d)
            if (g.bc[d] != AX_PERIODIC && (qq[d] < ulo[d] || qq[d] > uhi[d])) unknown = false;
        if (!unknown) continue;
        T Ax, dg;
        if (VEL) u_row<T, D, A>(gw, xw, cw, mass, cvisc, q0, q1, q2, Ax, dg);
        else p_row<T, D>(gw, xa, pw, cvisc, q0, q1, q2, Ax, dg);
        const long long f = at(gw, q0, q1, q2);
        const T xn = xa[f] + (bw[f] - Ax) / dg;
        xa[f] = xn;
        write_images_window<T, D>(gw, vmask, role, xa, q0, q1, q2, xn, o, wd);
    }
    __syncthreads();
    // black: the tile, enumerated by colour
    constexpr int TH = TL::TX / 2;
    for (int t = threadIdx.x; t < TH * TL::TY * TL::TZ; t += BS) {
        const int ih = t % TH, r = t / TH;
        const int q1 = lo[1] + r % TL::TY, q2 = D == 3 ? lo[2] + r / TL::TY : 0;
        const int q0 = lo[0] + 2 * ih + ((lo[0] + q1 + q2 + 1) & 1);
        if (q0 >= box.lo[0] + box.ext[0] || q1 >= box.lo[1] + box.ext[1]) continue;
        if (D == 3 && q2 >= box.lo[2] + box.ext[2]) continue;
        T Ax, dg;
        if (VEL) u_row<T, D, A>(gw, xw, cw, mass, cvisc, q0, q1, q2, Ax, dg);
        else p_row<T, D>(gw, xa, pw, cvisc, q0, q1, q2, Ax, dg);
        const long long f = at(gw, q0, q1, q2);
        xa[f] = xa[f] + (bw[f] - Ax) / dg;
    }
    __syncthreads();
    // the tile's unknowns and their ghost images to the output buffer
    constexpr int TT = TL::TX * TL::TY * TL::TZ;
    for (int sidx = threadIdx.x; sidx < TT; sidx += BS) {
        const int q0 = lo[0] + sidx % TL::TX, q1 = lo[1] + (sidx / TL::TX) % TL::TY;
        const int q2 = D == 3 ? lo[2] + sidx / (TL::TX * TL::TY) : 0;
        if (q0 >= box.lo[0] + box.ext[0] || q1 >= box.lo[1] + box.ext[1]) continue;
        if (D == 3 && q2 >= box.lo[2] + box.ext[2]) continue;
        const T val = xa[at(gw, q0, q1, q2)];
        xout[at(g, q0, q1, q2)] = val;
        write_images(g, vmask, role, xout, q0, q1, q2, val);
    }
}

// ---------------------------------------------------------------------------
// One launch per red-black sweep of a velocity component (3D), marching
// along z.  A workgroup owns a tile of ZM_TX x ZM_TY points in each plane of
// a run [z0, z1) of planes and holds u_a of ZM_NS consecutive planes, the
// tile widened by ZM_H points on every side, in LDS.  Stepping p = z0 ..
// z1 - 1, it loads plane p + 3, updates the red points of plane p + 1 (the
// tile and a ring of one point around it), then the black points of plane p
// (the tile).  Ring points, and the red planes z0 - 1 and z1, belong to other
// workgroups: they are updated again here, from the same values with the
// same arithmetic, so that the black points at the tile's edge see the red
// values of after the pass.  Every red point thus reads the black values of
// before the sweep and every black point the red values of after it: the
// bits of the two colour passes.  The other fields are read from global
// memory, each point's once per sweep, so the sweep streams every array
// about once instead of once per colour.  Results go to a second buffer,
// since the window's halo must see values from before the sweep.
//
// Window planes: red at p + 1 reads p .. p + 2 and writes ghost images up to
// two planes away (the one past the outflow face); black at p reads
// p - 1 .. p + 1.  Six slots let the load of plane p + 4 overwrite p - 2
// while black p may still be reading p - 1, so a step needs two barriers.
// (Running red p + 1 and black p - 1 in one phase, one barrier a step, was
// slower.)
// ---------------------------------------------------------------------------
constexpr int ZM_TX = 64, ZM_TY = 8, ZM_H = 2, ZM_WX = ZM_TX + 2 * ZM_H, ZM_WY = ZM_TY + 2 * ZM_H;
constexpr int ZM_PS = ZM_WX * ZM_WY, ZM_NS = 6, ZM_BS = 256;

// u_a at a point of the window and along its axes: in-plane neighbours in the
// point's plane, z neighbours in the planes below and above
template <typename T>
struct UaWin {
    const T *w;
    int c;       // position in the plane
    int pl[3];   // offsets of the planes z - 1, z, z + 1
    __device__ T here() const { return w[pl[1] + c]; }
    __device__ T nb(int ax, int s) const
    {
        return ax == 2 ? w[pl[1 + s] + c] : w[pl[1] + c + (ax == 0 ? s : s * ZM_WX)];
    }
};

__device__ inline int zm_slot(int z) { return (((z % ZM_NS) + ZM_NS) % ZM_NS) * ZM_PS; }

template <typename T, int A>
__global__ void __launch_bounds__(ZM_BS) k_smooth_zm(Grid g, Box box, VelArrC<T> xin, const T *__restrict__ b,
                                                      CoefU<T> cf, T mass, T cvisc, T *xout, int cz, int remap)
{
    __shared__ T w[ZM_NS * ZM_PS];
    constexpr int vmask = 1 << A;
    const int ntx = (box.ext[0] + ZM_TX - 1) / ZM_TX, nty = (box.ext[1] + ZM_TY - 1) / ZM_TY;
    const int tid = (int)xcd_block(remap);
    const int t0 = tid % ntx, t1 = (tid / ntx) % nty, ch = tid / (ntx * nty);
    const int lo0 = box.lo[0] + t0 * ZM_TX, lo1 = box.lo[1] + t1 * ZM_TY;
    const int hx = min(lo0 + ZM_TX, box.lo[0] + box.ext[0]), hy = min(lo1 + ZM_TY, box.lo[1] + box.ext[1]);
    const int z0 = box.lo[2] + ch * cz, z1 = min(z0 + cz, box.lo[2] + box.ext[2]);
    const int o0 = lo0 - ZM_H, o1 = lo1 - ZM_H;
    int ulo[3], uhi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) unk_range(g, d, (vmask >> d) & 1, ulo[d], uhi[d]);
    const bool per[3] = {g.bc[0] == AX_PERIODIC, g.bc[1] == AX_PERIODIC, g.bc[2] == AX_PERIODIC};
    // a lattice coordinate along a periodic axis, brought into [0, n)
    auto wrap = [&](int d, int q) { return !per[d] ? q : (q < 0 ? q + g.n[d] : (q >= g.n[d] ? q - g.n[d] : q)); };
    // positions stored along a non-periodic axis: -1 .. n + 1
    auto stored = [&](int d, int q) { return per[d] || (q >= -1 && q <= g.n[d] + 1); };
    const T *__restrict__ xa = xin.c[A];

    auto load_plane = [&](int z) {
        T *dst = w + zm_slot(z);
        const int rz = wrap(2, z);
        const bool zok = stored(2, z);
        constexpr int PER = (ZM_PS + ZM_BS - 1) / ZM_BS;
        T v[PER];
#pragma unroll
        for (int it = 0; it < PER; ++it) {
            const int sidx = threadIdx.x + it * ZM_BS;
            const int qx = o0 + sidx % ZM_WX, qy = o1 + sidx / ZM_WX;
            const bool ok = sidx < ZM_PS && zok && stored(0, qx) && stored(1, qy);
            v[it] = ok ? xa[at(g, wrap(0, qx), wrap(1, qy), rz)] : T(0);
        }
#pragma unroll
        for (int it = 0; it < PER; ++it) {
            const int sidx = threadIdx.x + it * ZM_BS;
            if (sidx < ZM_PS) dst[sidx] = v[it];
        }
    };

    // the ghost images (non-periodic axes) of window point (x, y, z) that
    // fall inside the window's planes zl .. zh
    auto win_images = [&](int x, int y, int z, T v, int zl, int zh) {
        const int q[3] = {x, y, z};
        AxisImages im[3];
#pragma unroll
        for (int d = 0; d < 3; ++d)
            im[d] = per[d] ? AxisImages{{0, 0}, {0, 0}} : images_of(g, d, (vmask >> d) & 1, ROLE_V, q[d]);
        if ((im[0].s[0] | im[0].s[1] | im[1].s[0] | im[1].s[1] | im[2].s[0] | im[2].s[1]) == 0) return;
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
#pragma unroll
            for (int bb = 0; bb < 3; ++bb)
#pragma unroll
                for (int aa = 0; aa < 3; ++aa) {
                    if (aa == 0 && bb == 0 && cc == 0) continue;
                    const int sa = aa ? im[0].s[aa - 1] : 1;
                    const int sb = bb ? im[1].s[bb - 1] : 1;
                    const int sc = cc ? im[2].s[cc - 1] : 1;
                    if (sa == 0 || sb == 0 || sc == 0) continue;
                    const int qa = aa ? im[0].q[aa - 1] : x;
                    const int qb = bb ? im[1].q[bb - 1] : y;
                    const int qc = cc ? im[2].q[cc - 1] : z;
                    if (qa < o0 || qa >= o0 + ZM_WX || qb < o1 || qb >= o1 + ZM_WY || qc < zl || qc > zh) continue;
                    w[zm_slot(qc) + (qb - o1) * ZM_WX + (qa - o0)] = sa * sb * sc > 0 ? v : -v;
                }
    };

    constexpr int RH = (ZM_TX + 2) / 2, RY = ZM_TY + 2, NRED = RH * RY;
    constexpr int BH = ZM_TX / 2, NBLACK = BH * ZM_TY;

    // the t-th red point of plane z in the tile and its ring; zl .. zh:
    // planes held
    auto red_point = [&](int z, int t, int zl, int zh) {
        const int ih = t % RH, r = t / RH;
        const int y = lo1 - 1 + r;
        const int x = lo0 - 1 + 2 * ih + ((lo0 - 1 + y + z) & 1);
        if (x > hx || y > hy) return;
        if (!per[0] && (x < ulo[0] || x > uhi[0])) return;
        if (!per[1] && (y < ulo[1] || y > uhi[1])) return;
        const int rx = wrap(0, x), ry = wrap(1, y), rz = wrap(2, z);
        const int f = (int)at(g, rx, ry, rz);
        const UaWin<T> ua{w, (y - o1) * ZM_WX + (x - o0), {zm_slot(z - 1), zm_slot(z), zm_slot(z + 1)}};
        const T rho = cf.rho[A][f];
        const T bf = b[f], xe = ua.here();
        T Ax, dg;
        u_row_core<T, 3, A>(g, ua, xin, cf, rho, mass, cvisc, f, rx, ry, rz, Ax, dg);
        const T xn = xe + (bf - Ax) / dg;
        w[ua.pl[1] + ua.c] = xn;
        win_images(x, y, z, xn, zl, zh);
        if (z >= z0 && z < z1 && x >= lo0 && x < hx && y >= lo1 && y < hy) {
            xout[f] = xn;
            write_images(g, vmask, ROLE_V, xout, x, y, z, xn);
        }
    };
    auto red_unknown_plane = [&](int z) { return per[2] || (z >= ulo[2] && z <= uhi[2]); };

    // the t-th black point of plane z (in [z0, z1)) in the tile
    auto black_point = [&](int z, int t) {
        const int ih = t % BH, r = t / BH;
        const int y = lo1 + r;
        const int x = lo0 + 2 * ih + ((lo0 + y + z + 1) & 1);
        if (x >= hx || y >= hy) return;
        const int f = (int)at(g, x, y, z);
        const UaWin<T> ua{w, (y - o1) * ZM_WX + (x - o0), {zm_slot(z - 1), zm_slot(z), zm_slot(z + 1)}};
        const T rho = cf.rho[A][f];
        const T bf = b[f], xe = ua.here();
        T Ax, dg;
        u_row_core<T, 3, A>(g, ua, xin, cf, rho, mass, cvisc, f, x, y, z, Ax, dg);
        const T xn = xe + (bf - Ax) / dg;
        xout[f] = xn;
        write_images(g, vmask, ROLE_V, xout, x, y, z, xn);
    };

    for (int z = z0 - 2; z <= z0 + 2; ++z) load_plane(z);
    __syncthreads();
    for (int t = threadIdx.x; t < 2 * NRED; t += ZM_BS) {
        const int z = t < NRED ? z0 - 1 : z0;
        if (red_unknown_plane(z)) red_point(z, t < NRED ? t : t - NRED, z0 - 2, z0 + 2);
    }
    __syncthreads();
    for (int p = z0; p < z1; ++p) {
        load_plane(p + 3);
        __syncthreads();
        if (red_unknown_plane(p + 1))
            for (int t = threadIdx.x; t < NRED; t += ZM_BS) red_point(p + 1, t, p, p + 3);
        __syncthreads();
        for (int t = threadIdx.x; t < NBLACK; t += ZM_BS) black_point(p, t);
    }
}


// ---------------------------------------------------------------------------
// block reduction of one double per thread into partial[slot] (fixed order)
// ---------------------------------------------------------------------------
__device__ inline void block_sum_store(double v, double *partial, long long slot)
{
    __shared__ double red[256];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[slot] = red[0];
}

// residual r = b - A x at every unknown (r may be null) and per-block
// partial sums of r^2 (partial may be null); grid-stride over the box
template <typename T, int D>
__global__ void __launch_bounds__(256) k_resid_p(Grid g, Box box, const T *__restrict__ b, const T *__restrict__ x,
                                                 CoefP<T> cf, T cvisc, T *r, double *partial)
{
    const int n = box.ext[0] * box.ext[1] * box.ext[2];
    double acc = 0.0;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        int i, j, k;
        box_pos(box, t, i, j, k);
        const long long c = at(g, i, j, k);
        const T bc = b[c];
        T Ax, dg;
        p_row<T, D>(g, x, cf, cvisc, i, j, k, Ax, dg);
        const T rv = bc - Ax;
        if (r) r[c] = rv;
        acc += (double)rv * (double)rv;
    }
    if (partial) block_sum_store(acc, partial, blockIdx.x);
}

template <typename T, int D>
__global__ void __launch_bounds__(256) k_resid_u(Grid g, VelBox boxes, VelArrC<T> b, VelArr<T> x, CoefU<T> cf, T mass,
                                                 T cvisc, VelArr<T> r, double *partial)
{
    const int a = blockIdx.y;
    const Box box = boxes.b[a];
    const int n = box.ext[0] * box.ext[1] * box.ext[2];
    double acc = 0.0;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        int i, j, k;
        box_pos(box, t, i, j, k);
        const long long f = at(g, i, j, k);
        const T bf = b.c[a][f];
        T Ax, dg;
        if (a == 0) u_row<T, D, 0>(g, x, cf, mass, cvisc, i, j, k, Ax, dg);
        else if (a == 1) u_row<T, D, 1>(g, x, cf, mass, cvisc, i, j, k, Ax, dg);
        else u_row<T, D, (D == 3 ? 2 : 1)>(g, x, cf, mass, cvisc, i, j, k, Ax, dg);
        const T rv = bf - Ax;
        if (r.c[a]) r.c[a][f] = rv;
        acc += (double)rv * (double)rv;
    }
    if (partial) block_sum_store(acc, partial, (long long)blockIdx.y * gridDim.x + blockIdx.x);
}

// sum of squares of a field over the unknowns of one or more lattices
template <typename T>
__global__ void __launch_bounds__(256) k_norm2(VelBox boxes, Grid g, VelArrC<T> v, double *partial)
{
    const int a = blockIdx.y;
    const Box box = boxes.b[a];
    const int n = box.ext[0] * box.ext[1] * box.ext[2];
    double acc = 0.0;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        int i, j, k;
        box_pos(box, t, i, j, k);
        const double w = (double)v.c[a][at(g, i, j, k)];
        acc += w * w;
    }
    block_sum_store(acc, partial, (long long)blockIdx.y * gridDim.x + blockIdx.x);
}

// one block: out[0] = sum of partial[0..n) in a fixed order
__global__ void __launch_bounds__(256) k_reduce_final(const double *__restrict__ partial, long long n, double *out)
{
    double acc = 0.0;
    for (long long t = threadIdx.x; t < n; t += blockDim.x) acc += partial[t];
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// ---------------------------------------------------------------------------
// transfers
// ---------------------------------------------------------------------------
// Per-axis taps of a transfer, resolved through the boundary rules once per
// axis: index along the axis, sign, and weight (zero for a fixed face).
struct AxisTaps {
    int q[4];
    double w[4];
};

template <int NT>
__device__ inline void resolve_taps(const Grid &g, int d, int vert, int role, const int *raw, const double *wraw,
                                    AxisTaps &t)
{
#pragma unroll
    for (int a = 0; a < NT; ++a) {
        int q = raw[a], s = 1;
        const bool live = resolve(g, d, vert, role, q, s);
        t.q[a] = live ? q : 0;
        t.w[a] = live ? (s > 0 ? wraw[a] : -wraw[a]) : 0.0;
    }
}

template <typename T, int D, int VM>
__device__ inline double restrict_point(const Grid &gf, int role, const T *__restrict__ src, int I, int J, int K)
{
    constexpr int N0 = (VM & 1) ? 3 : 4;
    constexpr int N1 = (VM & 2) ? 3 : 4;
    constexpr int N2 = D == 3 ? ((VM & 4) ? 3 : 4) : 1;
    const int Q[3] = {I, J, K};
    AxisTaps t[3];
    int raw[4];
    double wr[4];
    rst_weights(VM & 1, Q[0], raw, wr);
    resolve_taps<N0>(gf, 0, VM & 1, role, raw, wr, t[0]);
    rst_weights((VM >> 1) & 1, Q[1], raw, wr);
    resolve_taps<N1>(gf, 1, (VM >> 1) & 1, role, raw, wr, t[1]);
    if (D == 3) {
        rst_weights((VM >> 2) & 1, Q[2], raw, wr);
        resolve_taps<N2>(gf, 2, (VM >> 2) & 1, role, raw, wr, t[2]);
    } else {
        t[2].q[0] = 0;
        t[2].w[0] = 1.0;
    }
    T v[N2][N1][N0];
#pragma unroll
    for (int c = 0; c < N2; ++c)
#pragma unroll
        for (int b = 0; b < N1; ++b)
#pragma unroll
            for (int a = 0; a < N0; ++a) v[c][b][a] = src[at(gf, t[0].q[a], t[1].q[b], t[2].q[c])];
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < N2; ++c)
#pragma unroll
        for (int b = 0; b < N1; ++b) {
            double rs = 0.0;
#pragma unroll
            for (int a = 0; a < N0; ++a) rs += t[0].w[a] * (double)v[c][b][a];
            s += t[1].w[b] * t[2].w[c] * rs;
        }
    return s;
}

template <typename T, int D, int VM>
__device__ inline double prolong_point(const Grid &gc, int role, const T *__restrict__ src, int i, int j, int k)
{
    constexpr int N2 = D == 3 ? 2 : 1;
    const int q[3] = {i, j, k};
    AxisTaps t[3];
    int raw[2];
    double wr[2];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const int vert = (VM >> d) & 1;
        const int n = prl_weights(vert, q[d], raw, wr);
        if (n == 1) { raw[1] = raw[0]; wr[1] = 0.0; }
        resolve_taps<2>(gc, d, vert, role, raw, wr, t[d]);
    }
    if (D == 2) {
        t[2].q[0] = 0;
        t[2].w[0] = 1.0;
    }
    T v[N2][2][2];
#pragma unroll
    for (int c = 0; c < N2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) v[c][b][a] = src[at(gc, t[0].q[a], t[1].q[b], t[2].q[c])];
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < N2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) s += t[0].w[a] * t[1].w[b] * t[2].w[c] * (double)v[c][b][a];
    return s;
}

template <typename T, int D>
__device__ inline double restrict_any(int vm, const Grid &gf, int role, const T *src, int I, int J, int K)
{
    switch (vm) {
    case 0: return restrict_point<T, D, 0>(gf, role, src, I, J, K);
    case 1: return restrict_point<T, D, 1>(gf, role, src, I, J, K);
    case 2: return restrict_point<T, D, 2>(gf, role, src, I, J, K);
    case 3: return restrict_point<T, D, 3>(gf, role, src, I, J, K);
    case 4: return restrict_point<T, D, 4>(gf, role, src, I, J, K);
    case 5: return restrict_point<T, D, 5>(gf, role, src, I, J, K);
    case 6: return restrict_point<T, D, 6>(gf, role, src, I, J, K);
    default: return restrict_point<T, D, 7>(gf, role, src, I, J, K);
    }
}

template <typename T, int D>
__device__ inline double prolong_any(int vm, const Grid &gc, int role, const T *src, int i, int j, int k)
{
    switch (vm) {
    case 0: return prolong_point<T, D, 0>(gc, role, src, i, j, k);
    case 1: return prolong_point<T, D, 1>(gc, role, src, i, j, k);
    case 2: return prolong_point<T, D, 2>(gc, role, src, i, j, k);
    case 3: return prolong_point<T, D, 3>(gc, role, src, i, j, k);
    case 4: return prolong_point<T, D, 4>(gc, role, src, i, j, k);
    case 5: return prolong_point<T, D, 5>(gc, role, src, i, j, k);
    case 6: return prolong_point<T, D, 6>(gc, role, src, i, j, k);
    default: return prolong_point<T, D, 7>(gc, role, src, i, j, k);
    }
}

// coarse[c] = full-weighting restriction of fine[c] at every coarse unknown
// (or every stored coarse position for coefficients); zero_x[c], when set,
// is cleared at the same positions (the coarse correction starts at zero)
template <typename T, int D>
__global__ void __launch_bounds__(256) k_restrict(Grid gf, Grid gc, VelBox boxes, int masks, int role,
                                                  VelArrC<T> fine, VelArr<T> coarse, T scale, VelArr<T> zero_x)
{
    const int comp = blockIdx.y;
    const int vmask = (masks >> (4 * comp)) & 0xF;
    int I, J, K;
    if (!box_pos(boxes.b[comp], blockIdx.x * blockDim.x + threadIdx.x, I, J, K)) return;
    const double s = restrict_any<T, D>(vmask, gf, role, fine.c[comp], I, J, K);
    const long long e = at(gc, I, J, K);
    coarse.c[comp][e] = (T)(s * (double)scale);
    if (zero_x.c[comp]) {
        zero_x.c[comp][e] = T(0);
        write_images(gc, vmask, role, zero_x.c[comp], I, J, K, T(0));
    }
}

// fine[c] += linear interpolation of coarse[c] at every fine unknown
template <typename T, int D>
__global__ void __launch_bounds__(256) k_prolong_add(Grid gc, Grid gf, VelBox boxes, int masks, int role,
                                                     VelArrC<T> coarse, VelArr<T> fine)
{
    const int comp = blockIdx.y;
    const int vmask = (masks >> (4 * comp)) & 0xF;
    int i, j, k;
    if (!box_pos(boxes.b[comp], blockIdx.x * blockDim.x + threadIdx.x, i, j, k)) return;
    const long long e = at(gf, i, j, k);
    const T xe = fine.c[comp][e];
    const T v = xe + (T)prolong_any<T, D>(vmask, gc, role, coarse.c[comp], i, j, k);
    fine.c[comp][e] = v;
    write_images(gf, vmask, role, fine.c[comp], i, j, k, v);
}

// ---------------------------------------------------------------------------
// coarsest level: dense inverse, assembled by applying the stencil to unit
// vectors, inverted by Gauss-Jordan with partial pivoting (one workgroup)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_dense_assemble(Grid g, int velocity, int n, const long long *__restrict__ uidx,
                                                        const int *__restrict__ ucomp, CoefP<double> cp,
                                                        CoefU<double> cu, double mass, double cvisc, double *tmp,
                                                        double *Aw)
{
    // block j: column j of A (row-major n x n) = A applied to the unit vector e_j
    const int j = blockIdx.x;
    const int nc = velocity ? g.D : 1;
    const long long nel = g.nel;
    double *base = tmp + (long long)j * nc * nel;
    VelArr<double> x{{base, nc > 1 ? base + nel : nullptr, nc > 2 ? base + 2 * nel : nullptr}};
    for (long long e = threadIdx.x; e < nc * nel; e += blockDim.x) base[e] = 0.0;
    __syncthreads();
    if (threadIdx.x == 0) x.c[velocity ? ucomp[j] : 0][uidx[j]] = 1.0;
    __syncthreads();
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
        int i, jj, k;
        decode(g, uidx[r], i, jj, k);
        double Ax, dg;
        if (velocity) u_row_slow_any<double>(g, x, cu, mass, cvisc, ucomp[r], i, jj, k, Ax, dg);
        else p_row_slow_any<double>(g, x.c[0], cp, cvisc, i, jj, k, Ax, dg);
        Aw[r * n + j] = Ax;
    }
}

// Gauss-Jordan with partial pivoting on [A | I] held in LDS, one workgroup;
// singular (all-Neumann/periodic pressure): A + alpha 1 1^T, alpha = trace / n^2
__global__ void __launch_bounds__(1024) k_dense_gj(int n, int singular, const double *__restrict__ Aw, double *M)
{
    __shared__ double A[DENSE_LDS][DENSE_LDS + 1], B[DENSE_LDS][DENSE_LDS + 1];
    __shared__ double f[DENSE_LDS];
    __shared__ double tr;
    __shared__ int piv;
    const int t = threadIdx.x;
    for (int e = t; e < n * n; e += blockDim.x) {
        const int r = e / n, c = e % n;
        A[r][c] = Aw[e];
        B[r][c] = r == c ? 1.0 : 0.0;
    }
    __syncthreads();
    if (singular) {
        if (t == 0) {
            double s = 0.0;
            for (int i = 0; i < n; ++i) s += A[i][i];
            tr = s / ((double)n * (double)n);
        }
        __syncthreads();
        for (int e = t; e < n * n; e += blockDim.x) A[e / n][e % n] += tr;
        __syncthreads();
    }
    for (int k = 0; k < n; ++k) {
        if (t == 0) {
            int p = k;
            for (int i = k + 1; i < n; ++i)
                if (fabs(A[i][k]) > fabs(A[p][k])) p = i;
            piv = p;
        }
        __syncthreads();
        const int p = piv;
        if (p != k && t < n) {
            double v = A[k][t]; A[k][t] = A[p][t]; A[p][t] = v;
            v = B[k][t]; B[k][t] = B[p][t]; B[p][t] = v;
        }
        __syncthreads();
        const double pv = A[k][k];
        __syncthreads();
        if (t < n) {
            A[k][t] /= pv;
            B[k][t] /= pv;
        }
        __syncthreads();
        if (t < n) f[t] = A[t][k];
        __syncthreads();
        for (int e = t; e < n * n; e += blockDim.x) {
            const int r = e / n, c = e % n;
            if (r == k) continue;
            A[r][c] -= f[r] * A[k][c];
            B[r][c] -= f[r] * B[k][c];
        }
        __syncthreads();
    }
    for (int e = t; e < n * n; e += blockDim.x) M[e] = B[e / n][e % n];
}

// x = M b over the coarsest unknowns (M in FP64), ghost images updated
template <typename T>
__global__ void __launch_bounds__(64) k_dense_apply(Grid g, int velocity, int n, const long long *__restrict__ uidx,
                                                    const int *__restrict__ ucomp, const double *__restrict__ M,
                                                    VelArrC<T> b, VelArr<T> x)
{
    __shared__ double bv[64];
    const int r = threadIdx.x;
    if (r < n) bv[r] = (double)b.c[ucomp[r]][uidx[r]];
    __syncthreads();
    if (r < n) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += M[r * n + j] * bv[j];
        const int c = ucomp[r];
        x.c[c][uidx[r]] = (T)s;
        int i, jj, k;
        decode(g, uidx[r], i, jj, k);
        write_images(g, velocity ? face_mask(c) : 0, velocity ? ROLE_V : ROLE_P, x.c[c], i, jj, k, (T)s);
    }
}

// ---------------------------------------------------------------------------
// element-wise helpers
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_fill(T *p, long long n, T v)
{
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x)
        p[t] = v;
}

// dst(unknowns) = (Td) src(unknowns)
template <typename Ts, typename Td>
__global__ void __launch_bounds__(256) k_cast_unknowns(Grid g, VelBox boxes, VelArrC<Ts> src, VelArr<Td> dst)
{
    const int a = blockIdx.y;
    int i, j, k;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (!box_pos(boxes.b[a], t, i, j, k)) return;
    const long long e = at(g, i, j, k);
    dst.c[a][e] = (Td)src.c[a][e];
}

// Start of the FP32 inner cycles of a refined iteration, one launch for
// what a cast and a clear per component would do: b32 = (float) r64 at the
// unknowns of each component and x32 = 0 over the whole array (ghosts and
// fixed faces included).  One thread per array entry.
__global__ void __launch_bounds__(256) k_inner_start(Grid g, VelBox boxes, VelArrC<double> r, VelArr<float> b32,
                                                     VelArr<float> x32)
{
    const int a = blockIdx.y;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= g.nel) return;
    x32.c[a][e] = 0.0f;
    int i, j, k;
    decode(g, e, i, j, k);
    const Box &b = boxes.b[a];
    if (i >= b.lo[0] && i < b.lo[0] + b.ext[0] && j >= b.lo[1] && j < b.lo[1] + b.ext[1] && k >= b.lo[2] &&
        k < b.lo[2] + b.ext[2])
        b32.c[a][e] = (float)r.c[a][e];
}

// x(unknowns) += (double) e(unknowns), ghost images of x updated (role:
// velocity components or pressure)
__global__ void __launch_bounds__(256) k_add_correction(Grid g, VelBox boxes, int velocity, VelArrC<float> e,
                                                        VelArr<double> x)
{
    const int a = blockIdx.y;
    int i, j, k;
    if (!box_pos(boxes.b[a], blockIdx.x * blockDim.x + threadIdx.x, i, j, k)) return;
    const long long q = at(g, i, j, k);
    const double v = x.c[a][q] + (double)e.c[a][q];
    x.c[a][q] = v;
    write_images(g, velocity ? face_mask(a) : 0, velocity ? ROLE_V : ROLE_P, x.c[a], i, j, k, v);
}

// dst(unknowns) = src(unknowns) with the ghost images of dst written; fixed
// positions of dst are left as they are (zero in solver arrays)
template <typename T>
__global__ void __launch_bounds__(256) k_load_unknowns(Grid g, VelBox boxes, int velocity, VelArrC<T> src, VelArr<T> dst)
{
    const int a = blockIdx.y;
    int i, j, k;
    if (!box_pos(boxes.b[a], blockIdx.x * blockDim.x + threadIdx.x, i, j, k)) return;
    const long long q = at(g, i, j, k);
    const T v = src.c[a] ? src.c[a][q] : T(0);
    dst.c[a][q] = v;
    write_images(g, velocity ? face_mask(a) : 0, velocity ? ROLE_V : ROLE_P, dst.c[a], i, j, k, v);
}

// coefficient ghost layer: every stored position writes its even images
template <typename T>
__global__ void __launch_bounds__(256) k_coef_ghosts(Grid g, CoefSet<T> set)
{
    const int q = blockIdx.y;
    const int vmask = set.vmask[q];
    T *v = set.v[q];
    Box box{{0, 0, 0}, {1, 1, 1}};
    for (int d = 0; d < 3; ++d) box.ext[d] = stored_extent(g, d, (vmask >> d) & 1);
    int i, j, k;
    if (!box_pos(box, blockIdx.x * blockDim.x + threadIdx.x, i, j, k)) return;
    write_images(g, vmask, ROLE_C, v, i, j, k, v[at(g, i, j, k)]);
}

// ---------------------------------------------------------------------------
// V-cycle-preconditioned GCR on the finest level (FP64): operator apply,
// inner products over the unknowns, and the two updates.  The scalar
// coefficients stay on the device; every thread forms the same quotient.
// ---------------------------------------------------------------------------
template <int D>
__global__ void __launch_bounds__(256) k_apply_u(Grid g, VelBox boxes, VelArr<double> z, CoefU<double> cf,
                                                 double mass, double cvisc, VelArr<double> q)
{
    const int a = blockIdx.y;
    int i, j, k;
    if (!box_pos(boxes.b[a], blockIdx.x * blockDim.x + threadIdx.x, i, j, k)) return;
    double Ax, dg;
    if (a == 0) u_row<double, D, 0>(g, z, cf, mass, cvisc, i, j, k, Ax, dg);
    else if (a == 1) u_row<double, D, 1>(g, z, cf, mass, cvisc, i, j, k, Ax, dg);
    else u_row<double, D, (D == 3 ? 2 : 1)>(g, z, cf, mass, cvisc, i, j, k, Ax, dg);
    q.c[a][at(g, i, j, k)] = Ax;
}

template <int D>
__global__ void __launch_bounds__(256) k_apply_p(Grid g, Box box, const double *z, CoefP<double> cf, double cvisc,
                                                 double *q)
{
    int i, j, k;
    if (!box_pos(box, blockIdx.x * blockDim.x + threadIdx.x, i, j, k)) return;
    double Ax, dg;
    p_row<double, D>(g, z, cf, cvisc, i, j, k, Ax, dg);
    q[at(g, i, j, k)] = Ax;
}

// per-block sums of x . y over the unknowns of every component (blockIdx.y)
__global__ void __launch_bounds__(256) k_dot(VelBox boxes, Grid g, VelArrC<double> x, VelArrC<double> y,
                                             double *partial)
{
    const int a = blockIdx.y;
    const Box box = boxes.b[a];
    const int n = box.ext[0] * box.ext[1] * box.ext[2];
    double acc = 0.0;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        int i, j, k;
        box_pos(box, t, i, j, k);
        const long long e = at(g, i, j, k);
        acc += x.c[a][e] * y.c[a][e];
    }
    block_sum_store(acc, partial, (long long)blockIdx.y * gridDim.x + blockIdx.x);
}

// q -= s qi and z -= s zi at the unknowns, s = num / den
__global__ void __launch_bounds__(256) k_gcr_axpy2(Grid g, VelBox boxes, const double *num, const double *den,
                                                   VelArrC<double> qi, VelArrC<double> zi, VelArr<double> q,
                                                   VelArr<double> z)
{
    const int a = blockIdx.y;
    int i, j, k;
    if (!box_pos(boxes.b[a], blockIdx.x * blockDim.x + threadIdx.x, i, j, k)) return;
    const double sc = num[0] / den[0];
    const long long e = at(g, i, j, k);
    q.c[a][e] -= sc * qi.c[a][e];
    z.c[a][e] -= sc * zi.c[a][e];
}

// x += s z at the unknowns (s = num / den), ghost images of x updated
__global__ void __launch_bounds__(256) k_gcr_update(Grid g, VelBox boxes, int velocity, const double *num,
                                                    const double *den, VelArrC<double> z, VelArr<double> x)
{
    const int a = blockIdx.y;
    int i, j, k;
    if (!box_pos(boxes.b[a], blockIdx.x * blockDim.x + threadIdx.x, i, j, k)) return;
    const double sc = num[0] / den[0];
    const long long e = at(g, i, j, k);
    const double v = x.c[a][e] + sc * z.c[a][e];
    x.c[a][e] = v;
    write_images(g, velocity ? face_mask(a) : 0, velocity ? ROLE_V : ROLE_P, x.c[a], i, j, k, v);
}

// ---------------------------------------------------------------------------
// the coarse part of a V-cycle in one workgroup
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline CoefU<T> coef_u(const LevTab<T> &lt)
{
    CoefU<T> cf;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cf.rho[a] = lt.rho[a];
        cf.mue[a] = lt.mue[a];
    }
    cf.muc = lt.muc;
    cf.dec = lt.dec;
    return cf;
}

// A x and the diagonal of one row of the velocity (VEL) or pressure system
template <typename T, int D, int VEL, int A>
__device__ inline void wg_row(const LevTab<T> &lt, int i, int j, int k, T &Ax, T &dg)
{
    if (VEL) {
        const VelArr<T> x{{lt.xu[0], lt.xu[1], lt.xu[2]}};
        u_row<T, D, A>(lt.g, x, coef_u(lt), lt.mass, lt.cvu, i, j, k, Ax, dg);
    } else {
        const CoefP<T> cf{{lt.beta[0], lt.beta[1], lt.beta[2]}};
        p_row<T, D>(lt.g, lt.xp, cf, lt.cvp, i, j, k, Ax, dg);
    }
}

// ---- per-point bodies, shared by the one-workgroup cycle and the batched
// passes; the arithmetic is that of the launched kernels

// red-black Gauss-Seidel update of the t-th point of one colour
template <typename T, int D, int VEL, int A>
__device__ inline void sweep_at(const LevTab<T> &lt, const Box &box, int colour, int t)
{
    int i, j, k;
    if (!box_colour_pos(box, colour, t, i, j, k)) return;
    T *x = VEL ? lt.xu[A] : lt.xp;
    const T *b = VEL ? lt.bu[A] : lt.bp;
    const long long e = at(lt.g, i, j, k);
    const T be = b[e], xe = x[e];
    T Ax, dg;
    wg_row<T, D, VEL, A>(lt, i, j, k, Ax, dg);
    const T xn = xe + (be - Ax) / dg;
    x[e] = xn;
    write_images(lt.g, VEL ? face_mask(A) : 0, VEL ? ROLE_V : ROLE_P, x, i, j, k, xn);
}

// r = b - A x at the t-th unknown of the box (t in range); returns r
template <typename T, int D, int VEL, int A>
__device__ inline T resid_at(const LevTab<T> &lt, const Box &box, int t)
{
    int i, j, k;
    box_pos(box, t, i, j, k);
    const long long e = at(lt.g, i, j, k);
    const T be = (VEL ? lt.bu[A] : lt.bp)[e];
    T Ax, dg;
    wg_row<T, D, VEL, A>(lt, i, j, k, Ax, dg);
    const T rv = be - Ax;
    (VEL ? lt.ru[A] : lt.rp)[e] = rv;
    return rv;
}

// coarse right-hand side = restriction of the fine residual at the t-th
// coarse unknown; the coarse correction there is cleared with its images
template <typename T, int D, int VEL, int A>
__device__ inline void restrict_at(const LevTab<T> &lt, const LevTab<T> &lc, const Box &box, int t)
{
    const int vmask = VEL ? face_mask(A) : 0;
    const int role = VEL ? ROLE_V : ROLE_P;
    int I, J, K;
    box_pos(box, t, I, J, K);
    const long long e = at(lc.g, I, J, K);
    (VEL ? lc.bu[A] : lc.bp)[e] = (T)restrict_any<T, D>(vmask, lt.g, role, VEL ? lt.ru[A] : lt.rp, I, J, K);
    T *xc = VEL ? lc.xu[A] : lc.xp;
    xc[e] = T(0);
    write_images(lc.g, vmask, role, xc, I, J, K, T(0));
}

// fine x += prolongation of the coarse correction at the t-th fine unknown
template <typename T, int D, int VEL, int A>
__device__ inline void prolong_at(const LevTab<T> &lc, const LevTab<T> &lt, const Box &box, int t)
{
    const int vmask = VEL ? face_mask(A) : 0;
    const int role = VEL ? ROLE_V : ROLE_P;
    int i, j, k;
    box_pos(box, t, i, j, k);
    T *x = VEL ? lt.xu[A] : lt.xp;
    const long long e = at(lt.g, i, j, k);
    const T xe = x[e];
    const T v = xe + (T)prolong_any<T, D>(vmask, lc.g, role, VEL ? lc.xu[A] : lc.xp, i, j, k);
    x[e] = v;
    write_images(lt.g, vmask, role, x, i, j, k, v);
}

__device__ inline int colour_count(const Box &b) { return ((b.ext[0] + 1) >> 1) * b.ext[1] * b.ext[2]; }
__device__ inline int point_count(const Box &b) { return b.ext[0] * b.ext[1] * b.ext[2]; }

template <typename T, int D, int VEL, int A>
__device__ inline void wg_sweep_comp(const LevTab<T> &ltr)
{
    const LevTab<T> lt = ltr;
    const Grid &g = lt.g;
    const int vmask = VEL ? face_mask(A) : 0;
    const Box box = unk_box(g, vmask);
    const BoxDiv bd = lt.bd[VEL ? A : 3];
    const int n = ((box.ext[0] + 1) >> 1) * box.ext[1] * box.ext[2];
    T *x = VEL ? lt.xu[A] : lt.xp;
    const T *b = VEL ? lt.bu[A] : lt.bp;
    for (int colour = 0; colour < 2; ++colour) {
        for (int t = threadIdx.x; t < n; t += blockDim.x) {
            int i, j, k;
            if (!box_colour_pos(box, bd, colour, t, i, j, k)) continue;
            const long long e = at(g, i, j, k);
            const T be = b[e], xe = x[e];
            T Ax, dg;
            wg_row<T, D, VEL, A>(lt, i, j, k, Ax, dg);
            const T xn = xe + (be - Ax) / dg;
            x[e] = xn;
            write_images(g, vmask, VEL ? ROLE_V : ROLE_P, x, i, j, k, xn);
        }
        __syncthreads();
    }
}

template <typename T, int D, int VEL>
__device__ void wg_sweep(const LevTab<T> &lt)
{
    wg_sweep_comp<T, D, VEL, 0>(lt);
    if (VEL) {
        wg_sweep_comp<T, D, VEL, 1>(lt);
        if (D == 3) wg_sweep_comp<T, D, VEL, (D == 3 ? 2 : 1)>(lt);
    }
}

template <typename T, int D, int VEL, int A>
__device__ inline void wg_residual_comp(const LevTab<T> &ltr)
{
    const LevTab<T> lt = ltr;
    const Box box = unk_box(lt.g, VEL ? face_mask(A) : 0);
    const BoxDiv bd = lt.bd[VEL ? A : 3];
    const int n = box.ext[0] * box.ext[1] * box.ext[2];
    T *r = VEL ? lt.ru[A] : lt.rp;
    const T *b = VEL ? lt.bu[A] : lt.bp;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        int i, j, k;
        box_pos(box, bd, t, i, j, k);
        const long long e = at(lt.g, i, j, k);
        const T be = b[e];
        T Ax, dg;
        wg_row<T, D, VEL, A>(lt, i, j, k, Ax, dg);
        r[e] = be - Ax;
    }
}

// coarse right-hand side = restriction of the fine residual, coarse
// correction cleared (with its images)
template <typename T, int D, int VEL, int A>
__device__ inline void wg_restrict_comp(const LevTab<T> &ltr, const LevTab<T> &lcr)
{
    const LevTab<T> lt = ltr, lc = lcr;
    const int vmask = VEL ? face_mask(A) : 0;
    const int role = VEL ? ROLE_V : ROLE_P;
    const Box box = unk_box(lc.g, vmask);
    const BoxDiv bd = lc.bd[VEL ? A : 3];
    const int n = box.ext[0] * box.ext[1] * box.ext[2];
    const T *src = VEL ? lt.ru[A] : lt.rp;
    T *bc = VEL ? lc.bu[A] : lc.bp;
    T *xc = VEL ? lc.xu[A] : lc.xp;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        int I, J, K;
        box_pos(box, bd, t, I, J, K);
        const long long e = at(lc.g, I, J, K);
        bc[e] = (T)restrict_any<T, D>(vmask, lt.g, role, src, I, J, K);
        xc[e] = T(0);
        write_images(lc.g, vmask, role, xc, I, J, K, T(0));
    }
}

template <typename T, int D, int VEL, int A>
__device__ inline void wg_prolong_comp(const LevTab<T> &lcr, const LevTab<T> &ltr)
{
    const LevTab<T> lc = lcr, lt = ltr;
    const int vmask = VEL ? face_mask(A) : 0;
    const int role = VEL ? ROLE_V : ROLE_P;
    const Box box = unk_box(lt.g, vmask);
    const BoxDiv bd = lt.bd[VEL ? A : 3];
    const int n = box.ext[0] * box.ext[1] * box.ext[2];
    const T *src = VEL ? lc.xu[A] : lc.xp;
    T *x = VEL ? lt.xu[A] : lt.xp;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        int i, j, k;
        box_pos(box, bd, t, i, j, k);
        const long long e = at(lt.g, i, j, k);
        const T xe = x[e];
        const T v = xe + (T)prolong_any<T, D>(vmask, lc.g, role, src, i, j, k);
        x[e] = v;
        write_images(lt.g, vmask, role, x, i, j, k, v);
    }
}

// Restriction of the fine residual onto the tail's unknowns, as a compact
// vector (bv[t]: the t-th unknown of the tail level); the same arithmetic as
// the restriction into the coarse level's b.
template <typename T, int D, int VEL>
__device__ inline void wg_restrict_tail(const LevTab<T> &ltr, const Grid &gc, const Tail &tail, T *bv)
{
    const LevTab<T> lt = ltr;
    const int role = VEL ? ROLE_V : ROLE_P;
    for (int t = threadIdx.x; t < tail.n; t += blockDim.x) {
        const int a = tail.comp[t];
        int I, J, K;
        decode(gc, tail.idx[t], I, J, K);
        const T *src = VEL ? (a == 0 ? lt.ru[0] : (a == 1 ? lt.ru[1] : lt.ru[2])) : lt.rp;
        bv[t] = (T)restrict_any<T, D>(VEL ? face_mask(a) : 0, lt.g, role, src, I, J, K);
    }
}

// x = Tm bv at the tail's unknowns, with the ghost images of x; the rest of
// x is zero already.  Tm is stored in blocks of W columns (W = 16 bytes over
// the element size): block q holds, row after row, the W entries of columns
// qW .. qW+W-1, so that the 64 rows of a wave read one contiguous kilobyte
// per 16-byte load.  Each thread sums its own row in column order.
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
    using type = float4;
    static constexpr int n = 4;
};
template <>
struct Vec16<double> {
    using type = double2;
    static constexpr int n = 2;
};

__host__ __device__ inline int tail_ld(int n, int wsz) { return wsz == 4 ? (n + 3) & ~3 : (n + 1) & ~1; }

// position of entry (row r, column j) of an n-row tail matrix
template <typename T>
__device__ inline long long tail_at(int n, int r, int j)
{
    constexpr int W = Vec16<T>::n;
    return (long long)(j / W) * ((long long)n * W) + (long long)r * W + (j % W);
}

template <typename T, int D, int VEL>
__device__ inline void wg_apply_tail(const LevTab<T> &lcr, const Tail &tail, const T *bv)
{
    using V = typename Vec16<T>::type;
    constexpr int W = Vec16<T>::n;
    const LevTab<T> lc = lcr;
    const T *__restrict__ Tm = static_cast<const T *>(tail.Tm);
    const int n = tail.n;
    const int nq = n / W;
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
        const V *__restrict__ rv = reinterpret_cast<const V *>(Tm) + r;
        T sum = T(0);
#pragma unroll 8
        for (int q = 0; q < nq; ++q) {
            const V t = rv[(long long)q * n];
            const T *tt = reinterpret_cast<const T *>(&t);
#pragma unroll
            for (int w = 0; w < W; ++w) sum += tt[w] * bv[q * W + w];
        }
        for (int j = nq * W; j < n; ++j) sum += Tm[tail_at<T>(n, r, j)] * bv[j];
        const int a = tail.comp[r];
        T *x = VEL ? (a == 0 ? lc.xu[0] : (a == 1 ? lc.xu[1] : lc.xu[2])) : lc.xp;
        const long long e = tail.idx[r];
        x[e] = sum;
        int i, j, k;
        decode(lc.g, e, i, j, k);
        write_images(lc.g, VEL ? face_mask(a) : 0, VEL ? ROLE_V : ROLE_P, x, i, j, k, sum);
    }
}

// The part of a V-cycle from level l0 down to the coarsest level and back,
// in one workgroup: the same passes, in the same order, as the launched
// kernels, with a barrier where a launch boundary would be.  With a tail
// (tail.n > 0, tail.level = l0 + 1) the levels below l0 are the tail's
// matrix applied to the restricted residual (bv: shared scratch of
// TAIL_MAX values).
template <typename T, int D, int VEL>
__device__ __attribute__((always_inline)) inline void coarse_cycle(const LevTab<T> *__restrict__ tab, int l0, int L, int nu1,
                                                                  int nu2, int ndense,
                                    const long long *__restrict__ uidx, const int *__restrict__ ucomp,
                                    const double *__restrict__ M, const Tail &tail, T *bv)
{
    constexpr int A2 = D == 3 ? 2 : 1;
    const bool tailed = tail.n > 0;
    const int lb = tailed ? tail.level : L - 1;   // bottom of the recursion
    for (int l = l0; l < lb; ++l) {
        const LevTab<T> &lt = tab[l];
        for (int s = 0; s < nu1; ++s) wg_sweep<T, D, VEL>(lt);
        wg_residual_comp<T, D, VEL, 0>(lt);
        if (VEL) {
            wg_residual_comp<T, D, VEL, 1>(lt);
            if (D == 3) wg_residual_comp<T, D, VEL, A2>(lt);
        }
        __syncthreads();
        const LevTab<T> &lc = tab[l + 1];
        if (tailed && l + 1 == lb) {
            wg_restrict_tail<T, D, VEL>(lt, lc.g, tail, bv);
        } else {
            wg_restrict_comp<T, D, VEL, 0>(lt, lc);
            if (VEL) {
                wg_restrict_comp<T, D, VEL, 1>(lt, lc);
                if (D == 3) wg_restrict_comp<T, D, VEL, A2>(lt, lc);
            }
        }
        __syncthreads();
    }
    if (tailed) {
        wg_apply_tail<T, D, VEL>(tab[lb], tail, bv);
        __syncthreads();
    } else {
        const LevTab<T> lt = tab[L - 1];
        if (ndense > 0) {
            __shared__ double dv[64];
            const int r = threadIdx.x;
            if (r < ndense) {
                const int c = ucomp[r];
                const T *b = VEL ? (c == 0 ? lt.bu[0] : (c == 1 ? lt.bu[1] : lt.bu[2])) : lt.bp;
                dv[r] = (double)b[uidx[r]];
            }
            __syncthreads();
            if (r < ndense) {
                double sum = 0.0;
                for (int j = 0; j < ndense; ++j) sum += M[r * ndense + j] * dv[j];
                const int c = ucomp[r];
                T *x = VEL ? (c == 0 ? lt.xu[0] : (c == 1 ? lt.xu[1] : lt.xu[2])) : lt.xp;
                x[uidx[r]] = (T)sum;
                int i, jj, k;
                decode(lt.g, uidx[r], i, jj, k);
                write_images(lt.g, VEL ? face_mask(c) : 0, VEL ? ROLE_V : ROLE_P, x, i, jj, k, (T)sum);
            }
            __syncthreads();
        } else {
            for (int s = 0; s < nu1 + nu2; ++s) wg_sweep<T, D, VEL>(lt);
        }
    }
    for (int l = lb - 1; l >= l0; --l) {
        const LevTab<T> &lt = tab[l];
        const LevTab<T> &lc = tab[l + 1];
        wg_prolong_comp<T, D, VEL, 0>(lc, lt);
        if (VEL) {
            wg_prolong_comp<T, D, VEL, 1>(lc, lt);
            if (D == 3) wg_prolong_comp<T, D, VEL, A2>(lc, lt);
        }
        __syncthreads();
        for (int s = 0; s < nu2; ++s) wg_sweep<T, D, VEL>(lt);
    }
}


// an array of a staged level: its place in the arena, or (offset -1) the
// array where it already is
template <typename T>
__device__ inline T *arena_ptr(unsigned char *arena, int off, T *global)
{
    return off >= 0 ? reinterpret_cast<T *>(arena + off) : global;
}

// The workgroup's table of levels: the global tables, with the arrays of the
// levels from ls down that the plan places in the LDS arena rebased there.
// Staged coefficients are copied in.  Staged solver arrays are cleared,
// except on the start level l0, whose x and b carry the cycle's input.  Only
// levels ls .. lend - 1 are touched, and of them only the staged arrays.
template <typename T, int D, int VEL>
__device__ inline void stage_levels(const LevTab<T> *__restrict__ tab, int l0, int L, int ls, int lend,
                                    const LdsLevel *__restrict__ lev, unsigned char *arena, LevTab<T> *wt)
{
    for (int l = threadIdx.x; l < L; l += blockDim.x) {
        LevTab<T> t = tab[l];
        if (l >= ls) {
            const LdsLevel o = lev[l];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                t.xu[a] = arena_ptr<T>(arena, o.xu[a], t.xu[a]);
                t.bu[a] = arena_ptr<T>(arena, o.bu[a], t.bu[a]);
                t.ru[a] = arena_ptr<T>(arena, o.ru[a], t.ru[a]);
                t.rho[a] = arena_ptr<T>(arena, o.rho[a], const_cast<T *>(t.rho[a]));
                t.beta[a] = arena_ptr<T>(arena, o.beta[a], const_cast<T *>(t.beta[a]));
                t.mue[a] = arena_ptr<T>(arena, o.mue[a], const_cast<T *>(t.mue[a]));
            }
            t.xp = arena_ptr<T>(arena, o.xp, t.xp);
            t.bp = arena_ptr<T>(arena, o.bp, t.bp);
            t.rp = arena_ptr<T>(arena, o.rp, t.rp);
            t.muc = arena_ptr<T>(arena, o.muc, const_cast<T *>(t.muc));
        }
        wt[l] = t;
    }
    __syncthreads();
    for (int l = ls; l < lend; ++l) {
        const LevTab<T> src = tab[l];
        const LevTab<T> dst = wt[l];
        const bool start = l == l0;
        const int nel = (int)src.g.nel;
        // two elements per round, every load before any store, so that a
        // round costs one trip to global memory
        constexpr int U = 2;
        for (int e0 = threadIdx.x; e0 < nel; e0 += U * blockDim.x) {
            if (VEL) {
                T rh[U][3], xv[U][3], bv[U][3], mc[U], me[U][3];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int e = e0 + u * blockDim.x;
                    if (e >= nel) break;
#pragma unroll
                    for (int a = 0; a < D; ++a) {
                        if (dst.rho[a] != src.rho[a]) rh[u][a] = src.rho[a][e];
                        xv[u][a] = start ? src.xu[a][e] : T(0);
                        bv[u][a] = start ? src.bu[a][e] : T(0);
                    }
                    if (dst.muc != src.muc) mc[u] = src.muc[e];
#pragma unroll
                    for (int a = 0; a < 3; ++a)
                        if (dst.mue[a] && dst.mue[a] != src.mue[a]) me[u][a] = src.mue[a][e];
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int e = e0 + u * blockDim.x;
                    if (e >= nel) break;
#pragma unroll
                    for (int a = 0; a < D; ++a) {
                        if (dst.rho[a] != src.rho[a]) const_cast<T *>(dst.rho[a])[e] = rh[u][a];
                        if (dst.xu[a] != src.xu[a]) dst.xu[a][e] = xv[u][a];
                        if (dst.bu[a] != src.bu[a]) dst.bu[a][e] = bv[u][a];
                        if (dst.ru[a] != src.ru[a]) dst.ru[a][e] = T(0);
                    }
                    if (dst.muc != src.muc) const_cast<T *>(dst.muc)[e] = mc[u];
#pragma unroll
                    for (int a = 0; a < 3; ++a)
                        if (dst.mue[a] && dst.mue[a] != src.mue[a]) const_cast<T *>(dst.mue[a])[e] = me[u][a];
                }
            } else {
                T bt[U][3], xv[U], bv[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int e = e0 + u * blockDim.x;
                    if (e >= nel) break;
#pragma unroll
                    for (int a = 0; a < D; ++a)
                        if (dst.beta[a] != src.beta[a]) bt[u][a] = src.beta[a][e];
                    xv[u] = start ? src.xp[e] : T(0);
                    bv[u] = start ? src.bp[e] : T(0);
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int e = e0 + u * blockDim.x;
                    if (e >= nel) break;
#pragma unroll
                    for (int a = 0; a < D; ++a)
                        if (dst.beta[a] != src.beta[a]) const_cast<T *>(dst.beta[a])[e] = bt[u][a];
                    if (dst.xp != src.xp) dst.xp[e] = xv[u];
                    if (dst.bp != src.bp) dst.bp[e] = bv[u];
                    if (dst.rp != src.rp) dst.rp[e] = T(0);
                }
            }
        }
    }
    __syncthreads();
}

// a staged start level hands its iterate (with its ghost images) back
template <typename T, int D, int VEL>
__device__ inline void unstage_start(const LevTab<T> *__restrict__ tab, int l0, int ls, const LevTab<T> *wt)
{
    if (l0 < ls) return;
    __syncthreads();
    const LevTab<T> src = wt[l0];
    const LevTab<T> dst = tab[l0];
    const int nel = (int)dst.g.nel;
    for (int e = threadIdx.x; e < nel; e += blockDim.x) {
        if (VEL) {
#pragma unroll
            for (int a = 0; a < D; ++a) dst.xu[a][e] = src.xu[a][e];
        } else {
            dst.xp[e] = src.xp[e];
        }
    }
}

template <typename T, int D, int VEL>
__global__ void __launch_bounds__(wg_threads(D, VEL)) k_coarse_vcycle(const LevTab<T> *__restrict__ tab, int l0, int L, int nu1,
                                                               int nu2, int ndense, const long long *__restrict__ uidx,
                                                               const int *__restrict__ ucomp,
                                                               const double *__restrict__ M, LdsPlan plan, Tail tail)
{
    extern __shared__ __align__(16) unsigned char wg_arena[];
    __shared__ LevTab<T> wt[WG_MAXLEV];
    __shared__ T bv[TAIL_MAX];
    stage_levels<T, D, VEL>(tab, l0, L, plan.ls, tail.n > 0 ? tail.level + 1 : L, plan.lev, wg_arena, wt);
    coarse_cycle<T, D, VEL>(wt, l0, L, nu1, nu2, ndense, uidx, ucomp, M, tail, bv);
    unstage_start<T, D, VEL>(tab, l0, plan.ls, wt);
}

// Column j of a tail's matrix: the cycle from the tail's level down and back,
// on the unit right-hand side of its j-th unknown, every level staged in LDS
// (the plan stages all of them; no level is a start level, so every solver
// array begins at zero).
template <typename T, int D, int VEL>
__global__ void __launch_bounds__(wg_threads(D, VEL)) k_tail_columns(const LevTab<T> *__restrict__ tab, int L, int nu1,
                                                                    int nu2, int ndense,
                                                                    const long long *__restrict__ uidx,
                                                                    const int *__restrict__ ucomp,
                                                                    const double *__restrict__ M, LdsPlan plan,
                                                                    Tail tail)
{
    extern __shared__ __align__(16) unsigned char wg_arena[];
    __shared__ LevTab<T> wt[WG_MAXLEV];
    __shared__ T bv[1];
    const int lt = tail.level;
    const int j = blockIdx.x;
    stage_levels<T, D, VEL>(tab, -1, L, plan.ls, L, plan.lev, wg_arena, wt);
    if (threadIdx.x == 0) {
        const int a = tail.comp[j];
        T *b = VEL ? (a == 0 ? wt[lt].bu[0] : (a == 1 ? wt[lt].bu[1] : wt[lt].bu[2])) : wt[lt].bp;
        b[tail.idx[j]] = T(1);
    }
    __syncthreads();
    const Tail none{nullptr, nullptr, nullptr, 0, 0};
    coarse_cycle<T, D, VEL>(wt, lt, L, nu1, nu2, ndense, uidx, ucomp, M, none, bv);
    __syncthreads();
    T *Tm = const_cast<T *>(static_cast<const T *>(tail.Tm));
    for (int r = threadIdx.x; r < tail.n; r += blockDim.x) {
        const int a = tail.comp[r];
        const T *x = VEL ? (a == 0 ? wt[lt].xu[0] : (a == 1 ? wt[lt].xu[1] : wt[lt].xu[2])) : wt[lt].xp;
        Tm[tail_at<T>(tail.n, r, j)] = x[tail.idx[r]];
    }
}

// ---------------------------------------------------------------------------
// batched passes: one launch covers the same pass of several contexts.
// Block b of a launch works for the context described by ent[b]; a context
// whose flag is clear is skipped.  Each point is updated exactly as by the
// single-context kernels above.
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline const LevTab<T> &tab_of(const void *p) { return *static_cast<const LevTab<T> *>(p); }

// A copy of the i-th level table at p, read through scalar loads.  The tables
// are written once when a context is created and every lane of a block reads
// the same one; through a generic pointer they would come in with vector
// loads, one more round trip that the row's own loads wait behind.
template <typename T>
__device__ inline LevTab<T> tab_copy(const void *p, int i = 0)
{
    constexpr int N = sizeof(LevTab<T>) / 4;
    static_assert(sizeof(LevTab<T>) % 4 == 0, "the table is read in 4-byte words");
    typedef const __attribute__((address_space(4))) unsigned int ConstWord;
    const ConstWord *w = (const ConstWord *)p + (long long)i * N;
    struct Words {
        unsigned int v[N];
    } r;
#pragma unroll
    for (int k = 0; k < N; ++k) r.v[k] = w[k];
    return __builtin_bit_cast(LevTab<T>, r);
}

template <typename T, int D, int VEL, int A>
__global__ void __launch_bounds__(256) k_bsweep(const BEntry *__restrict__ ent, const int *__restrict__ flags,
                                                int colour)
{
    const BEntry E = ent[blockIdx.x];
    const int on = flags[E.ctx];
    const LevTab<T> lt = tab_copy<T>(E.tab);
    if (!on) return;
    const Box box = unk_box(lt.g, VEL ? face_mask(A) : 0);
    sweep_at<T, D, VEL, A>(lt, box, colour, (int)(blockIdx.x - E.base) * blockDim.x + threadIdx.x);
}

// residual of every component (blockIdx.y) with a grid-stride loop over the
// context's nb blocks; with E.partial set, per-block sums of r^2 in the
// layout of the single-context residual kernels
template <typename T, int D, int VEL>
__global__ void __launch_bounds__(256) k_bresid(const BEntry *__restrict__ ent, const int *__restrict__ flags)
{
    const BEntry E = ent[blockIdx.x];
    const int on = flags[E.ctx];
    const LevTab<T> lt = tab_copy<T>(E.tab);
    if (!on) return;
    const int a = blockIdx.y;
    const int lb = blockIdx.x - E.base;
    const Box box = unk_box(lt.g, VEL ? face_mask(a) : 0);
    const int n = point_count(box);
    double acc = 0.0;
    for (int t = lb * blockDim.x + threadIdx.x; t < n; t += E.nb * blockDim.x) {
        T rv;
        if (a == 0) rv = resid_at<T, D, VEL, 0>(lt, box, t);
        else if (a == 1) rv = resid_at<T, D, VEL, 1>(lt, box, t);
        else rv = resid_at<T, D, VEL, (D == 3 ? 2 : 1)>(lt, box, t);
        acc += (double)rv * (double)rv;
    }
    if (E.partial) block_sum_store(acc, E.partial, (long long)a * E.nb + lb);
}

// one block per context: norms[ctx] = sum of its E.nb partial sums, in the
// order of the single-context final reduction
__global__ void __launch_bounds__(256) k_breduce(const BEntry *__restrict__ ent, const int *__restrict__ flags,
                                                 double *norms)
{
    const BEntry E = ent[blockIdx.x];
    if (!flags[E.ctx]) return;
    double acc = 0.0;
    for (long long t = threadIdx.x; t < E.nb; t += blockDim.x) acc += E.partial[t];
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) norms[E.ctx] = red[0];
}

// restriction to the next level (the context's table at l and l + 1)
template <typename T, int D, int VEL>
__global__ void __launch_bounds__(256) k_brestrict(const BEntry *__restrict__ ent, const int *__restrict__ flags)
{
    const BEntry E = ent[blockIdx.x];
    if (!flags[E.ctx]) return;
    const LevTab<T> lt = tab_copy<T>(E.tab, 0);
    const LevTab<T> lc = tab_copy<T>(E.tab, 1);
    const int a = blockIdx.y;
    const Box box = unk_box(lc.g, VEL ? face_mask(a) : 0);
    const int t = (blockIdx.x - E.base) * blockDim.x + threadIdx.x;
    if (t >= point_count(box)) return;
    if (a == 0) restrict_at<T, D, VEL, 0>(lt, lc, box, t);
    else if (a == 1) restrict_at<T, D, VEL, 1>(lt, lc, box, t);
    else restrict_at<T, D, VEL, (D == 3 ? 2 : 1)>(lt, lc, box, t);
}

template <typename T, int D, int VEL>
__global__ void __launch_bounds__(256) k_bprolong(const BEntry *__restrict__ ent, const int *__restrict__ flags)
{
    const BEntry E = ent[blockIdx.x];
    if (!flags[E.ctx]) return;
    const LevTab<T> lt = tab_copy<T>(E.tab, 0);
    const LevTab<T> lc = tab_copy<T>(E.tab, 1);
    const int a = blockIdx.y;
    const Box box = unk_box(lt.g, VEL ? face_mask(a) : 0);
    const int t = (blockIdx.x - E.base) * blockDim.x + threadIdx.x;
    if (t >= point_count(box)) return;
    if (a == 0) prolong_at<T, D, VEL, 0>(lc, lt, box, t);
    else if (a == 1) prolong_at<T, D, VEL, 1>(lc, lt, box, t);
    else prolong_at<T, D, VEL, (D == 3 ? 2 : 1)>(lc, lt, box, t);
}

// refined solver, start of an outer iteration: FP32 right-hand side = the
// FP64 residual at the unknowns, FP32 correction cleared (whole arrays)
template <int VEL>
__global__ void __launch_bounds__(256) k_bprep32(const BEntry *__restrict__ ent, const int *__restrict__ flags)
{
    const BEntry E = ent[blockIdx.x];
    if (!flags[E.ctx]) return;
    const LevTab<double> &l64 = tab_of<double>(E.tab);
    const LevTab<float> &l32 = tab_of<float>(E.tab2);
    const int t = (blockIdx.x - E.base) * blockDim.x + threadIdx.x;
    const int ncomp = VEL ? l64.g.D : 1;
    for (int a = 0; a < ncomp; ++a) {
        float *x32 = VEL ? l32.xu[a] : l32.xp;
        if (t < l64.g.nel) x32[t] = 0.0f;
        const Box box = unk_box(l64.g, VEL ? face_mask(a) : 0);
        int i, j, k;
        if (t < point_count(box)) {
            box_pos(box, t, i, j, k);
            const long long e = at(l64.g, i, j, k);
            (VEL ? l32.bu[a] : l32.bp)[e] = (float)(VEL ? l64.ru[a] : l64.rp)[e];
        }
    }
}

// refined solver, end of an outer iteration: x += (double) e at the unknowns
template <int VEL>
__global__ void __launch_bounds__(256) k_badd(const BEntry *__restrict__ ent, const int *__restrict__ flags)
{
    const BEntry E = ent[blockIdx.x];
    if (!flags[E.ctx]) return;
    const LevTab<double> &l64 = tab_of<double>(E.tab);
    const LevTab<float> &l32 = tab_of<float>(E.tab2);
    const int a = blockIdx.y;
    const int vmask = VEL ? face_mask(a) : 0;
    const Box box = unk_box(l64.g, vmask);
    const int t = (blockIdx.x - E.base) * blockDim.x + threadIdx.x;
    if (t >= point_count(box)) return;
    int i, j, k;
    box_pos(box, t, i, j, k);
    const long long q = at(l64.g, i, j, k);
    double *x = VEL ? l64.xu[a] : l64.xp;
    const double v = x[q] + (double)(VEL ? l32.xu[a] : l32.xp)[q];
    x[q] = v;
    write_images(l64.g, vmask, VEL ? ROLE_V : ROLE_P, x, i, j, k, v);
}

// the coarse part of the V-cycle of every context, one workgroup each
template <typename T, int D, int VEL>
__global__ void __launch_bounds__(wg_threads(D, VEL)) k_bcoarse(const BCoarse *__restrict__ items, const int *__restrict__ flags,
                                                  int nu1, int nu2)
{
    const BCoarse I = items[blockIdx.x];
    if (!flags[I.ctx]) return;
    extern __shared__ __align__(16) unsigned char wg_arena[];
    __shared__ LevTab<T> wt[WG_MAXLEV];
    __shared__ T bv[TAIL_MAX];
    const LevTab<T> *tab = static_cast<const LevTab<T> *>(I.tab);
    stage_levels<T, D, VEL>(tab, I.l0, I.L, I.lds_from, I.tail.n > 0 ? I.tail.level + 1 : I.L, I.lds, wg_arena, wt);
    coarse_cycle<T, D, VEL>(wt, I.l0, I.L, nu1, nu2, I.ndense, I.uidx, I.ucomp, I.M, I.tail, bv);
    unstage_start<T, D, VEL>(tab, I.l0, I.lds_from, wt);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(long long n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

// events armed for the next timed launch (set_launch_events): the kernel's
// own start and end are recorded into them by the dispatch
static thread_local hipEvent_t t_ev_start = nullptr, t_ev_stop = nullptr;

void set_launch_events(hipEvent_t start, hipEvent_t stop)
{
    t_ev_start = start;
    t_ev_stop = stop;
}

bool take_launch_events(hipEvent_t *start, hipEvent_t *stop)
{
    if (!t_ev_start) return false;
    *start = t_ev_start;
    *stop = t_ev_stop;
    t_ev_start = t_ev_stop = nullptr;
    return true;
}

static inline long long box_count(const Box &b) { return (long long)b.ext[0] * b.ext[1] * b.ext[2]; }

// rows per band of a z-blocked pass: about one point of the colour per
// thread in each plane, at least 4 rows
static inline int zb_rows(const Box &P) { return std::max(4, 256 / std::max(1, (P.ext[0] + 1) / 2)); }

template <typename T>
void launch_smooth_p(const Grid &g, const T *b, T *x, const CoefP<T> &cf, T cvisc, int colour, hipStream_t s, int zb)
{
    const Box P = unk_box(g, 0);
    const long long n = (long long)((P.ext[0] + 1) / 2) * P.ext[1] * P.ext[2];
    if (n <= 0) return;
    if (zb && g.D == 3) {
        const int rows = zb_rows(P), nbands = (P.ext[1] + rows - 1) / rows;
        const int nz = (P.ext[2] + ZB_PLANES - 1) / ZB_PLANES;
        launch_timed(k_smooth_p_zb<T>, dim3((unsigned)(nbands * nz)), dim3(256), s, g, P, b, x, cf, cvisc, colour, rows,
                     nbands);
        return;
    }
    const int remap = g.nel <= XCD_REMAP_MAX_NEL;
    if (g.D == 3)
        launch_timed(k_smooth_p<T, 3>, dim3(blocks_for(n)), dim3(256), s, g, P, b, x, cf, cvisc, colour, remap);
    else
        launch_timed(k_smooth_p<T, 2>, dim3(blocks_for(n)), dim3(256), s, g, P, b, x, cf, cvisc, colour, remap);
}

template <typename T>
void launch_smooth_u(const Grid &g, int a, const T *b, const VelArr<T> &x, const CoefU<T> &cf, T mass, T cvisc,
                     int colour, hipStream_t s, int zb)
{
    const Box P = unk_box(g, face_mask(a));
    const long long n = (long long)((P.ext[0] + 1) / 2) * P.ext[1] * P.ext[2];
    if (n <= 0) return;
    if (zb && g.D == 3) {
        const int rows = zb_rows(P), nbands = (P.ext[1] + rows - 1) / rows;
        const int nz = (P.ext[2] + ZB_PLANES - 1) / ZB_PLANES;
        const dim3 grid((unsigned)(nbands * nz)), blk(256);
        if (a == 0) launch_timed(k_smooth_u_zb<T, 0>, grid, blk, s, g, P, b, x, cf, mass, cvisc, colour, rows, nbands);
        else if (a == 1) launch_timed(k_smooth_u_zb<T, 1>, grid, blk, s, g, P, b, x, cf, mass, cvisc, colour, rows, nbands);
        else launch_timed(k_smooth_u_zb<T, 2>, grid, blk, s, g, P, b, x, cf, mass, cvisc, colour, rows, nbands);
        return;
    }
    const dim3 grid(blocks_for(n)), blk(256);
    const int remap = g.nel <= XCD_REMAP_MAX_NEL;
    if (g.D == 3) {
        if (a == 0) launch_timed(k_smooth_u<T, 3, 0>, grid, blk, s, g, P, b, x, cf, mass, cvisc, colour, remap);
        else if (a == 1) launch_timed(k_smooth_u<T, 3, 1>, grid, blk, s, g, P, b, x, cf, mass, cvisc, colour, remap);
        else launch_timed(k_smooth_u<T, 3, 2>, grid, blk, s, g, P, b, x, cf, mass, cvisc, colour, remap);
    } else {
        if (a == 0) launch_timed(k_smooth_u<T, 2, 0>, grid, blk, s, g, P, b, x, cf, mass, cvisc, colour, remap);
        else launch_timed(k_smooth_u<T, 2, 1>, grid, blk, s, g, P, b, x, cf, mass, cvisc, colour, remap);
    }
}

template <typename T>
void launch_smooth_u_dec(const Grid &g, const VelArrC<T> &b, const VelArr<T> &x, const CoefU<T> &cf, T mass, T cvisc,
                         int colour, hipStream_t s)
{
    VelBox parts;
    long long mx = 0;
    for (int a = 0; a < 3; ++a) {
        parts.b[a] = a < g.D ? unk_box(g, face_mask(a)) : Box{{0, 0, 0}, {0, 0, 0}};
        if (a >= g.D) continue;
        const Box &P = parts.b[a];
        const long long n = (long long)((P.ext[0] + 1) / 2) * P.ext[1] * P.ext[2];
        mx = n > mx ? n : mx;
    }
    if (mx <= 0) return;
    const dim3 grid(blocks_for(mx), g.D), blk(256);
    const int remap = g.nel <= XCD_REMAP_MAX_NEL;
    if (g.D == 3) launch_timed(k_smooth_u_dec<T, 3>, grid, blk, s, g, parts, b, x, cf, mass, cvisc, colour, remap);
    else launch_timed(k_smooth_u_dec<T, 2>, grid, blk, s, g, parts, b, x, cf, mass, cvisc, colour, remap);
}

template <typename T>
void launch_smooth_rb(const Grid &g, int vel, int a, const VelArrC<T> &xin, const T *b, const CoefU<T> &cu,
                      const CoefP<T> &cp, T mass, T cvisc, T *xout, hipStream_t s)
{
    const Box P = unk_box(g, vel ? face_mask(a) : 0);
    if (box_count(P) <= 0) return;
    const int D = g.D;
    const int TX = D == 3 ? 8 : 16, TY = D == 3 ? 8 : 16, TZ = D == 3 ? (sizeof(T) == 8 ? 4 : 8) : 1;
    const unsigned nt = (unsigned)(((P.ext[0] + TX - 1) / TX) * ((P.ext[1] + TY - 1) / TY) * ((P.ext[2] + TZ - 1) / TZ));
    const dim3 grid(nt), blk(256);
#define RB(DD, VV, AA) launch_timed(k_smooth_rb<T, DD, VV, AA>, grid, blk, s, g, P, xin, b, cu, cp, mass, cvisc, xout)
    if (D == 3) {
        if (!vel) RB(3, 0, 0);
        else if (a == 0) RB(3, 1, 0);
        else if (a == 1) RB(3, 1, 1);
        else RB(3, 1, 2);
    } else {
        if (!vel) RB(2, 0, 0);
        else if (a == 0) RB(2, 1, 0);
        else RB(2, 1, 1);
    }
#undef RB
}

// Runs of planes per workgroup for the z-marching sweep: about
// ZM_TARGET_BLOCKS workgroups, at least ZM_MIN_RUN planes each (each run also
// updates the red points of the two planes around it).
constexpr int ZM_TARGET_BLOCKS = 8192, ZM_MIN_RUN = 4;

int zm_run(const Box &P)
{
    const long long tiles = (long long)((P.ext[0] + ZM_TX - 1) / ZM_TX) * ((P.ext[1] + ZM_TY - 1) / ZM_TY);
    const long long want = std::max<long long>(1, (ZM_TARGET_BLOCKS + tiles - 1) / tiles);
    const int runs = (int)std::max<long long>(1, std::min<long long>(want, P.ext[2] / ZM_MIN_RUN));
    return (P.ext[2] + runs - 1) / runs;
}

bool zm_fits(const Grid &g)
{
    if (g.D != 3) return false;
    const int need[3] = {ZM_WX, ZM_WY, ZM_NS + 2};
    for (int d = 0; d < 3; ++d)
        if (g.bc[d] == AX_PERIODIC && (g.n[d] < need[d] || g.n[d] % 2)) return false;
    return true;
}

template <typename T>
void launch_smooth_zm(const Grid &g, int a, const VelArrC<T> &xin, const T *b, const CoefU<T> &cu, T mass, T cvisc,
                      T *xout, hipStream_t s)
{
    const Box P = unk_box(g, face_mask(a));
    if (box_count(P) <= 0) return;
    const int cz = zm_run(P);
    const long long nb = (long long)((P.ext[0] + ZM_TX - 1) / ZM_TX) * ((P.ext[1] + ZM_TY - 1) / ZM_TY) *
                         ((P.ext[2] + cz - 1) / cz);
    const dim3 grid((unsigned)nb), blk(ZM_BS);
    const int remap = 1;
#define ZM(AA) launch_timed(k_smooth_zm<T, AA>, grid, blk, s, g, P, xin, b, cu, mass, cvisc, xout, cz, remap)
    if (a == 0) ZM(0);
    else if (a == 1) ZM(1);
    else ZM(2);
#undef ZM
}

static inline unsigned stride_blocks(long long n)
{
    const unsigned b = blocks_for(n);
    const long long want = std::max<long long>(NORM_BLOCKS, (n + 256 * 16 - 1) / (256 * 16));
    const unsigned cap = (unsigned)std::min<long long>(want, NORM_BLOCKS_MAX);
    return b < cap ? (b ? b : 1) : cap;
}

template <typename T>
int launch_resid_p(const Grid &g, const T *b, const T *x, const CoefP<T> &cf, T cvisc, T *r, double *partial,
                   hipStream_t s)
{
    const Box P = unk_box(g, 0);
    const unsigned nb = stride_blocks(box_count(P));
    if (g.D == 3) launch_timed(k_resid_p<T, 3>, dim3(nb), dim3(256), s, g, P, b, x, cf, cvisc, r, partial);
    else launch_timed(k_resid_p<T, 2>, dim3(nb), dim3(256), s, g, P, b, x, cf, cvisc, r, partial);
    return (int)nb;
}

template <typename T>
int launch_resid_u(const Grid &g, const VelArrC<T> &b, const VelArr<T> &x, const CoefU<T> &cf, T mass, T cvisc,
                   const VelArr<T> &r, double *partial, hipStream_t s)
{
    VelBox parts;
    long long mx = 0;
    for (int a = 0; a < 3; ++a) {
        parts.b[a] = a < g.D ? unk_box(g, face_mask(a)) : Box{{0, 0, 0}, {0, 0, 0}};
        if (a < g.D && box_count(parts.b[a]) > mx) mx = box_count(parts.b[a]);
    }
    const unsigned nb = stride_blocks(mx);
    if (g.D == 3)
        launch_timed(k_resid_u<T, 3>, dim3(nb, 3), dim3(256), s, g, parts, b, x, cf, mass, cvisc, r, partial);
    else
        launch_timed(k_resid_u<T, 2>, dim3(nb, 2), dim3(256), s, g, parts, b, x, cf, mass, cvisc, r, partial);
    return (int)nb * g.D;
}

template <typename T>
int launch_norm2(const Grid &g, int ncomp, const int *vmasks, const VelArrC<T> &v, double *partial, hipStream_t s)
{
    VelBox boxes;
    long long mx = 0;
    for (int a = 0; a < 3; ++a) {
        boxes.b[a] = a < ncomp ? unk_box(g, vmasks[a]) : Box{{0, 0, 0}, {0, 0, 0}};
        if (a < ncomp && box_count(boxes.b[a]) > mx) mx = box_count(boxes.b[a]);
    }
    const unsigned nb = stride_blocks(mx);
    launch_timed(k_norm2<T>, dim3(nb, ncomp), dim3(256), s, boxes, g, v, partial);
    return (int)nb * ncomp;
}

void launch_reduce_final(const double *partial, long long n, double *out, hipStream_t s)
{
    launch_timed(k_reduce_final, dim3(1), dim3(256), s, partial, n, out);
}

static inline Box stored_box(const Grid &g, int vmask)
{
    Box b;
    for (int d = 0; d < 3; ++d) {
        b.lo[d] = 0;
        b.ext[d] = stored_extent(g, d, (vmask >> d) & 1);
    }
    return b;
}

template <typename T>
void launch_restrict(const Grid &gf, const Grid &gc, int ncomp, const int *vmasks, int role, bool all_stored,
                     const VelArrC<T> &fine, const VelArr<T> &coarse, T scale, hipStream_t s,
                     const VelArr<T> *zero_x)
{
    VelBox parts;
    int masks = 0;
    long long mx = 0;
    for (int a = 0; a < 3; ++a) {
        if (a < ncomp) {
            parts.b[a] = all_stored ? stored_box(gc, vmasks[a]) : unk_box(gc, vmasks[a]);
            masks |= vmasks[a] << (4 * a);
            mx = box_count(parts.b[a]) > mx ? box_count(parts.b[a]) : mx;
        } else {
            parts.b[a] = parts.b[0];
        }
    }
    const VelArr<T> zx = zero_x ? *zero_x : VelArr<T>{{nullptr, nullptr, nullptr}};
    if (mx <= 0) return;
    if (gf.D == 3)
        launch_timed(k_restrict<T, 3>, dim3(blocks_for(mx), ncomp), dim3(256), s, gf, gc, parts, masks, role, fine,
                     coarse, scale, zx);
    else
        launch_timed(k_restrict<T, 2>, dim3(blocks_for(mx), ncomp), dim3(256), s, gf, gc, parts, masks, role, fine,
                     coarse, scale, zx);
}

template <typename T>
void launch_prolong_add(const Grid &gc, const Grid &gf, int ncomp, const int *vmasks, int role,
                        const VelArrC<T> &coarse, const VelArr<T> &fine, hipStream_t s)
{
    VelBox parts;
    int masks = 0;
    long long mx = 0;
    for (int a = 0; a < 3; ++a) {
        if (a < ncomp) {
            parts.b[a] = unk_box(gf, vmasks[a]);
            masks |= vmasks[a] << (4 * a);
            mx = box_count(parts.b[a]) > mx ? box_count(parts.b[a]) : mx;
        } else {
            parts.b[a] = parts.b[0];
        }
    }
    if (mx <= 0) return;
    if (gf.D == 3)
        launch_timed(k_prolong_add<T, 3>, dim3(blocks_for(mx), ncomp), dim3(256), s, gc, gf, parts, masks, role,
                     coarse, fine);
    else
        launch_timed(k_prolong_add<T, 2>, dim3(blocks_for(mx), ncomp), dim3(256), s, gc, gf, parts, masks, role,
                     coarse, fine);
}

void launch_dense_inverse(const Grid &g, int velocity, int n, const long long *uidx, const int *ucomp,
                          const CoefP<double> &cp, const CoefU<double> &cu, double mass, double cvisc, double *tmp,
                          int singular, double *Aw, double *M, hipStream_t s)
{
    if (n <= 0 || n > DENSE_LDS) return;
    hipLaunchKernelGGL(k_dense_assemble, dim3(n), dim3(256), 0, s, g, velocity, n, uidx, ucomp, cp, cu, mass, cvisc,
                       tmp, Aw);
    hipLaunchKernelGGL(k_dense_gj, dim3(1), dim3(1024), 0, s, n, singular, Aw, M);
}

void launch_dense_gj(int n, int singular, const double *Aw, double *M, hipStream_t s)
{
    if (n <= 0 || n > DENSE_LDS) return;
    hipLaunchKernelGGL(k_dense_gj, dim3(1), dim3(1024), 0, s, n, singular, Aw, M);
}

template <typename T>
void launch_dense_apply(const Grid &g, int velocity, int n, const long long *uidx, const int *ucomp, const double *M,
                        const VelArrC<T> &b, const VelArr<T> &x, hipStream_t s)
{
    launch_timed(k_dense_apply<T>, dim3(1), dim3(64), s, g, velocity, n, uidx, ucomp, M, b, x);
}

template <typename T>
void launch_fill(T *p, long long n, T v, hipStream_t s)
{
    unsigned nb = blocks_for(n);
    if (nb > 2048) nb = 2048;
    if (nb == 0) nb = 1;
    launch_timed(k_fill<T>, dim3(nb), dim3(256), s, p, n, v);
}

template <typename Ts, typename Td>
void launch_cast_unknowns(const Grid &g, int ncomp, const int *vmasks, const VelArrC<Ts> &src, const VelArr<Td> &dst,
                          hipStream_t s)
{
    VelBox boxes;
    long long mx = 0;
    for (int a = 0; a < 3; ++a) {
        boxes.b[a] = a < ncomp ? unk_box(g, vmasks[a]) : Box{{0, 0, 0}, {0, 0, 0}};
        if (a < ncomp && box_count(boxes.b[a]) > mx) mx = box_count(boxes.b[a]);
    }
    launch_timed(k_cast_unknowns<Ts, Td>, dim3(blocks_for(mx), ncomp), dim3(256), s, g, boxes, src, dst);
}

void launch_inner_start(const Grid &g, int ncomp, const int *vmasks, const VelArrC<double> &r, const VelArr<float> &b32,
                        const VelArr<float> &x32, hipStream_t s)
{
    VelBox boxes;
    for (int a = 0; a < 3; ++a) boxes.b[a] = a < ncomp ? unk_box(g, vmasks[a]) : Box{{0, 0, 0}, {0, 0, 0}};
    launch_timed(k_inner_start, dim3(blocks_for(g.nel), ncomp), dim3(256), s, g, boxes, r, b32, x32);
}

void launch_add_correction(const Grid &g, int ncomp, const int *vmasks, const VelArrC<float> &e,
                           const VelArr<double> &x, hipStream_t s)
{
    const int velocity = vmasks[0] != 0 ? 1 : 0;
    VelBox boxes;
    long long mx = 0;
    for (int a = 0; a < 3; ++a) {
        boxes.b[a] = a < ncomp ? unk_box(g, vmasks[a]) : Box{{0, 0, 0}, {0, 0, 0}};
        if (a < ncomp && box_count(boxes.b[a]) > mx) mx = box_count(boxes.b[a]);
    }
    launch_timed(k_add_correction, dim3(blocks_for(mx), ncomp), dim3(256), s, g, boxes, velocity, e, x);
}

template <typename T>
void launch_load_unknowns(const Grid &g, int ncomp, const int *vmasks, const VelArrC<T> &src, const VelArr<T> &dst,
                          hipStream_t s)
{
    VelBox boxes;
    long long mx = 0;
    for (int a = 0; a < 3; ++a) {
        boxes.b[a] = a < ncomp ? unk_box(g, vmasks[a]) : Box{{0, 0, 0}, {0, 0, 0}};
        if (a < ncomp && box_count(boxes.b[a]) > mx) mx = box_count(boxes.b[a]);
    }
    const int velocity = vmasks[0] != 0 ? 1 : 0;
    launch_timed(k_load_unknowns<T>, dim3(blocks_for(mx), ncomp), dim3(256), s, g, boxes, velocity, src, dst);
}

template <typename T>
void launch_coef_ghosts(const Grid &g, const CoefSet<T> &set, hipStream_t s)
{
    long long mx = 0;
    for (int q = 0; q < set.n; ++q) mx = std::max(mx, box_count(stored_box(g, set.vmask[q])));
    if (set.n > 0 && mx > 0)
        hipLaunchKernelGGL(k_coef_ghosts<T>, dim3(blocks_for(mx), set.n), dim3(256), 0, s, g, set);
}

int wg_lds_budget()
{
    static int budget = -1;
    if (budget < 0) {
        int dev = 0, v = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) v = 65536;
        // the kernel's own shared data: the level table, the coarsest
        // right-hand side and the tail's right-hand side
        budget = v - (int)(WG_MAXLEV * sizeof(LevTab<double>)) - 1024 - (int)(TAIL_MAX * sizeof(double));
        if (budget < 0) budget = 0;
    }
    return budget;
}

// allow a dynamic arena above the default limit (once per kernel)
template <typename K>
static void allow_lds(K kernel, int bytes)
{
    static int allowed = 0;
    if (bytes > allowed) {
        if (hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                                bytes) == hipSuccess)
            allowed = bytes;
    }
}

// raise the dynamic-LDS limit of every one-workgroup kernel to the full
// budget once, so that no launch needs the attribute call (which has no
// place inside a captured graph)
void wg_prepare()
{
    const int b = wg_lds_budget();
#define PREP(T, DD, VV)                              \
    do {                                             \
        allow_lds(k_coarse_vcycle<T, DD, VV>, b);    \
        allow_lds(k_bcoarse<T, DD, VV>, b);          \
        allow_lds(k_tail_columns<T, DD, VV>, b);     \
    } while (0)
    PREP(double, 2, 0); PREP(double, 2, 1); PREP(double, 3, 0); PREP(double, 3, 1);
    PREP(float, 2, 0); PREP(float, 2, 1); PREP(float, 3, 0); PREP(float, 3, 1);
#undef PREP
}

template <typename T>
void launch_coarse_vcycle(int D, const LevTab<T> *tab, int l0, int L, int vel, int nu1, int nu2, int ndense,
                          const long long *uidx, const int *ucomp, const double *M, const LdsPlan &plan,
                          const Tail &tail, hipStream_t s)
{
#define LAUNCH(DD, VV)                                                                                              \
    do {                                                                                                            \
        allow_lds(k_coarse_vcycle<T, DD, VV>, plan.bytes);                                                          \
        launch_timed_shm(k_coarse_vcycle<T, DD, VV>, dim3(1), dim3(wg_threads(DD, VV)), plan.bytes, s, tab, l0, L, \
                         nu1, nu2, ndense, uidx, ucomp, M, plan, tail);                                             \
    } while (0)
    if (D == 3) {
        if (vel) LAUNCH(3, 1);
        else LAUNCH(3, 0);
    } else {
        if (vel) LAUNCH(2, 1);
        else LAUNCH(2, 0);
    }
#undef LAUNCH
}
template void launch_coarse_vcycle<double>(int, const LevTab<double> *, int, int, int, int, int, int,
                                           const long long *, const int *, const double *, const LdsPlan &,
                                           const Tail &, hipStream_t);
template void launch_coarse_vcycle<float>(int, const LevTab<float> *, int, int, int, int, int, int,
                                          const long long *, const int *, const double *, const LdsPlan &,
                                          const Tail &, hipStream_t);

template <typename T>
void launch_tail_columns(int D, const LevTab<T> *tab, int L, int vel, int nu1, int nu2, int ndense,
                         const long long *uidx, const int *ucomp, const double *M, const LdsPlan &plan,
                         const Tail &tail, hipStream_t s)
{
    if (tail.n <= 0) return;
#define LAUNCH(DD, VV)                                                                                              \
    do {                                                                                                            \
        allow_lds(k_tail_columns<T, DD, VV>, plan.bytes);                                                           \
        hipLaunchKernelGGL((k_tail_columns<T, DD, VV>), dim3(tail.n), dim3(wg_threads(DD, VV)), plan.bytes, s, tab, \
                           L, nu1, nu2, ndense, uidx, ucomp, M, plan, tail);                                         \
    } while (0)
    if (D == 3) {
        if (vel) LAUNCH(3, 1);
        else LAUNCH(3, 0);
    } else {
        if (vel) LAUNCH(2, 1);
        else LAUNCH(2, 0);
    }
#undef LAUNCH
}
template void launch_tail_columns<double>(int, const LevTab<double> *, int, int, int, int, int, const long long *,
                                          const int *, const double *, const LdsPlan &, const Tail &, hipStream_t);
template void launch_tail_columns<float>(int, const LevTab<float> *, int, int, int, int, int, const long long *,
                                         const int *, const double *, const LdsPlan &, const Tail &, hipStream_t);

int batch_blocks(int kind, const Grid &g, const Grid &gc, int vel, int A)
{
    const int nc = vel ? g.D : 1;
    long long mx = 0;
    switch (kind) {
    case BK_SWEEP: {
        const Box b = unk_box(g, vel ? face_mask(A) : 0);
        return (int)blocks_for((long long)((b.ext[0] + 1) / 2) * b.ext[1] * b.ext[2]);
    }
    case BK_RESID:
        for (int a = 0; a < nc; ++a) mx = std::max(mx, box_count(unk_box(g, vel ? face_mask(a) : 0)));
        return (int)stride_blocks(mx);
    case BK_RESTRICT:
        for (int a = 0; a < nc; ++a) mx = std::max(mx, box_count(unk_box(gc, vel ? face_mask(a) : 0)));
        return (int)blocks_for(mx);
    case BK_PROLONG:
    case BK_ADD:
        for (int a = 0; a < nc; ++a) mx = std::max(mx, box_count(unk_box(g, vel ? face_mask(a) : 0)));
        return (int)blocks_for(mx);
    case BK_PREP: return (int)blocks_for(g.nel);
    }
    return 0;
}

template <typename T>
void launch_bpass(int kind, int D, int vel, int A, int colour, const BEntry *ent, unsigned nblocks, const int *flags,
                  hipStream_t s)
{
    if (nblocks == 0) return;
    const dim3 blk(256);
    const dim3 gc(nblocks, vel ? D : 1);
#define PASS3(K, ...)                                                                                               \
    do {                                                                                                            \
        if (vel) hipLaunchKernelGGL((K<T, 3, 1>), gc, blk, 0, s, ent, flags);                                       \
        else hipLaunchKernelGGL((K<T, 3, 0>), gc, blk, 0, s, ent, flags);                                           \
    } while (0)
#define PASS2(K)                                                                                                    \
    do {                                                                                                            \
        if (vel) hipLaunchKernelGGL((K<T, 2, 1>), gc, blk, 0, s, ent, flags);                                       \
        else hipLaunchKernelGGL((K<T, 2, 0>), gc, blk, 0, s, ent, flags);                                           \
    } while (0)
    switch (kind) {
    case BK_SWEEP: {
        const dim3 g1(nblocks);
        if (D == 3) {
            if (!vel) hipLaunchKernelGGL((k_bsweep<T, 3, 0, 0>), g1, blk, 0, s, ent, flags, colour);
            else if (A == 0) hipLaunchKernelGGL((k_bsweep<T, 3, 1, 0>), g1, blk, 0, s, ent, flags, colour);
            else if (A == 1) hipLaunchKernelGGL((k_bsweep<T, 3, 1, 1>), g1, blk, 0, s, ent, flags, colour);
            else hipLaunchKernelGGL((k_bsweep<T, 3, 1, 2>), g1, blk, 0, s, ent, flags, colour);
        } else {
            if (!vel) hipLaunchKernelGGL((k_bsweep<T, 2, 0, 0>), g1, blk, 0, s, ent, flags, colour);
            else if (A == 0) hipLaunchKernelGGL((k_bsweep<T, 2, 1, 0>), g1, blk, 0, s, ent, flags, colour);
            else hipLaunchKernelGGL((k_bsweep<T, 2, 1, 1>), g1, blk, 0, s, ent, flags, colour);
        }
        break;
    }
    case BK_RESID:
        if (D == 3) PASS3(k_bresid);
        else PASS2(k_bresid);
        break;
    case BK_RESTRICT:
        if (D == 3) PASS3(k_brestrict);
        else PASS2(k_brestrict);
        break;
    case BK_PROLONG:
        if (D == 3) PASS3(k_bprolong);
        else PASS2(k_bprolong);
        break;
    case BK_PREP:
        if (vel) hipLaunchKernelGGL(k_bprep32<1>, dim3(nblocks), blk, 0, s, ent, flags);
        else hipLaunchKernelGGL(k_bprep32<0>, dim3(nblocks), blk, 0, s, ent, flags);
        break;
    case BK_ADD:
        if (vel) hipLaunchKernelGGL(k_badd<1>, gc, blk, 0, s, ent, flags);
        else hipLaunchKernelGGL(k_badd<0>, gc, blk, 0, s, ent, flags);
        break;
    }
#undef PASS3
#undef PASS2
}

void launch_breduce(const BEntry *ent, unsigned nitems, const int *flags, double *norms, hipStream_t s)
{
    if (nitems) hipLaunchKernelGGL(k_breduce, dim3(nitems), dim3(256), 0, s, ent, flags, norms);
}

template <typename T>
void launch_bcoarse(int D, int vel, const BCoarse *items, unsigned nitems, const int *flags, int nu1, int nu2,
                    int lds_bytes, hipStream_t s)
{
    if (nitems == 0) return;
    const dim3 g(nitems), b(wg_threads(D, vel));
#define LAUNCH(DD, VV)                                                                                              \
    do {                                                                                                            \
        allow_lds(k_bcoarse<T, DD, VV>, lds_bytes);                                                                 \
        hipLaunchKernelGGL((k_bcoarse<T, DD, VV>), g, b, lds_bytes, s, items, flags, nu1, nu2);                     \
    } while (0)
    if (D == 3) {
        if (vel) LAUNCH(3, 1);
        else LAUNCH(3, 0);
    } else {
        if (vel) LAUNCH(2, 1);
        else LAUNCH(2, 0);
    }
#undef LAUNCH
}
template void launch_bpass<double>(int, int, int, int, int, const BEntry *, unsigned, const int *, hipStream_t);
template void launch_bpass<float>(int, int, int, int, int, const BEntry *, unsigned, const int *, hipStream_t);
template void launch_bcoarse<double>(int, int, const BCoarse *, unsigned, const int *, int, int, int, hipStream_t);
template void launch_bcoarse<float>(int, int, const BCoarse *, unsigned, const int *, int, int, int, hipStream_t);

static VelBox unknown_boxes(const Grid &g, int velocity, long long &mx)
{
    VelBox boxes;
    mx = 0;
    const int nc = velocity ? g.D : 1;
    for (int a = 0; a < 3; ++a) {
        boxes.b[a] = a < nc ? unk_box(g, velocity ? face_mask(a) : 0) : Box{{0, 0, 0}, {0, 0, 0}};
        if (a < nc && box_count(boxes.b[a]) > mx) mx = box_count(boxes.b[a]);
    }
    return boxes;
}

void launch_apply(const Grid &g, int velocity, const VelArr<double> &z, const CoefP<double> &cp,
                  const CoefU<double> &cu, double mass, double cvisc, const VelArr<double> &q, hipStream_t s)
{
    long long mx;
    const VelBox boxes = unknown_boxes(g, velocity, mx);
    if (mx <= 0) return;
    if (velocity) {
        const dim3 grid(blocks_for(mx), g.D);
        if (g.D == 3) hipLaunchKernelGGL(k_apply_u<3>, grid, dim3(256), 0, s, g, boxes, z, cu, mass, cvisc, q);
        else hipLaunchKernelGGL(k_apply_u<2>, grid, dim3(256), 0, s, g, boxes, z, cu, mass, cvisc, q);
    } else {
        if (g.D == 3)
            hipLaunchKernelGGL(k_apply_p<3>, dim3(blocks_for(mx)), dim3(256), 0, s, g, boxes.b[0], z.c[0], cp, cvisc,
                               q.c[0]);
        else
            hipLaunchKernelGGL(k_apply_p<2>, dim3(blocks_for(mx)), dim3(256), 0, s, g, boxes.b[0], z.c[0], cp, cvisc,
                               q.c[0]);
    }
}

int launch_dot(const Grid &g, int velocity, const VelArrC<double> &x, const VelArrC<double> &y, double *partial,
               hipStream_t s)
{
    long long mx;
    const VelBox boxes = unknown_boxes(g, velocity, mx);
    const unsigned nb = stride_blocks(mx);
    const int nc = velocity ? g.D : 1;
    hipLaunchKernelGGL(k_dot, dim3(nb, nc), dim3(256), 0, s, boxes, g, x, y, partial);
    return (int)nb * nc;
}

void launch_gcr_axpy2(const Grid &g, int velocity, const double *num, const double *den, const VelArrC<double> &qi,
                      const VelArrC<double> &zi, const VelArr<double> &q, const VelArr<double> &z, hipStream_t s)
{
    long long mx;
    const VelBox boxes = unknown_boxes(g, velocity, mx);
    if (mx <= 0) return;
    hipLaunchKernelGGL(k_gcr_axpy2, dim3(blocks_for(mx), velocity ? g.D : 1), dim3(256), 0, s, g, boxes, num, den,
                       qi, zi, q, z);
}

void launch_gcr_update(const Grid &g, int velocity, const double *num, const double *den, const VelArrC<double> &z,
                       const VelArr<double> &x, hipStream_t s)
{
    long long mx;
    const VelBox boxes = unknown_boxes(g, velocity, mx);
    if (mx <= 0) return;
    hipLaunchKernelGGL(k_gcr_update, dim3(blocks_for(mx), velocity ? g.D : 1), dim3(256), 0, s, g, boxes, velocity,
                       num, den, z, x);
}

// explicit instantiations
#define INST(T)                                                                                                     \
    template void launch_smooth_p<T>(const Grid &, const T *, T *, const CoefP<T> &, T, int, hipStream_t, int);          \
    template void launch_smooth_u<T>(const Grid &, int, const T *, const VelArr<T> &, const CoefU<T> &, T, T, int,  \
                                     hipStream_t, int);                                                                  \
    template void launch_smooth_u_dec<T>(const Grid &, const VelArrC<T> &, const VelArr<T> &, const CoefU<T> &, T,  \
                                         T, int, hipStream_t);                                                      \
    template void launch_smooth_rb<T>(const Grid &, int, int, const VelArrC<T> &, const T *, const CoefU<T> &,      \
                                      const CoefP<T> &, T, T, T *, hipStream_t);                                    \
    template void launch_smooth_zm<T>(const Grid &, int, const VelArrC<T> &, const T *, const CoefU<T> &, T, T, T *, \
                                      hipStream_t);                                                                 \
    template int launch_resid_p<T>(const Grid &, const T *, const T *, const CoefP<T> &, T, T *, double *,          \
                                   hipStream_t);                                                                    \
    template int launch_resid_u<T>(const Grid &, const VelArrC<T> &, const VelArr<T> &, const CoefU<T> &, T, T,     \
                                   const VelArr<T> &, double *, hipStream_t);                                       \
    template int launch_norm2<T>(const Grid &, int, const int *, const VelArrC<T> &, double *, hipStream_t);        \
    template void launch_restrict<T>(const Grid &, const Grid &, int, const int *, int, bool, const VelArrC<T> &,   \
                                     const VelArr<T> &, T, hipStream_t, const VelArr<T> *);                         \
    template void launch_prolong_add<T>(const Grid &, const Grid &, int, const int *, int, const VelArrC<T> &,      \
                                        const VelArr<T> &, hipStream_t);                                            \
    template void launch_dense_apply<T>(const Grid &, int, int, const long long *, const int *, const double *,    \
                                        const VelArrC<T> &, const VelArr<T> &, hipStream_t);                        \
    template void launch_load_unknowns<T>(const Grid &, int, const int *, const VelArrC<T> &, const VelArr<T> &,    \
                                          hipStream_t);                                                             \
    template void launch_coef_ghosts<T>(const Grid &, const CoefSet<T> &, hipStream_t);                                       \
    template void launch_fill<T>(T *, long long, T, hipStream_t);
INST(double)
INST(float)
#undef INST
template void launch_cast_unknowns<double, float>(const Grid &, int, const int *, const VelArrC<double> &,
                                                  const VelArr<float> &, hipStream_t);
template void launch_cast_unknowns<float, double>(const Grid &, int, const int *, const VelArrC<float> &,
                                                  const VelArr<double> &, hipStream_t);
template void launch_cast_unknowns<double, double>(const Grid &, int, const int *, const VelArrC<double> &,
                                                   const VelArr<double> &, hipStream_t);
template void launch_fill<int>(int *, long long, int, hipStream_t);
template void launch_fill<unsigned char>(unsigned char *, long long, unsigned char, hipStream_t);

}  // namespace ibmg
