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
#include "common.h"
#include "kernels.h"

namespace ibmg {

// ---------------------------------------------------------------------------
// rows of the two operators: (A x) at one unknown and the diagonal entry
// ---------------------------------------------------------------------------
__device__ inline int self_sign(Ref r, long long c) { return (r.s != 0 && r.idx == c) ? r.s : 0; }

template <typename T>
__device__ inline void p_row_fast(const Grid &g, const T *__restrict__ x, const CoefP<T> &cf, T cvisc, long long c,
                                  T &Ax, T &dg)
{
    const T xc = x[c];
    T acc = 0, d = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (a >= g.D) break;
        const long long s = stride_of(g, a);
        const T bp = cf.beta[a][c + s], bm = cf.beta[a][c];
        acc += bp * (xc - x[c + s]) + bm * (xc - x[c - s]);
        d += bp + bm;
    }
    Ax = acc * cvisc;
    dg = d * cvisc;
}

template <typename T>
__device__ inline void p_row_slow(const Grid &g, const T *__restrict__ x, const CoefP<T> &cf, T cvisc, int i, int j,
                                  int k, T &Ax, T &dg)
{
    const long long c = at(g, i, j, k);
    const T xc = x[c];
    T acc = 0, d = 0;
    for (int a = 0; a < g.D; ++a) {
        int qp[3] = {i, j, k}, qm[3] = {i, j, k};
        qp[a] += 1;
        qm[a] -= 1;
        const T bp = load_ref(cf.beta[a], ref_at(g, face_mask(a), ROLE_C, qp[0], qp[1], qp[2]));
        const T bm = load_ref(cf.beta[a], ref_at(g, face_mask(a), ROLE_C, i, j, k));
        const Ref rp = ref_at(g, 0, ROLE_P, qp[0], qp[1], qp[2]);
        const Ref rm = ref_at(g, 0, ROLE_P, qm[0], qm[1], qm[2]);
        acc += bp * (xc - load_ref(x, rp)) + bm * (xc - load_ref(x, rm));
        d += bp * T(1 - self_sign(rp, c)) + bm * T(1 - self_sign(rm, c));
    }
    Ax = acc * cvisc;
    dg = d * cvisc;
}

template <typename T>
__device__ inline bool p_interior(const Grid &g, int i, int j, int k)
{
    const int q[3] = {i, j, k};
    for (int a = 0; a < g.D; ++a)
        if (q[a] < 1 || q[a] > g.n[a] - 2) return false;
    return true;
}

template <typename T>
__device__ inline void p_row(const Grid &g, const T *__restrict__ x, const CoefP<T> &cf, T cvisc, int i, int j, int k,
                             T &Ax, T &dg)
{
    if (p_interior<T>(g, i, j, k)) p_row_fast<T>(g, x, cf, cvisc, at(g, i, j, k), Ax, dg);
    else p_row_slow<T>(g, x, cf, cvisc, i, j, k, Ax, dg);
}

template <typename T>
__device__ inline void u_row_fast(const Grid &g, const VelArr<T> &x, const CoefU<T> &cf, T mass, T cvisc, int a,
                                  long long f, T &Ax, T &dg)
{
    const T *__restrict__ ua = x.c[a];
    const long long sa = stride_of(g, a);
    const T xf = ua[f];
    const T cp = T(2) * cf.muc[f], cm = T(2) * cf.muc[f - sa];
    T acc = cp * (ua[f + sa] - xf) - cm * (xf - ua[f - sa]);
    T d = cp + cm;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        if (b >= g.D) break;
        if (b == a) continue;
        const long long sb = stride_of(g, b);
        const T *__restrict__ ub = x.c[b];
        const T *__restrict__ me = cf.mue[3 - a - b];
        const T mp = me[f + sb], mm = me[f];
        acc += mp * ((ua[f + sb] - xf) + (ub[f + sb] - ub[f + sb - sa])) -
               mm * ((xf - ua[f - sb]) + (ub[f] - ub[f - sa]));
        d += mp + mm;
    }
    const T m = mass * cf.rho[a][f];
    Ax = m * xf - cvisc * acc;
    dg = m + cvisc * d;
}

template <typename T>
__device__ inline void u_row_slow(const Grid &g, const VelArr<T> &x, const CoefU<T> &cf, T mass, T cvisc, int a, int i,
                                  int j, int k, T &Ax, T &dg)
{
    const int q[3] = {i, j, k};
    const long long f = at(g, i, j, k);
    const T *__restrict__ ua = x.c[a];
    const int ma = face_mask(a);
    const T xf = ua[f];
    int qa_p[3] = {i, j, k}, qa_m[3] = {i, j, k};
    qa_p[a] += 1;
    qa_m[a] -= 1;
    // viscosity at the cells right (index q) and left (q - e_a) of the face
    const T cp = T(2) * load_ref(cf.muc, ref_at(g, 0, ROLE_C, i, j, k));
    const T cm = T(2) * load_ref(cf.muc, ref_at(g, 0, ROLE_C, qa_m[0], qa_m[1], qa_m[2]));
    const Ref rvp = ref_at(g, ma, ROLE_V, qa_p[0], qa_p[1], qa_p[2]);
    const Ref rvm = ref_at(g, ma, ROLE_V, qa_m[0], qa_m[1], qa_m[2]);
    T acc = cp * (load_ref(ua, rvp) - xf) - cm * (xf - load_ref(ua, rvm));
    T d = cp * T(1 - self_sign(rvp, f)) + cm * T(1 - self_sign(rvm, f));
    for (int b = 0; b < g.D; ++b) {
        if (b == a) continue;
        const int c = 3 - a - b;
        const int mb = face_mask(b), me_mask = edge_mask(g.D, c);
        const T *__restrict__ ub = x.c[b];
        const T *__restrict__ me = cf.mue[c];
        int qb_p[3] = {q[0], q[1], q[2]}, qb_m[3] = {q[0], q[1], q[2]};
        qb_p[b] += 1;
        qb_m[b] -= 1;
        int qbp_am[3] = {qb_p[0], qb_p[1], qb_p[2]};
        qbp_am[a] -= 1;
        // edges above (q + e_b) and below (q) along b
        const T mp = load_ref(me, ref_at(g, me_mask, ROLE_C, qb_p[0], qb_p[1], qb_p[2]));
        const T mm = load_ref(me, ref_at(g, me_mask, ROLE_C, i, j, k));
        const Ref rap = ref_at(g, ma, ROLE_V, qb_p[0], qb_p[1], qb_p[2]);
        const Ref ram = ref_at(g, ma, ROLE_V, qb_m[0], qb_m[1], qb_m[2]);
        const T ubpp = load_ref(ub, ref_at(g, mb, ROLE_V, qb_p[0], qb_p[1], qb_p[2]));
        const T ubpm = load_ref(ub, ref_at(g, mb, ROLE_V, qbp_am[0], qbp_am[1], qbp_am[2]));
        const T ub0p = load_ref(ub, ref_at(g, mb, ROLE_V, i, j, k));
        const T ub0m = load_ref(ub, ref_at(g, mb, ROLE_V, qa_m[0], qa_m[1], qa_m[2]));
        acc += mp * ((load_ref(ua, rap) - xf) + (ubpp - ubpm)) - mm * ((xf - load_ref(ua, ram)) + (ub0p - ub0m));
        d += mp * T(1 - self_sign(rap, f)) + mm * T(1 - self_sign(ram, f));
    }
    const T m = mass * cf.rho[a][f];
    Ax = m * xf - cvisc * acc;
    dg = m + cvisc * d;
}

__device__ inline bool u_interior(const Grid &g, int i, int j, int k)
{
    const int q[3] = {i, j, k};
    for (int a = 0; a < g.D; ++a)
        if (q[a] < 2 || q[a] > g.n[a] - 2) return false;
    return true;
}

template <typename T>
__device__ inline void u_row(const Grid &g, const VelArr<T> &x, const CoefU<T> &cf, T mass, T cvisc, int a, int i,
                             int j, int k, T &Ax, T &dg)
{
    if (u_interior(g, i, j, k)) u_row_fast<T>(g, x, cf, mass, cvisc, a, at(g, i, j, k), Ax, dg);
    else u_row_slow<T>(g, x, cf, mass, cvisc, a, i, j, k, Ax, dg);
}

// ---------------------------------------------------------------------------
// index helpers: unknown boxes and their colour classes
// ---------------------------------------------------------------------------
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

__device__ inline bool box_pos(const Box &b, long long t, int &i, int &j, int &k)
{
    const long long n = (long long)b.ext[0] * b.ext[1] * b.ext[2];
    if (t >= n) return false;
    i = b.lo[0] + (int)(t % b.ext[0]);
    t /= b.ext[0];
    j = b.lo[1] + (int)(t % b.ext[1]);
    k = b.lo[2] + (int)(t / b.ext[1]);
    return true;
}

// t-th point of colour `colour` ((i + j + k) mod 2) in the box
__device__ inline bool box_colour_pos(const Box &b, int colour, long long t, int &i, int &j, int &k)
{
    const int half = (b.ext[0] + 1) >> 1;
    const long long n = (long long)half * b.ext[1] * b.ext[2];
    if (t >= n) return false;
    const int ih = (int)(t % half);
    t /= half;
    j = b.lo[1] + (int)(t % b.ext[1]);
    k = b.lo[2] + (int)(t / b.ext[1]);
    i = b.lo[0] + 2 * ih + ((b.lo[0] + j + k + colour) & 1);
    return i < b.lo[0] + b.ext[0];
}

// ---------------------------------------------------------------------------
// smoothers
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_smooth_p(Grid g, Box box, const T *__restrict__ b, T *x, CoefP<T> cf, T cvisc,
                                                  int colour)
{
    int i, j, k;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (!box_colour_pos(box, colour, t, i, j, k)) return;
    T Ax, dg;
    p_row<T>(g, x, cf, cvisc, i, j, k, Ax, dg);
    const long long c = at(g, i, j, k);
    x[c] += (b[c] - Ax) / dg;
}

template <typename T>
__global__ void __launch_bounds__(256) k_smooth_u(Grid g, Box box, int a, const T *__restrict__ b, VelArr<T> x,
                                                  CoefU<T> cf, T mass, T cvisc, int colour)
{
    int i, j, k;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (!box_colour_pos(box, colour, t, i, j, k)) return;
    T Ax, dg;
    u_row<T>(g, x, cf, mass, cvisc, a, i, j, k, Ax, dg);
    const long long f = at(g, i, j, k);
    x.c[a][f] += (b[f] - Ax) / dg;
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
template <typename T>
__global__ void __launch_bounds__(256) k_resid_p(Grid g, Box box, const T *__restrict__ b, const T *__restrict__ x,
                                                 CoefP<T> cf, T cvisc, T *r, double *partial)
{
    const long long n = (long long)box.ext[0] * box.ext[1] * box.ext[2];
    double acc = 0.0;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        box_pos(box, t, i, j, k);
        T Ax, dg;
        p_row<T>(g, x, cf, cvisc, i, j, k, Ax, dg);
        const long long c = at(g, i, j, k);
        const T rv = b[c] - Ax;
        if (r) r[c] = rv;
        acc += (double)rv * (double)rv;
    }
    if (partial) block_sum_store(acc, partial, blockIdx.x);
}

template <typename T>
__global__ void __launch_bounds__(256) k_resid_u(Grid g, VelBox boxes, VelArrC<T> b, VelArr<T> x, CoefU<T> cf, T mass,
                                                 T cvisc, VelArr<T> r, double *partial)
{
    const int a = blockIdx.y;
    const Box box = boxes.b[a];
    const long long n = (long long)box.ext[0] * box.ext[1] * box.ext[2];
    double acc = 0.0;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        box_pos(box, t, i, j, k);
        T Ax, dg;
        u_row<T>(g, x, cf, mass, cvisc, a, i, j, k, Ax, dg);
        const long long f = at(g, i, j, k);
        const T rv = b.c[a][f] - Ax;
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
    const long long n = (long long)box.ext[0] * box.ext[1] * box.ext[2];
    double acc = 0.0;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x) {
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
__device__ inline int rst_weights(int vert, int I, int *fq, double *w)
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

__device__ inline int prl_weights(int vert, int f, int *cq, double *w)
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

// coarse[c] = full-weighting restriction of fine[c] at every coarse unknown
// (or every stored coarse position when `all_stored`, for coefficients)
template <typename T>
__global__ void __launch_bounds__(256) k_restrict(Grid gf, Grid gc, VelBox cboxes, int masks, int role, VelArrC<T> fine,
                                                  VelArr<T> coarse, T scale)
{
    const int comp = blockIdx.y;
    const int vmask = (masks >> (4 * comp)) & 0xF;
    const Box box = cboxes.b[comp];
    int I, J, K;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (!box_pos(box, t, I, J, K)) return;
    const int Q[3] = {I, J, K};
    int fq[3][4];
    double w[3][4];
    int nf[3];
    bool direct = true;
    for (int d = 0; d < 3; ++d) {
        if (d >= gf.D) { fq[d][0] = 0; w[d][0] = 1.0; nf[d] = 1; continue; }
        const int vert = (vmask >> d) & 1;
        nf[d] = rst_weights(vert, Q[d], fq[d], w[d]);
        int lo, hi;
        if (role == ROLE_C) { lo = 0; hi = stored_extent(gf, d, vert) - 1; }
        else unk_range(gf, d, vert, lo, hi);
        if (fq[d][0] < lo || fq[d][nf[d] - 1] > hi) direct = false;
    }
    const T *__restrict__ src = fine.c[comp];
    double s = 0.0;
    for (int c = 0; c < nf[2]; ++c)
        for (int b = 0; b < nf[1]; ++b) {
            const double wbc = w[1][b] * w[2][c];
            for (int a = 0; a < nf[0]; ++a) {
                double v;
                if (direct) v = (double)src[at(gf, fq[0][a], fq[1][b], fq[2][c])];
                else v = (double)load_ref(src, ref_at(gf, vmask, role, fq[0][a], fq[1][b], fq[2][c]));
                s += w[0][a] * wbc * v;
            }
        }
    coarse.c[comp][at(gc, I, J, K)] = (T)(s * (double)scale);
}

// fine[c] += linear interpolation of coarse[c] at every fine unknown
template <typename T>
__global__ void __launch_bounds__(256) k_prolong_add(Grid gc, Grid gf, VelBox fboxes, int masks, int role,
                                                     VelArrC<T> coarse, VelArr<T> fine)
{
    const int comp = blockIdx.y;
    const int vmask = (masks >> (4 * comp)) & 0xF;
    const Box box = fboxes.b[comp];
    int i, j, k;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (!box_pos(box, t, i, j, k)) return;
    const int q[3] = {i, j, k};
    int cq[3][2];
    double w[3][2];
    int nc[3];
    for (int d = 0; d < 3; ++d) {
        if (d >= gf.D) { cq[d][0] = 0; w[d][0] = 1.0; nc[d] = 1; continue; }
        nc[d] = prl_weights((vmask >> d) & 1, q[d], cq[d], w[d]);
    }
    const T *__restrict__ src = coarse.c[comp];
    double s = 0.0;
    for (int c = 0; c < nc[2]; ++c)
        for (int b = 0; b < nc[1]; ++b)
            for (int a = 0; a < nc[0]; ++a)
                s += w[0][a] * w[1][b] * w[2][c] *
                     (double)load_ref(src, ref_at(gc, vmask, role, cq[0][a], cq[1][b], cq[2][c]));
    fine.c[comp][at(gf, i, j, k)] += (T)s;
}

// ---------------------------------------------------------------------------
// coarsest level: dense inverse, assembled by applying the stencil to unit
// vectors, inverted by Gauss-Jordan with partial pivoting (one workgroup)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_dense_inverse(Grid g, int velocity, int n, const long long *__restrict__ uidx,
                                                      const int *__restrict__ ucomp, CoefP<double> cp,
                                                      CoefU<double> cu, double mass, double cvisc, VelArr<double> tmp,
                                                      int singular, double *Aw, double *M)
{
    const int r = threadIdx.x;
    // assemble A column by column into Aw (row-major n x n)
    for (int j = 0; j < n; ++j) {
        for (long long e = r; e < g.nel; e += blockDim.x)
            for (int c = 0; c < (velocity ? g.D : 1); ++c) tmp.c[c][e] = 0.0;
        __syncthreads();
        if (r == 0) tmp.c[velocity ? ucomp[j] : 0][uidx[j]] = 1.0;
        __syncthreads();
        if (r < n) {
            const long long e = uidx[r];
            const int k = (int)(e / g.NXY), jj = (int)((e % g.NXY) / g.NX), i = (int)(e % g.NX);
            double Ax, dg;
            if (velocity) u_row_slow<double>(g, tmp, cu, mass, cvisc, ucomp[r], i, jj, k, Ax, dg);
            else p_row_slow<double>(g, tmp.c[0], cp, cvisc, i, jj, k, Ax, dg);
            Aw[r * n + j] = Ax;
        }
        __syncthreads();
    }
    // singular (all-Neumann/periodic pressure): add alpha 1 1^T, alpha = trace / n^2
    if (singular) {
        __shared__ double tr;
        if (r == 0) {
            double s = 0.0;
            for (int i = 0; i < n; ++i) s += Aw[i * n + i];
            tr = s / ((double)n * (double)n);
        }
        __syncthreads();
        if (r < n)
            for (int j = 0; j < n; ++j) Aw[r * n + j] += tr;
        __syncthreads();
    }
    if (r < n)
        for (int j = 0; j < n; ++j) M[r * n + j] = (r == j) ? 1.0 : 0.0;
    __syncthreads();
    __shared__ int piv;
    for (int kcol = 0; kcol < n; ++kcol) {
        if (r == 0) {
            int p = kcol;
            for (int i = kcol + 1; i < n; ++i)
                if (fabs(Aw[i * n + kcol]) > fabs(Aw[p * n + kcol])) p = i;
            piv = p;
        }
        __syncthreads();
        const int p = piv;
        if (p != kcol && r < n) {
            double t = Aw[kcol * n + r]; Aw[kcol * n + r] = Aw[p * n + r]; Aw[p * n + r] = t;
            t = M[kcol * n + r]; M[kcol * n + r] = M[p * n + r]; M[p * n + r] = t;
        }
        __syncthreads();
        const double pv = Aw[kcol * n + kcol];
        __syncthreads();
        if (r < n) {
            Aw[kcol * n + r] /= pv;
            M[kcol * n + r] /= pv;
        }
        __syncthreads();
        if (r < n && r != kcol) {
            const double f = Aw[r * n + kcol];
            for (int j = 0; j < n; ++j) {
                Aw[r * n + j] -= f * Aw[kcol * n + j];
                M[r * n + j] -= f * M[kcol * n + j];
            }
        }
        __syncthreads();
    }
}

// x = M b over the coarsest unknowns (M in FP64)
template <typename T>
__global__ void __launch_bounds__(64) k_dense_apply(int n, const long long *__restrict__ uidx,
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
        x.c[ucomp[r]][uidx[r]] = (T)s;
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

// x(unknowns) += (double) e(unknowns)
__global__ void __launch_bounds__(256) k_add_correction(Grid g, VelBox boxes, VelArrC<float> e, VelArr<double> x)
{
    const int a = blockIdx.y;
    int i, j, k;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (!box_pos(boxes.b[a], t, i, j, k)) return;
    const long long q = at(g, i, j, k);
    x.c[a][q] += (double)e.c[a][q];
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(long long n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }
static inline long long box_count(const Box &b) { return (long long)b.ext[0] * b.ext[1] * b.ext[2]; }

template <typename T>
void launch_smooth_p(const Grid &g, const T *b, T *x, const CoefP<T> &cf, T cvisc, int colour, hipStream_t s)
{
    const Box box = unk_box(g, 0);
    const long long n = (long long)((box.ext[0] + 1) / 2) * box.ext[1] * box.ext[2];
    hipLaunchKernelGGL(k_smooth_p<T>, dim3(blocks_for(n)), dim3(256), 0, s, g, box, b, x, cf, cvisc, colour);
}

template <typename T>
void launch_smooth_u(const Grid &g, int a, const T *b, const VelArr<T> &x, const CoefU<T> &cf, T mass, T cvisc,
                     int colour, hipStream_t s)
{
    const Box box = unk_box(g, face_mask(a));
    const long long n = (long long)((box.ext[0] + 1) / 2) * box.ext[1] * box.ext[2];
    hipLaunchKernelGGL(k_smooth_u<T>, dim3(blocks_for(n)), dim3(256), 0, s, g, box, a, b, x, cf, mass, cvisc, colour);
}

static inline unsigned stride_blocks(long long n)
{
    unsigned b = blocks_for(n);
    return b < NORM_BLOCKS ? (b ? b : 1) : NORM_BLOCKS;
}

template <typename T>
int launch_resid_p(const Grid &g, const T *b, const T *x, const CoefP<T> &cf, T cvisc, T *r, double *partial,
                   hipStream_t s)
{
    const Box box = unk_box(g, 0);
    const unsigned nb = stride_blocks(box_count(box));
    hipLaunchKernelGGL(k_resid_p<T>, dim3(nb), dim3(256), 0, s, g, box, b, x, cf, cvisc, r, partial);
    return (int)nb;
}

template <typename T>
int launch_resid_u(const Grid &g, const VelArrC<T> &b, const VelArr<T> &x, const CoefU<T> &cf, T mass, T cvisc,
                   const VelArr<T> &r, double *partial, hipStream_t s)
{
    VelBox boxes;
    long long mx = 0;
    for (int a = 0; a < 3; ++a) {
        boxes.b[a] = a < g.D ? unk_box(g, face_mask(a)) : Box{{0, 0, 0}, {0, 0, 0}};
        if (a < g.D && box_count(boxes.b[a]) > mx) mx = box_count(boxes.b[a]);
    }
    const unsigned nb = stride_blocks(mx);
    hipLaunchKernelGGL(k_resid_u<T>, dim3(nb, g.D), dim3(256), 0, s, g, boxes, b, x, cf, mass, cvisc, r, partial);
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
    hipLaunchKernelGGL(k_norm2<T>, dim3(nb, ncomp), dim3(256), 0, s, boxes, g, v, partial);
    return (int)nb * ncomp;
}

void launch_reduce_final(const double *partial, long long n, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, s, partial, n, out);
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
                     const VelArrC<T> &fine, const VelArr<T> &coarse, T scale, hipStream_t s)
{
    VelBox boxes;
    int masks = 0;
    long long mx = 0;
    for (int a = 0; a < 3; ++a) {
        if (a < ncomp) {
            boxes.b[a] = all_stored ? stored_box(gc, vmasks[a]) : unk_box(gc, vmasks[a]);
            masks |= vmasks[a] << (4 * a);
            mx = box_count(boxes.b[a]) > mx ? box_count(boxes.b[a]) : mx;
        } else {
            boxes.b[a] = Box{{0, 0, 0}, {0, 0, 0}};
        }
    }
    hipLaunchKernelGGL(k_restrict<T>, dim3(blocks_for(mx), ncomp), dim3(256), 0, s, gf, gc, boxes, masks, role, fine,
                       coarse, scale);
}

template <typename T>
void launch_prolong_add(const Grid &gc, const Grid &gf, int ncomp, const int *vmasks, int role,
                        const VelArrC<T> &coarse, const VelArr<T> &fine, hipStream_t s)
{
    VelBox boxes;
    int masks = 0;
    long long mx = 0;
    for (int a = 0; a < 3; ++a) {
        if (a < ncomp) {
            boxes.b[a] = unk_box(gf, vmasks[a]);
            masks |= vmasks[a] << (4 * a);
            mx = box_count(boxes.b[a]) > mx ? box_count(boxes.b[a]) : mx;
        } else {
            boxes.b[a] = Box{{0, 0, 0}, {0, 0, 0}};
        }
    }
    hipLaunchKernelGGL(k_prolong_add<T>, dim3(blocks_for(mx), ncomp), dim3(256), 0, s, gc, gf, boxes, masks, role,
                       coarse, fine);
}

void launch_dense_inverse(const Grid &g, int velocity, int n, const long long *uidx, const int *ucomp,
                          const CoefP<double> &cp, const CoefU<double> &cu, double mass, double cvisc,
                          const VelArr<double> &tmp, int singular, double *Aw, double *M, hipStream_t s)
{
    hipLaunchKernelGGL(k_dense_inverse, dim3(1), dim3(64), 0, s, g, velocity, n, uidx, ucomp, cp, cu, mass, cvisc, tmp,
                       singular, Aw, M);
}

template <typename T>
void launch_dense_apply(int n, const long long *uidx, const int *ucomp, const double *M, const VelArrC<T> &b,
                        const VelArr<T> &x, hipStream_t s)
{
    hipLaunchKernelGGL(k_dense_apply<T>, dim3(1), dim3(64), 0, s, n, uidx, ucomp, M, b, x);
}

template <typename T>
void launch_fill(T *p, long long n, T v, hipStream_t s)
{
    unsigned nb = blocks_for(n);
    if (nb > 2048) nb = 2048;
    if (nb == 0) nb = 1;
    hipLaunchKernelGGL(k_fill<T>, dim3(nb), dim3(256), 0, s, p, n, v);
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
    hipLaunchKernelGGL((k_cast_unknowns<Ts, Td>), dim3(blocks_for(mx), ncomp), dim3(256), 0, s, g, boxes, src, dst);
}

void launch_add_correction(const Grid &g, int ncomp, const int *vmasks, const VelArrC<float> &e,
                           const VelArr<double> &x, hipStream_t s)
{
    VelBox boxes;
    long long mx = 0;
    for (int a = 0; a < 3; ++a) {
        boxes.b[a] = a < ncomp ? unk_box(g, vmasks[a]) : Box{{0, 0, 0}, {0, 0, 0}};
        if (a < ncomp && box_count(boxes.b[a]) > mx) mx = box_count(boxes.b[a]);
    }
    hipLaunchKernelGGL(k_add_correction, dim3(blocks_for(mx), ncomp), dim3(256), 0, s, g, boxes, e, x);
}

// explicit instantiations
#define INST(T)                                                                                                     \
    template void launch_smooth_p<T>(const Grid &, const T *, T *, const CoefP<T> &, T, int, hipStream_t);          \
    template void launch_smooth_u<T>(const Grid &, int, const T *, const VelArr<T> &, const CoefU<T> &, T, T, int,  \
                                     hipStream_t);                                                                  \
    template int launch_resid_p<T>(const Grid &, const T *, const T *, const CoefP<T> &, T, T *, double *,          \
                                   hipStream_t);                                                                    \
    template int launch_resid_u<T>(const Grid &, const VelArrC<T> &, const VelArr<T> &, const CoefU<T> &, T, T,     \
                                   const VelArr<T> &, double *, hipStream_t);                                       \
    template int launch_norm2<T>(const Grid &, int, const int *, const VelArrC<T> &, double *, hipStream_t);        \
    template void launch_restrict<T>(const Grid &, const Grid &, int, const int *, int, bool, const VelArrC<T> &,   \
                                     const VelArr<T> &, T, hipStream_t);                                            \
    template void launch_prolong_add<T>(const Grid &, const Grid &, int, const int *, int, const VelArrC<T> &,      \
                                        const VelArr<T> &, hipStream_t);                                            \
    template void launch_dense_apply<T>(int, const long long *, const int *, const double *, const VelArrC<T> &,    \
                                        const VelArr<T> &, hipStream_t);                                            \
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
