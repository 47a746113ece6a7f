// Finest-level field kernels of the projection step: the momentum
// right-hand side of eq:NSdis1-1 (skew-symmetric advection, force, body
// force, fixed boundary values moved to the right), the pressure right-hand
// side of eq:NSdis4, the projection of eq:NSdis2, and the layout
// conversions between the compact exchange layout and the uniform
// per-level arrays.
#include "common.h"
#include "kernels.h"

namespace ibmg {

static inline unsigned nblk(long long n) { return (unsigned)((n + 255) / 256); }

__device__ inline bool box_at(const int ext[3], long long t, int &i, int &j, int &k)
{
    const long long n = (long long)ext[0] * ext[1] * ext[2];
    if (t >= n) return false;
    i = (int)(t % ext[0]);
    t /= ext[0];
    j = (int)(t % ext[1]);
    k = (int)(t / ext[1]);
    return true;
}

// ---------------------------------------------------------------------------
// layouts
// ---------------------------------------------------------------------------
__global__ void k_layout(Grid g, int vmask, const double *__restrict__ src, double *__restrict__ dst, int to_uniform)
{
    int ext[3];
    for (int d = 0; d < 3; ++d) ext[d] = stored_extent(g, d, (vmask >> d) & 1);
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int i, j, k;
    if (!box_at(ext, t, i, j, k)) return;
    const long long u = at(g, i, j, k);
    if (to_uniform) dst[u] = src[t];
    else dst[t] = src[u];
}

void launch_layout(const Grid &g, int vmask, const double *src, double *dst, bool to_uniform, hipStream_t s)
{
    long long n = 1;
    for (int d = 0; d < 3; ++d) n *= stored_extent(g, d, (vmask >> d) & 1);
    hipLaunchKernelGGL(k_layout, dim3(nblk(n)), dim3(256), 0, s, g, vmask, src, dst, to_uniform ? 1 : 0);
}

// ---------------------------------------------------------------------------
// the full velocity field (fixed boundary values kept)
// ---------------------------------------------------------------------------
// Component b of the velocity at lattice index (i, j, k), one layer beyond
// the domain allowed.  Along the cell-centred axes the tangential rules
// apply (odd across walls and the inflow plane, even across the outflow
// plane, wrap when periodic).  Along b itself the stored faces hold the
// boundary values; one layer beyond a fixed face is the odd reflection
// through the face value (2 v(face) - v(inside)), one layer beyond the
// outflow face mirrors evenly.  With bd_only the unknown faces read as zero,
// leaving only the boundary data.
__device__ double vfull(const Grid &g, const double *__restrict__ ub, int b, int i, int j, int k, bool bd_only)
{
    int q[3] = {i, j, k};
    int s = 1;
    for (int d = 0; d < g.D; ++d)
        if (d != b) resolve(g, d, 0, ROLE_V, q[d], s);
    const int n = g.n[b];
    int lo, hi;
    unk_range(g, b, 1, lo, hi);
    auto V = [&](int t) -> double {
        if (bd_only && t >= lo && t <= hi) return 0.0;
        int r[3] = {q[0], q[1], q[2]};
        r[b] = t;
        return ub[at(g, r[0], r[1], r[2])];
    };
    int t = q[b];
    double v;
    if (g.bc[b] == AX_PERIODIC) {
        if (t < 0) t += n;
        else if (t >= n) t -= n;
        v = V(t);
    } else if (t < 0) {
        v = 2.0 * V(0) - V(1);
    } else if (t > n) {
        v = g.bc[b] == AX_WALLS ? 2.0 * V(n) - V(n - 1) : V(n - 1);
    } else {
        v = V(t);
    }
    return s > 0 ? v : -v;
}

// u_b averaged to an a-face position p: the four surrounding b-faces
__device__ inline double ubar(const Grid &g, const VelArrC<double> &u, int a, int b, int i, int j, int k)
{
    if (b == a) return vfull(g, u.c[a], a, i, j, k, false);
    int q1[3] = {i, j, k};
    int q2[3] = {i, j, k};
    q2[b] += 1;
    int q3[3] = {i, j, k};
    q3[a] -= 1;
    int q4[3] = {q2[0], q2[1], q2[2]};
    q4[a] -= 1;
    return 0.25 * (vfull(g, u.c[b], b, q1[0], q1[1], q1[2], false) + vfull(g, u.c[b], b, q2[0], q2[1], q2[2], false) +
                   vfull(g, u.c[b], b, q3[0], q3[1], q3[2], false) + vfull(g, u.c[b], b, q4[0], q4[1], q4[2], false));
}

// b_a = rho_a (sigma u_a / dt - N_a(u)) + C_f f_a + g_a + Re^-1 V(u_bd)_a
// at every unknown a-face, N_a = 1/2 sum_b [ub_b D0_b u_a + D0_b (ub_b u_a)]
__global__ void __launch_bounds__(256) k_momentum_rhs(Grid g, Phys ph, VelArrC<double> u, CoefU<double> cf,
                                                      VelArrC<double> f, VelArr<double> bout, VelBox boxes)
{
    const int a = blockIdx.y;
    const Box box = boxes.b[a];
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n = (long long)box.ext[0] * box.ext[1] * box.ext[2];
    if (t >= n) return;
    const int i = box.lo[0] + (int)(t % box.ext[0]);
    t /= box.ext[0];
    const int j = box.lo[1] + (int)(t % box.ext[1]);
    const int k = box.lo[2] + (int)(t / box.ext[1]);
    const int q[3] = {i, j, k};
    const double h = g.h;
    // advection
    double N = 0.0;
    for (int b = 0; b < g.D; ++b) {
        int qp[3] = {i, j, k}, qm[3] = {i, j, k};
        qp[b] += 1;
        qm[b] -= 1;
        const double uap = vfull(g, u.c[a], a, qp[0], qp[1], qp[2], false);
        const double uam = vfull(g, u.c[a], a, qm[0], qm[1], qm[2], false);
        const double bc = ubar(g, u, a, b, i, j, k);
        const double bp = ubar(g, u, a, b, qp[0], qp[1], qp[2]);
        const double bm = ubar(g, u, a, b, qm[0], qm[1], qm[2]);
        N += bc * (uap - uam) / (2.0 * h) + (bp * uap - bm * uam) / (2.0 * h);
    }
    N *= 0.5;
    // viscous stencil applied to the boundary data alone
    int qa_p[3] = {i, j, k}, qa_m[3] = {i, j, k};
    qa_p[a] += 1;
    qa_m[a] -= 1;
    const double cp = 2.0 * load_ref(cf.muc, ref_at(g, 0, ROLE_C, i, j, k));
    const double cm = 2.0 * load_ref(cf.muc, ref_at(g, 0, ROLE_C, qa_m[0], qa_m[1], qa_m[2]));
    const double x0 = vfull(g, u.c[a], a, i, j, k, true);
    double acc = cp * (vfull(g, u.c[a], a, qa_p[0], qa_p[1], qa_p[2], true) - x0) -
                 cm * (x0 - vfull(g, u.c[a], a, qa_m[0], qa_m[1], qa_m[2], true));
    for (int b = 0; b < g.D; ++b) {
        if (b == a) continue;
        const int c = 3 - a - b;
        int qb_p[3] = {q[0], q[1], q[2]}, qb_m[3] = {q[0], q[1], q[2]};
        qb_p[b] += 1;
        qb_m[b] -= 1;
        int qbp_am[3] = {qb_p[0], qb_p[1], qb_p[2]};
        qbp_am[a] -= 1;
        const double mp = load_ref(cf.mue[c], ref_at(g, edge_mask(g.D, c), ROLE_C, qb_p[0], qb_p[1], qb_p[2]));
        const double mm = load_ref(cf.mue[c], ref_at(g, edge_mask(g.D, c), ROLE_C, i, j, k));
        acc += mp * ((vfull(g, u.c[a], a, qb_p[0], qb_p[1], qb_p[2], true) - x0) +
                     (vfull(g, u.c[b], b, qb_p[0], qb_p[1], qb_p[2], true) -
                      vfull(g, u.c[b], b, qbp_am[0], qbp_am[1], qbp_am[2], true))) -
               mm * ((x0 - vfull(g, u.c[a], a, qb_m[0], qb_m[1], qb_m[2], true)) +
                     (vfull(g, u.c[b], b, i, j, k, true) - vfull(g, u.c[b], b, qa_m[0], qa_m[1], qa_m[2], true)));
    }
    const long long e = at(g, i, j, k);
    const double rho = cf.rho[a][e];
    bout.c[a][e] = rho * (ph.sigma * u.c[a][e] / ph.dt - N) + ph.force_coef * f.c[a][e] + ph.body_force[a] +
                   ph.inv_re * (acc / (h * h));
}

void launch_momentum_rhs(const Grid &g, const Phys &ph, const VelArrC<double> &u, const CoefU<double> &cf,
                         const VelArrC<double> &f, const VelArr<double> &b, hipStream_t s)
{
    VelBox boxes;
    long long mx = 0;
    for (int a = 0; a < 3; ++a) {
        Box bx{{0, 0, 0}, {0, 0, 0}};
        if (a < g.D) {
            for (int d = 0; d < 3; ++d) {
                int lo, hi;
                unk_range(g, d, d == a, lo, hi);
                bx.lo[d] = lo;
                bx.ext[d] = hi - lo + 1;
            }
            const long long n = (long long)bx.ext[0] * bx.ext[1] * bx.ext[2];
            mx = n > mx ? n : mx;
        }
        boxes.b[a] = bx;
    }
    hipLaunchKernelGGL(k_momentum_rhs, dim3(nblk(mx), g.D), dim3(256), 0, s, g, ph, u, cf, f, b, boxes);
}

// b_p = -(sigma / (eps dt)) D u~ at every cell: unknown faces from ut, fixed
// faces (walls, inflow) from ubd, periodic faces wrap
__global__ void __launch_bounds__(256) k_pressure_div(Grid g, double coef, VelArrC<double> ut, VelArrC<double> ubd,
                                                      double *bp)
{
    const int ext[3] = {g.n[0], g.n[1], g.D == 3 ? g.n[2] : 1};
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int i, j, k;
    if (!box_at(ext, t, i, j, k)) return;
    const int q[3] = {i, j, k};
    double div = 0.0;
    for (int a = 0; a < g.D; ++a) {
        int qp[3] = {i, j, k};
        qp[a] += 1;
        if (g.bc[a] == AX_PERIODIC && qp[a] == g.n[a]) qp[a] = 0;
        int lo, hi;
        unk_range(g, a, 1, lo, hi);
        const double up = (qp[a] >= lo && qp[a] <= hi ? ut.c[a] : ubd.c[a])[at(g, qp[0], qp[1], qp[2])];
        const double um = (q[a] >= lo && q[a] <= hi ? ut.c[a] : ubd.c[a])[at(g, q[0], q[1], q[2])];
        div += (up - um) / g.h;
    }
    bp[at(g, i, j, k)] = coef * div;
}

void launch_pressure_div(const Grid &g, const Phys &ph, const VelArrC<double> &ut, const VelArrC<double> &ubd,
                         double *bp, hipStream_t s)
{
    const long long n = (long long)g.n[0] * g.n[1] * (g.D == 3 ? g.n[2] : 1);
    hipLaunchKernelGGL(k_pressure_div, dim3(nblk(n)), dim3(256), 0, s, g, -ph.sigma / (ph.eps * ph.dt), ut, ubd, bp);
}

// v(cells) += scale * sum[0]
__global__ void k_add_scalar_cells(Grid g, double *v, const double *sum, double scale)
{
    const int ext[3] = {g.n[0], g.n[1], g.D == 3 ? g.n[2] : 1};
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int i, j, k;
    if (!box_at(ext, t, i, j, k)) return;
    v[at(g, i, j, k)] += scale * sum[0];
}

void launch_add_scalar_cells(const Grid &g, double *v, const double *sum, double scale, hipStream_t s)
{
    const long long n = (long long)g.n[0] * g.n[1] * (g.D == 3 ? g.n[2] : 1);
    hipLaunchKernelGGL(k_add_scalar_cells, dim3(nblk(n)), dim3(256), 0, s, g, v, sum, scale);
}

// u_a = u~_a - (eps dt / sigma) beta_a G_a p at every unknown face
__global__ void __launch_bounds__(256) k_project(Grid g, double coef, VelArrC<double> ut, const double *__restrict__ p,
                                                 CoefP<double> beta, VelArr<double> u, VelBox boxes)
{
    const int a = blockIdx.y;
    const Box box = boxes.b[a];
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n = (long long)box.ext[0] * box.ext[1] * box.ext[2];
    if (t >= n) return;
    const int i = box.lo[0] + (int)(t % box.ext[0]);
    t /= box.ext[0];
    const int j = box.lo[1] + (int)(t % box.ext[1]);
    const int k = box.lo[2] + (int)(t / box.ext[1]);
    int qm[3] = {i, j, k};
    qm[a] -= 1;
    const double pr = load_ref(p, ref_at(g, 0, ROLE_P, i, j, k));
    const double pl = load_ref(p, ref_at(g, 0, ROLE_P, qm[0], qm[1], qm[2]));
    const long long e = at(g, i, j, k);
    u.c[a][e] = ut.c[a][e] - coef * ((pr - pl) / g.h) * beta.beta[a][e];
}

void launch_project(const Grid &g, const Phys &ph, const VelArrC<double> &ut, const double *p,
                    const CoefP<double> &beta, const VelArr<double> &u, hipStream_t s)
{
    VelBox boxes;
    long long mx = 0;
    for (int a = 0; a < 3; ++a) {
        Box bx{{0, 0, 0}, {0, 0, 0}};
        if (a < g.D) {
            for (int d = 0; d < 3; ++d) {
                int lo, hi;
                unk_range(g, d, d == a, lo, hi);
                bx.lo[d] = lo;
                bx.ext[d] = hi - lo + 1;
            }
            const long long n = (long long)bx.ext[0] * bx.ext[1] * bx.ext[2];
            mx = n > mx ? n : mx;
        }
        boxes.b[a] = bx;
    }
    hipLaunchKernelGGL(k_project, dim3(nblk(mx), g.D), dim3(256), 0, s, g, ph.eps * ph.dt / ph.sigma, ut, p, beta, u,
                       boxes);
}

__global__ void k_copy(const double *__restrict__ src, double *__restrict__ dst, long long n)
{
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x)
        dst[t] = src[t];
}

void launch_copy(const double *src, double *dst, long long n, hipStream_t s)
{
    unsigned b = nblk(n);
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(k_copy, dim3(b ? b : 1), dim3(256), 0, s, src, dst, n);
}

// beta = 1 / rho on every stored position of the faces normal to axis
// a = blockIdx.y
__global__ void k_beta(Grid g, VelArrC<double> rho, VelArr<double> beta)
{
    const int a = blockIdx.y;
    const int vmask = face_mask(a);
    int ext[3];
    for (int d = 0; d < 3; ++d) ext[d] = stored_extent(g, d, (vmask >> d) & 1);
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int i, j, k;
    if (!box_at(ext, t, i, j, k)) return;
    const long long e = at(g, i, j, k);
    beta.c[a][e] = 1.0 / rho.c[a][e];
}

void launch_beta_faces(const Grid &g, const VelArrC<double> &rho, const VelArr<double> &beta, hipStream_t s)
{
    long long mx = 0;
    for (int a = 0; a < g.D; ++a) {
        long long n = 1;
        for (int d = 0; d < 3; ++d) n *= stored_extent(g, d, d == a);
        mx = n > mx ? n : mx;
    }
    hipLaunchKernelGGL(k_beta, dim3(nblk(mx), g.D), dim3(256), 0, s, g, rho, beta);
}

// array q = blockIdx.y of the set
struct F32Dst {
    float *v[COEF_SET];
};
__global__ void k_to_f32(CoefSet<double> src, F32Dst dst, long long n)
{
    const double *__restrict__ a = src.v[blockIdx.y];
    float *__restrict__ b = dst.v[blockIdx.y];
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x)
        b[t] = (float)a[t];
}

void launch_to_f32(const CoefSet<double> &src, float *const dst[COEF_SET], long long n, hipStream_t s)
{
    if (src.n <= 0 || n <= 0) return;
    F32Dst d;
    for (int q = 0; q < COEF_SET; ++q) d.v[q] = q < src.n ? dst[q] : nullptr;
    unsigned b = nblk(n);
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(k_to_f32, dim3(b, src.n), dim3(256), 0, s, src, d, n);
}

// plain sum of a cell field into partial sums (for the mean of the pressure)
__global__ void __launch_bounds__(256) k_sum_cells(Grid g, const double *__restrict__ v, double *partial)
{
    const int ext[3] = {g.n[0], g.n[1], g.D == 3 ? g.n[2] : 1};
    const long long n = (long long)ext[0] * ext[1] * ext[2];
    double acc = 0.0;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        box_at(ext, t, i, j, k);
        acc += v[at(g, i, j, k)];
    }
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

int launch_sum_cells(const Grid &g, const double *v, double *partial, hipStream_t s)
{
    const long long n = (long long)g.n[0] * g.n[1] * (g.D == 3 ? g.n[2] : 1);
    unsigned b = nblk(n);
    if (b > NORM_BLOCKS) b = NORM_BLOCKS;
    hipLaunchKernelGGL(k_sum_cells, dim3(b), dim3(256), 0, s, g, v, partial);
    return (int)b;
}

}  // namespace ibmg
