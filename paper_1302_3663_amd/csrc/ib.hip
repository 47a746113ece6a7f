// Immersed-boundary kernels: node binning, the spread of force and density
// to the faces (eq:discrForceCouple, eq:discrDensCouple) and of the
// viscosity maximum to cells and edges (eq:ViscExp), the interpolation of
// face velocities to nodes (eq:discrVelCouple), the Euler move of the
// nodes, and the spring breakage and force passes (eq:springF and the
// breakage rule of the "Elastic Forces" section).
//
// The spread runs as a gather: each lattice point visits the nodes of the
// bins around it, in ascending node order within a bin, so the result does
// not depend on thread timing and no atomics touch the fields.
#include "common.h"
#include "kernels.h"

namespace ibmg {

static inline unsigned nblk(long long n) { return (unsigned)((n + 255) / 256); }

__device__ inline double domain_len(const Grid &g, int d) { return g.n[d] * g.h; }

// nearest periodic image of a separation along axis d
__device__ inline double min_image(const Grid &g, int d, double v)
{
    if (g.bc[d] != AX_PERIODIC) return v;
    const double L = domain_len(g, d);
    return v - L * floor(v / L + 0.5);
}

// ---------------------------------------------------------------------------
// counting sort with a deterministic order inside each bucket
// ---------------------------------------------------------------------------
__global__ void k_count_keys(const int *__restrict__ keys, int n, int *count)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) atomicAdd(&count[keys[t]], 1);
}

// exclusive scan of count[0..nb) into start[0..nb] in three passes over
// tiles of SCAN_TILE buckets: tile sums, a scan of the tile sums, and a
// scan inside every tile offset by its tile's start
constexpr int SCAN_TILE = 1024;

// inclusive scan of one int per thread across a 1024-thread block
__device__ inline int block_incl_scan(int v, int *buf)
{
    const int t = threadIdx.x;
    buf[t] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_TILE; off <<= 1) {
        const int w = t >= off ? buf[t - off] : 0;
        __syncthreads();
        buf[t] += w;
        __syncthreads();
    }
    const int r = buf[t];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(1024) k_scan_tiles(const int *__restrict__ count, int nb, int *tsum)
{
    __shared__ int buf[SCAN_TILE];
    const int i = blockIdx.x * SCAN_TILE + threadIdx.x;
    const int r = block_incl_scan(i < nb ? count[i] : 0, buf);
    if (threadIdx.x == SCAN_TILE - 1) tsum[blockIdx.x] = r;
}

// one block: tsum[0..nt) -> exclusive prefix in place; start[nb] = total
__global__ void __launch_bounds__(1024) k_scan_tsum(int *tsum, int nt, int *start, int nb)
{
    __shared__ int buf[SCAN_TILE];
    int carry = 0;
    for (int base = 0; base < nt; base += SCAN_TILE) {
        const int i = base + threadIdx.x;
        const int v = i < nt ? tsum[i] : 0;
        const int r = block_incl_scan(v, buf);
        if (i < nt) tsum[i] = carry + r - v;
        carry += buf[SCAN_TILE - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) start[nb] = carry;
}

__global__ void __launch_bounds__(1024) k_scan_apply(const int *__restrict__ count, int nb, const int *__restrict__ tsum,
                                                     int *start)
{
    __shared__ int buf[SCAN_TILE];
    const int i = blockIdx.x * SCAN_TILE + threadIdx.x;
    const int v = i < nb ? count[i] : 0;
    const int r = block_incl_scan(v, buf);
    if (i < nb) start[i] = tsum[blockIdx.x] + r - v;
}

int scan_scratch_ints(long long nb) { return (int)((nb + SCAN_TILE - 1) / SCAN_TILE) + 2; }

__global__ void k_scatter_keys(const int *__restrict__ keys, int n, const int *__restrict__ start, int *cursor, int *ids)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int k = keys[t];
    const int pos = start[k] + atomicAdd(&cursor[k], 1);
    ids[pos] = t;
}

// order each bucket by id modulo `mod` (mod = 0: by id).  A one-wavefront
// workgroup takes the buckets blockIdx.x, + gridDim.x, ...: it loads the
// bucket's ids into LDS and writes every entry to its rank, the number of
// entries with a smaller key (keys within a bucket are distinct).  A bucket
// longer than the LDS tile is ordered by the first lane, by insertion.
constexpr int RANK_TILE = 1024;
constexpr int RANK_GRID = 8192;

__global__ void __launch_bounds__(64) k_sort_buckets(const int *__restrict__ start, int nb, int *ids, int mod)
{
    __shared__ int tile[RANK_TILE];
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        const int lo = start[b], hi = start[b + 1], n = hi - lo;
        if (n < 2) continue;
        if (n <= RANK_TILE) {
            for (int q = threadIdx.x; q < n; q += blockDim.x) tile[q] = ids[lo + q];
            __syncthreads();
            for (int q = threadIdx.x; q < n; q += blockDim.x) {
                const int v = tile[q];
                const int kv = mod ? v % mod : v;
                int rank = 0;
                for (int r = 0; r < n; ++r) {
                    const int w = tile[r];
                    rank += (mod ? w % mod : w) < kv;
                }
                ids[lo + rank] = v;
            }
            __syncthreads();
        } else if (threadIdx.x == 0) {
            for (int i = lo + 1; i < hi; ++i) {
                const int v = ids[i];
                const int kv = mod ? v % mod : v;
                int j = i - 1;
                while (j >= lo && (mod ? ids[j] % mod : ids[j]) > kv) {
                    ids[j + 1] = ids[j];
                    --j;
                }
                ids[j + 1] = v;
            }
        }
    }
}

void launch_bucket_sort(const int *keys, int n, int nbuckets, int *count, int *start, int *ids, int mod,
                        int *scan_tmp, hipStream_t s)
{
    launch_fill<int>(count, nbuckets, 0, s);
    if (n > 0) hipLaunchKernelGGL(k_count_keys, dim3(nblk(n)), dim3(256), 0, s, keys, n, count);
    const int nt = (nbuckets + SCAN_TILE - 1) / SCAN_TILE;
    hipLaunchKernelGGL(k_scan_tiles, dim3(nt), dim3(SCAN_TILE), 0, s, count, nbuckets, scan_tmp);
    hipLaunchKernelGGL(k_scan_tsum, dim3(1), dim3(SCAN_TILE), 0, s, scan_tmp, nt, start, nbuckets);
    hipLaunchKernelGGL(k_scan_apply, dim3(nt), dim3(SCAN_TILE), 0, s, count, nbuckets, scan_tmp, start);
    launch_fill<int>(count, nbuckets, 0, s);
    if (n > 0) hipLaunchKernelGGL(k_scatter_keys, dim3(nblk(n)), dim3(256), 0, s, keys, n, start, count, ids);
    const unsigned ng = (unsigned)(nbuckets < RANK_GRID ? (nbuckets > 0 ? nbuckets : 1) : RANK_GRID);
    launch_timed(k_sort_buckets, dim3(ng), dim3(64), s, start, nbuckets, ids, mod);
}

// ---------------------------------------------------------------------------
// bins: cell size at least twice the delta width along each axis, so every
// node within the support of a point lies in the point's bin or a neighbour
// ---------------------------------------------------------------------------
__device__ inline int bin_coord(const Bins &bins, int d, double x)
{
    int b = (int)floor(x / bins.bs[d]);
    return b < 0 ? 0 : (b >= bins.nb[d] ? bins.nb[d] - 1 : b);
}

__global__ void k_bin_of(Grid g, Bins bins, const double *__restrict__ X, long long stride, int eta)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= eta) return;
    int b[3] = {0, 0, 0};
    for (int d = 0; d < g.D; ++d) {
        double x = X[d * stride + s];
        if (g.bc[d] == AX_PERIODIC) {
            const double L = domain_len(g, d);
            x -= L * floor(x / L);
        }
        b[d] = bin_coord(bins, d, x);
    }
    bins.bin_of[s] = (b[2] * bins.nb[1] + b[1]) * bins.nb[0] + b[0];
}

// Bins are at least the delta width w wide (bins_for_width), so the nodes
// within a point's support lie in its own bin or the BIN_REACH bins on
// either side.
constexpr int BIN_REACH = 2, BIN_SPAN = 2 * BIN_REACH + 1;

// distinct bins along axis d where the points of bin b look for nodes, in
// increasing offset from b - BIN_REACH (wrapped on a periodic axis; every
// bin, in order, when a periodic axis has no more than 2 BIN_REACH)
__device__ inline int bin_candidates(const Grid &g, const Bins &bins, int d, int b, int lst[BIN_SPAN])
{
    if (d >= g.D) {
        lst[0] = 0;
        return 1;
    }
    const int nb = bins.nb[d];
    if (g.bc[d] == AX_PERIODIC && nb <= 2 * BIN_REACH) {
        for (int t = 0; t < nb; ++t) lst[t] = t;
        return nb;
    }
    int c = 0;
    for (int o = -BIN_REACH; o <= BIN_REACH; ++o) {
        int t = b + o;
        if (g.bc[d] == AX_PERIODIC) t = (t + nb) % nb;
        else if (t < 0 || t >= nb) continue;
        lst[c++] = t;
    }
    return c;
}

// The candidate bins along x as at most two runs of consecutive bins (a
// wrap splits them): each run's nodes are one range of the sorted ids, in
// bin order and ascending within a bin, as bin by bin.
struct XRuns {
    int lo[2], hi[2];
    int n;
};

__device__ inline XRuns x_runs(const int lst[BIN_SPAN], int cnt)
{
    XRuns r;
    r.n = 1;
    r.lo[0] = r.hi[0] = lst[0];
    r.lo[1] = r.hi[1] = 0;
    for (int e = 1; e < cnt; ++e) {
        if (lst[e] == r.hi[r.n - 1] + 1) {
            r.hi[r.n - 1] = lst[e];
        } else {
            r.lo[r.n] = r.hi[r.n] = lst[e];
            ++r.n;
        }
    }
    return r;
}

// near[bin]: does any bin where the bin's points look hold a node?
__global__ void __launch_bounds__(256) k_bin_near(Grid g, Bins bins)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= bins.nbins) return;
    const int b[3] = {t % bins.nb[0], (t / bins.nb[0]) % bins.nb[1], t / (bins.nb[0] * bins.nb[1])};
    int lst[3][BIN_SPAN], cnt[3];
    for (int d = 0; d < 3; ++d) cnt[d] = bin_candidates(g, bins, d, b[d], lst[d]);
    const XRuns xr = x_runs(lst[0], cnt[0]);
    unsigned char any = 0;
    for (int c = 0; c < cnt[2]; ++c)
        for (int bb = 0; bb < cnt[1]; ++bb) {
            const int row = (lst[2][c] * bins.nb[1] + lst[1][bb]) * bins.nb[0];
            for (int q = 0; q < xr.n; ++q)
                if (bins.start[row + xr.hi[q] + 1] > bins.start[row + xr.lo[q]]) any = 1;
        }
    bins.near[t] = any;
}

void launch_bin_nodes(const Grid &g, const Bins &bins, const double *X, long long stride, int eta, int *scan_tmp,
                      hipStream_t s)
{
    if (eta > 0) hipLaunchKernelGGL(k_bin_of, dim3(nblk(eta)), dim3(256), 0, s, g, bins, X, stride, eta);
    launch_bucket_sort(bins.bin_of, eta, bins.nbins, bins.count, bins.start, bins.sorted, 0, scan_tmp, s);
    if (bins.near) hipLaunchKernelGGL(k_bin_near, dim3(nblk(bins.nbins)), dim3(256), 0, s, g, bins);
}

// the bins where a point looks for nodes, along each axis, and its own bin
struct BinNbr {
    int cnt[3];
    int lst[3][BIN_SPAN];
    int own;
};

__device__ inline BinNbr bin_neighbours(const Grid &g, const Bins &bins, const double x[3])
{
    BinNbr r;
    int b[3];
    for (int d = 0; d < 3; ++d) {
        b[d] = 0;
        if (d < g.D) {
            double xx = x[d];
            if (g.bc[d] == AX_PERIODIC) {
                const double L = domain_len(g, d);
                xx -= L * floor(xx / L);
            }
            b[d] = bin_coord(bins, d, xx);
        }
        r.cnt[d] = bin_candidates(g, bins, d, b[d], r.lst[d]);
    }
    r.own = (b[2] * bins.nb[1] + b[1]) * bins.nb[0] + b[0];
    return r;
}

// no node where the point looks: every sum over candidates is empty
__device__ inline bool nothing_near(const Bins &bins, const BinNbr &nbr)
{
    return bins.near && !bins.near[nbr.own];
}

// delta~(x - X_s, w) = w^-D prod_d phi((x_d - X_d) / w), zero outside the support
__device__ inline double delta_w(const Grid &g, int kernel, double inv_w, double scale, const double x[3],
                                 const double *__restrict__ X, long long stride, int s)
{
    double w = scale;
    for (int d = 0; d < g.D; ++d) {
        const double r = min_image(g, d, x[d] - X[d * stride + s]) * inv_w;
        if (!(fabs(r) < 2.0)) return 0.0;
        w *= phi_eval(kernel, r);
    }
    return w;
}

__device__ inline void lattice_coord(const Grid &g, int vmask, int i, int j, int k, double x[3])
{
    const int q[3] = {i, j, k};
    for (int d = 0; d < 3; ++d) x[d] = ((vmask >> d) & 1) ? q[d] * g.h : (q[d] + 0.5) * g.h;
}

// f_a(x) = sum_s F_a(s) delta~ and rho_a(x) = rho0 + rho_b d0^D sum_s delta~
// at every closed-domain a-face
__global__ void __launch_bounds__(256) k_spread_face(Grid g, Phys ph, Bins bins, const double *__restrict__ X,
                                                     const double *__restrict__ F, long long stride, int a,
                                                     double width, double *f_out, double *rho_out)
{
    const int vmask = face_mask(a);
    int ext[3];
    for (int d = 0; d < 3; ++d) ext[d] = stored_extent(g, d, (vmask >> d) & 1);
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)ext[0] * ext[1] * ext[2]) return;
    const int i = (int)(t % ext[0]);
    t /= ext[0];
    const int j = (int)(t % ext[1]);
    const int k = (int)(t / ext[1]);
    double x[3];
    lattice_coord(g, vmask, i, j, k, x);
    const double inv_w = 1.0 / width;
    double scale = 1.0;
    for (int d = 0; d < g.D; ++d) scale /= width;
    const BinNbr nbr = bin_neighbours(g, bins, x);
    double accf = 0.0, accw = 0.0;
    const int nz = nothing_near(bins, nbr) ? 0 : nbr.cnt[2];
    const XRuns xr = x_runs(nbr.lst[0], nbr.cnt[0]);
    for (int c = 0; c < nz; ++c)
        for (int b = 0; b < nbr.cnt[1]; ++b)
            for (int rq = 0; rq < xr.n; ++rq) {
                const int row = (nbr.lst[2][c] * bins.nb[1] + nbr.lst[1][b]) * bins.nb[0];
                const int p1 = bins.start[row + xr.hi[rq] + 1];
                for (int p = bins.start[row + xr.lo[rq]]; p < p1; ++p) {
                    const int s = bins.sorted[p];
                    const double w = delta_w(g, ph.kernel, inv_w, scale, x, X, stride, s);
                    if (w == 0.0) continue;
                    if (F) accf += F[a * stride + s] * w;
                    accw += w;
                }
            }
    const long long u = at(g, i, j, k);
    if (f_out) f_out[u] = accf;
    if (rho_out) rho_out[u] = ph.rho0 + ph.rho_b * ph.d0_pow_d * accw;
}

// The same gather with one wave per lattice point, for lattices too small
// to fill the chip with one point per thread while a point may see
// thousands of nodes (small grids, dense biofilms).  The 64 lanes evaluate
// the weights of 64 consecutive candidates at once; the sums then take them
// in candidate order, through the same expressions as k_spread_face, so
// the result is the same bits.
constexpr long long SPREAD_WAVE_MAX_POINTS = 65536;

__global__ void __launch_bounds__(256) k_spread_face_w(Grid g, Phys ph, Bins bins, const double *__restrict__ X,
                                                       const double *__restrict__ F, long long stride, int a,
                                                       double width, double *f_out, double *rho_out)
{
    const int vmask = face_mask(a);
    const int lane = threadIdx.x & 63;
    int ext[3];
    for (int d = 0; d < 3; ++d) ext[d] = stored_extent(g, d, (vmask >> d) & 1);
    long long t = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= (long long)ext[0] * ext[1] * ext[2]) return;   // the whole wave
    const int i = (int)(t % ext[0]);
    t /= ext[0];
    const int j = (int)(t % ext[1]);
    const int k = (int)(t / ext[1]);
    double x[3];
    lattice_coord(g, vmask, i, j, k, x);
    const double inv_w = 1.0 / width;
    double scale = 1.0;
    for (int d = 0; d < g.D; ++d) scale /= width;
    const BinNbr nbr = bin_neighbours(g, bins, x);
    double accf = 0.0, accw = 0.0;
    const int nz = nothing_near(bins, nbr) ? 0 : nbr.cnt[2];
    const XRuns xr = x_runs(nbr.lst[0], nbr.cnt[0]);
    for (int c = 0; c < nz; ++c)
        for (int b = 0; b < nbr.cnt[1]; ++b)
            for (int rq = 0; rq < xr.n; ++rq) {
                const int row = (nbr.lst[2][c] * bins.nb[1] + nbr.lst[1][b]) * bins.nb[0];
                const int p1 = bins.start[row + xr.hi[rq] + 1];
                for (int base = bins.start[row + xr.lo[rq]]; base < p1; base += 64) {
                    const int p = base + lane;
                    double w = 0.0, fv = 0.0;
                    if (p < p1) {
                        const int s = bins.sorted[p];
                        w = delta_w(g, ph.kernel, inv_w, scale, x, X, stride, s);
                        if (F) fv = F[a * stride + s];
                    }
                    const int cnt = p1 - base < 64 ? p1 - base : 64;
                    for (int q = 0; q < cnt; ++q) {
                        const double wq = __shfl(w, q);
                        const double fq = __shfl(fv, q);
                        if (wq == 0.0) continue;
                        if (F) accf += fq * wq;
                        accw += wq;
                    }
                }
            }
    if (lane == 0) {
        const long long u = at(g, i, j, k);
        if (f_out) f_out[u] = accf;
        if (rho_out) rho_out[u] = ph.rho0 + ph.rho_b * ph.d0_pow_d * accw;
    }
}

void launch_spread_face(const Grid &g, const Phys &ph, const Bins &bins, const double *X, const double *F,
                        long long stride, int a, double width, double *f_out, double *rho_out, hipStream_t s)
{
    long long n = 1;
    for (int d = 0; d < 3; ++d) n *= stored_extent(g, d, d == a);
    if (n <= SPREAD_WAVE_MAX_POINTS)
        launch_timed(k_spread_face_w, dim3((unsigned)((n + 3) / 4)), dim3(256), s, g, ph, bins, X, F, stride, a,
                     width, f_out, rho_out);
    else
        launch_timed(k_spread_face, dim3(nblk(n)), dim3(256), s, g, ph, bins, X, F, stride, a, width, f_out,
                     rho_out);
}

// mu(x) = max over nodes of (2 omega)^D (mu_max - mu_out) delta~ + mu_out,
// mu_out where no node reaches
__global__ void __launch_bounds__(256) k_spread_visc(Grid g, Phys ph, Bins bins, const double *__restrict__ X,
                                                     long long stride, int vmask, double *mu_out)
{
    int ext[3];
    for (int d = 0; d < 3; ++d) ext[d] = stored_extent(g, d, (vmask >> d) & 1);
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)ext[0] * ext[1] * ext[2]) return;
    const int i = (int)(t % ext[0]);
    t /= ext[0];
    const int j = (int)(t % ext[1]);
    const int k = (int)(t / ext[1]);
    double x[3];
    lattice_coord(g, vmask, i, j, k, x);
    const double width = ph.omega;
    const double inv_w = 1.0 / width;
    double scale = 1.0, vol = 1.0;
    for (int d = 0; d < g.D; ++d) {
        scale /= width;
        vol *= 2.0 * width;
    }
    const double dmu = ph.mu_max - ph.mu_out;
    double best = ph.mu_out;
    if (dmu > 0.0) {
        const BinNbr nbr = bin_neighbours(g, bins, x);
        double wmax = 0.0;
        const int nz = nothing_near(bins, nbr) ? 0 : nbr.cnt[2];
        const XRuns xr = x_runs(nbr.lst[0], nbr.cnt[0]);
        for (int c = 0; c < nz; ++c)
            for (int b = 0; b < nbr.cnt[1]; ++b)
                for (int rq = 0; rq < xr.n; ++rq) {
                    const int row = (nbr.lst[2][c] * bins.nb[1] + nbr.lst[1][b]) * bins.nb[0];
                    const int p1 = bins.start[row + xr.hi[rq] + 1];
                    for (int p = bins.start[row + xr.lo[rq]]; p < p1; ++p) {
                        const double w = delta_w(g, ph.kernel, inv_w, scale, x, X, stride, bins.sorted[p]);
                        wmax = w > wmax ? w : wmax;
                    }
                }
        if (wmax > 0.0) {
            const double cand = vol * dmu * wmax + ph.mu_out;
            best = cand > best ? cand : best;
        }
    }
    mu_out[at(g, i, j, k)] = best;
}

// k_spread_visc with one wave per lattice point (see k_spread_face_w); the
// largest weight does not depend on the order the candidates are taken in
__global__ void __launch_bounds__(256) k_spread_visc_w(Grid g, Phys ph, Bins bins, const double *__restrict__ X,
                                                       long long stride, int vmask, double *mu_out)
{
    const int lane = threadIdx.x & 63;
    int ext[3];
    for (int d = 0; d < 3; ++d) ext[d] = stored_extent(g, d, (vmask >> d) & 1);
    long long t = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= (long long)ext[0] * ext[1] * ext[2]) return;   // the whole wave
    const int i = (int)(t % ext[0]);
    t /= ext[0];
    const int j = (int)(t % ext[1]);
    const int k = (int)(t / ext[1]);
    double x[3];
    lattice_coord(g, vmask, i, j, k, x);
    const double width = ph.omega;
    const double inv_w = 1.0 / width;
    double scale = 1.0, vol = 1.0;
    for (int d = 0; d < g.D; ++d) {
        scale /= width;
        vol *= 2.0 * width;
    }
    const double dmu = ph.mu_max - ph.mu_out;
    double best = ph.mu_out;
    if (dmu > 0.0) {
        const BinNbr nbr = bin_neighbours(g, bins, x);
        double wmax = 0.0;
        const int nz = nothing_near(bins, nbr) ? 0 : nbr.cnt[2];
        const XRuns xr = x_runs(nbr.lst[0], nbr.cnt[0]);
        for (int c = 0; c < nz; ++c)
            for (int b = 0; b < nbr.cnt[1]; ++b)
                for (int rq = 0; rq < xr.n; ++rq) {
                    const int row = (nbr.lst[2][c] * bins.nb[1] + nbr.lst[1][b]) * bins.nb[0];
                    const int p1 = bins.start[row + xr.hi[rq] + 1];
                    for (int p = bins.start[row + xr.lo[rq]] + lane; p < p1; p += 64) {
                        const double w = delta_w(g, ph.kernel, inv_w, scale, x, X, stride, bins.sorted[p]);
                        wmax = w > wmax ? w : wmax;
                    }
                }
        for (int o = 32; o > 0; o >>= 1) {
            const double v = __shfl_xor(wmax, o);
            wmax = v > wmax ? v : wmax;
        }
        if (wmax > 0.0) {
            const double cand = vol * dmu * wmax + ph.mu_out;
            best = cand > best ? cand : best;
        }
    }
    if (lane == 0) mu_out[at(g, i, j, k)] = best;
}

void launch_spread_visc(const Grid &g, const Phys &ph, const Bins &bins, const double *X, long long stride, int vmask,
                        double *mu_out, hipStream_t s)
{
    long long n = 1;
    for (int d = 0; d < 3; ++d) n *= stored_extent(g, d, (vmask >> d) & 1);
    if (n <= SPREAD_WAVE_MAX_POINTS)
        launch_timed(k_spread_visc_w, dim3((unsigned)((n + 3) / 4)), dim3(256), s, g, ph, bins, X, stride, vmask,
                     mu_out);
    else
        launch_timed(k_spread_visc, dim3(nblk(n)), dim3(256), s, g, ph, bins, X, stride, vmask, mu_out);
}

// ---------------------------------------------------------------------------
// interpolation U_a(s) = sum_x u_a(x) delta~(x - X_s, w) h^D over the
// closed-domain a-faces (fixed faces contribute the values they hold)
// ---------------------------------------------------------------------------
//
// One workgroup per (node, component): each thread takes lattice points of
// the support box, the partial sums are combined in a fixed tree order.
constexpr int INTERP_BLOCK = 128;

__global__ void __launch_bounds__(INTERP_BLOCK) k_interp(Grid g, int kernel, double width, VelArrC<double> u,
                                                         const double *__restrict__ X, long long xstride, int eta,
                                                         double *U, long long ustride)
{
    const int s = blockIdx.x;
    const int a = blockIdx.y;
    if (s >= eta) return;
    const double inv_w = 1.0 / width;
    double scale = 1.0, hD = 1.0;
    for (int d = 0; d < g.D; ++d) {
        scale /= width;
        hD *= g.h;
    }
    double Xs[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < g.D; ++d) Xs[d] = X[d * xstride + s];
    const int vmask = face_mask(a);
    int qlo[3], ext[3];
    for (int d = 0; d < 3; ++d) {
        if (d >= g.D) { qlo[d] = 0; ext[d] = 1; continue; }
        const double off = ((vmask >> d) & 1) ? 0.0 : 0.5;
        qlo[d] = (int)floor((Xs[d] - 2.0 * width) / g.h - off);
        ext[d] = (int)ceil((Xs[d] + 2.0 * width) / g.h - off) - qlo[d] + 1;
    }
    const int ntap = ext[0] * ext[1] * ext[2];
    double acc = 0.0;
    for (int t = threadIdx.x; t < ntap; t += blockDim.x) {
        const int q[3] = {qlo[0] + t % ext[0], qlo[1] + (t / ext[0]) % ext[1], qlo[2] + t / (ext[0] * ext[1])};
        int qs[3] = {0, 0, 0};
        double w = scale;
        bool keep = true;
        for (int d = 0; d < g.D; ++d) {
            const int vert = (vmask >> d) & 1;
            const double xc = vert ? q[d] * g.h : (q[d] + 0.5) * g.h;
            const double r = (xc - Xs[d]) * inv_w;
            if (!(fabs(r) < 2.0)) { keep = false; break; }
            int tq = q[d];
            const int se = stored_extent(g, d, vert);
            if (g.bc[d] == AX_PERIODIC) tq = ((tq % g.n[d]) + g.n[d]) % g.n[d];
            else if (tq < 0 || tq >= se) { keep = false; break; }
            qs[d] = tq;
            w *= phi_eval(kernel, r);
        }
        if (keep) acc += u.c[a][at(g, qs[0], qs[1], qs[2])] * w;
    }
    __shared__ double red[INTERP_BLOCK];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = INTERP_BLOCK / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) U[a * ustride + s] = red[0] * hD;
}

void launch_interp(const Grid &g, int kernel, double width, const VelArrC<double> &u, const double *X,
                   long long xstride, int eta, double *U, long long ustride, hipStream_t s)
{
    if (eta <= 0) return;
    launch_timed(k_interp, dim3(eta, g.D), dim3(INTERP_BLOCK), s, g, kernel, width, u, X, xstride, eta, U,
                       ustride);
}

// X += c U, periodic axes wrapped back into [0, L)
__global__ void k_euler(Grid g, double c, const double *__restrict__ U, double *X, long long stride, int eta)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= eta) return;
    for (int d = 0; d < g.D; ++d) {
        double x = X[d * stride + s] + c * U[d * stride + s];
        if (g.bc[d] == AX_PERIODIC) {
            const double L = domain_len(g, d);
            x -= L * floor(x / L);
        }
        X[d * stride + s] = x;
    }
}

void launch_euler(const Grid &g, double c, const double *U, double *X, long long stride, int eta, hipStream_t s)
{
    if (eta > 0) hipLaunchKernelGGL(k_euler, dim3(nblk(eta)), dim3(256), 0, s, g, c, U, X, stride, eta);
}

// ---------------------------------------------------------------------------
// springs
// ---------------------------------------------------------------------------
// separation X_j - X_i (nearest periodic image), each operation rounded on
// its own so that the breakage decision is reproducible
__device__ inline void separation_rn(const Grid &g, const double *__restrict__ X, long long stride, int i, int j,
                                     double v[3])
{
    for (int d = 0; d < 3; ++d) {
        v[d] = 0.0;
        if (d >= g.D) continue;
        double x = __dsub_rn(X[d * stride + j], X[d * stride + i]);
        if (g.bc[d] == AX_PERIODIC) {
            const double L = domain_len(g, d);
            x = __dsub_rn(x, __dmul_rn(L, floor(__dadd_rn(__ddiv_rn(x, L), 0.5))));
        }
        v[d] = x;
    }
}

__device__ inline double len2_rn(const double v[3])
{
    return __dadd_rn(__dadd_rn(__dmul_rn(v[0], v[0]), __dmul_rn(v[1], v[1])), __dmul_rn(v[2], v[2]));
}

__global__ void k_spring_break(Grid g, double ratio, const double *__restrict__ X, long long stride,
                               const int *__restrict__ ij, int m, const double *__restrict__ rest,
                               unsigned char *alive, int *n_broken)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m || !alive[e]) return;
    double v[3];
    separation_rn(g, X, stride, ij[e], ij[m + e], v);
    const double lim = __dmul_rn(ratio, rest[e]);
    if (len2_rn(v) > __dmul_rn(lim, lim)) {
        alive[e] = 0;
        atomicAdd(n_broken, 1);
    }
}

void launch_spring_break(const Grid &g, double ratio, const double *X, long long stride, const int *ij, int m,
                         const double *rest, unsigned char *alive, int *n_broken, hipStream_t s)
{
    if (m > 0)
        hipLaunchKernelGGL(k_spring_break, dim3(nblk(m)), dim3(256), 0, s, g, ratio, X, stride, ij, m, rest, alive,
                           n_broken);
}

// F_s = sum over surviving springs at s, in ascending spring order, of
// K (l - r) d / l with d = X_j - X_i (added at i, subtracted at j)
__global__ void __launch_bounds__(256) k_spring_force(Grid g, const double *__restrict__ X, long long stride, int eta,
                                                      const int *__restrict__ ij, int m,
                                                      const double *__restrict__ rest, const double *__restrict__ K,
                                                      const unsigned char *__restrict__ alive,
                                                      const int *__restrict__ inc_start,
                                                      const int *__restrict__ inc_list, double *F)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= eta) return;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int p = inc_start[s]; p < inc_start[s + 1]; ++p) {
        const int entry = inc_list[p];
        const int e = entry >= m ? entry - m : entry;
        if (!alive[e]) continue;
        const int i = ij[e], j = ij[m + e];
        double v[3];
        separation_rn(g, X, stride, i, j, v);
        const double l = sqrt(len2_rn(v));
        if (l == 0.0) continue;
        const double T = K[e] * (l - rest[e]);
        const double sg = (s == i) ? 1.0 : -1.0;
        for (int d = 0; d < g.D; ++d) acc[d] += sg * (T * v[d] / l);
    }
    for (int d = 0; d < g.D; ++d) F[d * stride + s] = acc[d];
}

void launch_spring_force(const Grid &g, const double *X, long long stride, int eta, const int *ij, int m,
                         const double *rest, const double *K, const unsigned char *alive, const int *inc_start,
                         const int *inc_list, double *F, hipStream_t s)
{
    if (eta > 0)
        launch_timed(k_spring_force, dim3(nblk(eta)), dim3(256), s, g, X, stride, eta, ij, m, rest, K, alive,
                           inc_start, inc_list, F);
}

// incidence keys: entry e -> node i of spring e, entry m + e -> node j
__global__ void k_incidence_keys(const int *__restrict__ ij, int m, int *keys)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 2 * m) keys[t] = ij[t];
}

void launch_incidence_keys(const int *ij, int m, int *keys, hipStream_t s)
{
    if (m > 0) hipLaunchKernelGGL(k_incidence_keys, dim3(nblk(2LL * m)), dim3(256), 0, s, ij, m, keys);
}

__global__ void k_count_alive(const unsigned char *__restrict__ alive, int m, int *out)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m && alive[e]) atomicAdd(out, 1);
}

void launch_count_alive(const unsigned char *alive, int m, int *out, hipStream_t s)
{
    launch_fill<int>(out, 1, 0, s);
    if (m > 0) hipLaunchKernelGGL(k_count_alive, dim3(nblk(m)), dim3(256), 0, s, alive, m, out);
}

// ---------------------------------------------------------------------------
// detached fragments: connected components of the alive springs, each
// labelled by its smallest node id.  Labels only decrease and always name a
// node of the same component, so the fixed point does not depend on the
// order of the atomic updates: every component ends with one root, which is
// its smallest id.
// ---------------------------------------------------------------------------
__global__ void k_frag_anchor(Grid g, const double *__restrict__ X, long long stride, int eta, int axis, double dist,
                              unsigned char *anchored)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < eta) anchored[s] = X[axis * stride + s] < dist ? 1 : 0;
}

__global__ void k_frag_init(int *label, int eta)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < eta) label[s] = s;
}

// hook: for an alive spring whose ends carry different labels, point the
// larger label at the smaller one
__global__ void k_frag_hook(const int *__restrict__ ij, int m, const unsigned char *__restrict__ alive, int *label,
                            int *changed)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m || !alive[e]) return;
    const int a = label[ij[e]], b = label[ij[m + e]];
    if (a == b) return;
    const int hi = a > b ? a : b, lo = a > b ? b : a;
    if (atomicMin(&label[hi], lo) > lo) *changed = 1;
}

// shortcut: every node points straight at the end of its label chain
__global__ void k_frag_jump(int *label, int eta, int *changed)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= eta) return;
    const int l0 = label[s];
    int l = l0;
    while (true) {
        const int n = label[l];
        if (n == l) break;
        l = n;
    }
    if (l != l0) {
        label[s] = l;
        *changed = 1;
    }
}

__global__ void k_frag_mark(const int *__restrict__ label, const unsigned char *__restrict__ anchored, int eta,
                            int *root_anchored)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < eta && anchored[s]) root_anchored[label[s]] = 1;
}

// counts[0] += fragments, counts[1] += detached fragments
__global__ void k_frag_count(const int *__restrict__ label, const int *__restrict__ root_anchored, int eta,
                             int *counts)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= eta || label[s] != s) return;
    atomicAdd(&counts[0], 1);
    if (!root_anchored[s]) atomicAdd(&counts[1], 1);
}

void launch_frag_anchor(const Grid &g, const double *X, long long stride, int eta, int axis, double dist,
                        unsigned char *anchored, hipStream_t s)
{
    if (eta > 0)
        hipLaunchKernelGGL(k_frag_anchor, dim3(nblk(eta)), dim3(256), 0, s, g, X, stride, eta, axis, dist, anchored);
}

void launch_frag_init(int *label, int eta, hipStream_t s)
{
    if (eta > 0) hipLaunchKernelGGL(k_frag_init, dim3(nblk(eta)), dim3(256), 0, s, label, eta);
}

void launch_frag_round(const int *ij, int m, const unsigned char *alive, int *label, int eta, int *changed,
                       hipStream_t s)
{
    launch_fill<int>(changed, 1, 0, s);
    if (m > 0) hipLaunchKernelGGL(k_frag_hook, dim3(nblk(m)), dim3(256), 0, s, ij, m, alive, label, changed);
    if (eta > 0) hipLaunchKernelGGL(k_frag_jump, dim3(nblk(eta)), dim3(256), 0, s, label, eta, changed);
}

void launch_frag_count(const int *label, const unsigned char *anchored, int eta, int *root_anchored, int *counts,
                       hipStream_t s)
{
    launch_fill<int>(counts, 2, 0, s);
    if (eta <= 0) return;
    launch_fill<int>(root_anchored, eta, 0, s);
    hipLaunchKernelGGL(k_frag_mark, dim3(nblk(eta)), dim3(256), 0, s, label, anchored, eta, root_anchored);
    hipLaunchKernelGGL(k_frag_count, dim3(nblk(eta)), dim3(256), 0, s, label, root_anchored, eta, counts);
}

}  // namespace ibmg
