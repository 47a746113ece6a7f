// Internal definitions shared by the HIP translation units of the library:
// the per-level grid descriptor passed to kernels, the boundary rules that
// map an out-of-range lattice index to the value it stands for, and the
// regularised delta.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ibmg {

// axis kinds (same numbering as ibb_axis_bc)
enum { AX_PERIODIC = 0, AX_WALLS = 1, AX_INOUT = 2 };

// How a field behaves beyond the domain:
//  ROLE_P  pressure / pressure corrections: zero normal derivative at walls
//          and inflow, zero value on the outflow face;
//  ROLE_V  velocity with homogeneous boundary data (unknowns, corrections,
//          residuals): the fixed normal faces read as zero, the tangential
//          component is odd across walls and the inflow plane and even
//          across the outflow plane, the outflow face mirrors evenly;
//  ROLE_C  coefficient fields: even reflection.
// Periodic axes wrap for every role.
enum { ROLE_P = 0, ROLE_V = 1, ROLE_C = 3 };

// One multigrid level.  Every field of the level (cell, face or edge
// lattice) uses the same uniform array covering lattice indices -1 .. n[d]+1
// along each axis ((n[0]+3) x (n[1]+3) (x (n[2]+3)) entries), so that
// neighbouring positions of different lattices sit at fixed offsets and one
// layer of ghost positions surrounds the domain.  Lattice position (i, j, k)
// is entry at(i, j, k).
struct Grid {
    int D;
    int n[3];
    int bc[3];
    int NX, NY;        // row length and rows per plane of the uniform array
    long long NXY;     // entries per plane
    long long nel;     // entries per array
    double h;
};

// every array holds fewer than 2^31 entries (checked when a context is
// created), so the index is formed in 32-bit arithmetic
__host__ __device__ inline long long at(const Grid &g, int i, int j, int k)
{
    const unsigned kk = (unsigned)(k + (g.D == 3 ? 1 : 0));
    return (long long)((kk * (unsigned)g.NY + (unsigned)(j + 1)) * (unsigned)g.NX + (unsigned)(i + 1));
}

// lattice index of entry e (inverse of at)
__host__ __device__ inline void decode(const Grid &g, long long e, int &i, int &j, int &k)
{
    k = (int)(e / g.NXY) - (g.D == 3 ? 1 : 0);
    const long long r = e % g.NXY;
    j = (int)(r / g.NX) - 1;
    i = (int)(r % g.NX) - 1;
}

__host__ __device__ inline long long stride_of(const Grid &g, int d)
{
    return d == 0 ? 1 : (d == 1 ? (long long)g.NX : g.NXY);
}

// Range of unknowns along axis d for a lattice that is vertex-centred
// (vert) or cell-centred along d.  Fixed faces (walls, inflow) are not
// unknowns; the outflow face is.
__host__ __device__ inline void unk_range(const Grid &g, int d, int vert, int &lo, int &hi)
{
    if (d >= g.D) { lo = hi = 0; return; }
    if (!vert) { lo = 0; hi = g.n[d] - 1; return; }
    if (g.bc[d] == AX_PERIODIC) { lo = 0; hi = g.n[d] - 1; }
    else if (g.bc[d] == AX_WALLS) { lo = 1; hi = g.n[d] - 1; }
    else { lo = 1; hi = g.n[d]; }
}

// Closed-domain positions stored along axis d (the compact layout).
__host__ __device__ inline int stored_extent(const Grid &g, int d, int vert)
{
    if (d >= g.D) return 1;
    if (!vert) return g.n[d];
    return g.bc[d] == AX_PERIODIC ? g.n[d] : g.n[d] + 1;
}

// Map coordinate q along axis d into the stored range under a role.
// Returns false when the value there is the zero of a fixed face;
// otherwise updates q and multiplies s by the reflection sign.
__host__ __device__ inline bool resolve(const Grid &g, int d, int vert, int role, int &q, int &s)
{
    const int n = g.n[d], bc = g.bc[d];
    if (!vert) {
        if (q >= 0 && q < n) return true;
        if (bc == AX_PERIODIC) { q = q < 0 ? q + n : q - n; return true; }
        if (q < 0) {                 // wall or inflow side
            q = 0;
            if (role == ROLE_V) s = -s;
            return true;
        }
        q = n - 1;                   // wall or outflow side
        if (role == ROLE_P && bc == AX_INOUT) s = -s;
        if (role == ROLE_V && bc == AX_WALLS) s = -s;
        return true;
    }
    if (bc == AX_PERIODIC) {
        if (q < 0) q += n;
        else if (q >= n) q -= n;
        return true;
    }
    if (role == ROLE_C) {
        if (q < 0) q = -q;
        else if (q > n) q = 2 * n - q;
        return true;
    }
    if (q <= 0) return false;        // fixed low face
    if (q < n) return true;
    if (q == n) return bc == AX_INOUT;
    q = 2 * n - q;                   // one past the outflow face mirrors evenly
    return true;
}

// Resolved reference: entry index and sign (s == 0 means the value is 0).
struct Ref {
    long long idx;
    int s;
};

// vmask bit d set: the lattice is vertex-centred along axis d
__host__ __device__ inline Ref ref_at(const Grid &g, int vmask, int role, int i, int j, int k)
{
    int q[3] = {i, j, k};
    int s = 1;
    for (int d = 0; d < g.D; ++d)
        if (!resolve(g, d, (vmask >> d) & 1, role, q[d], s)) return Ref{0, 0};
    return Ref{at(g, q[0], q[1], q[2]), s};
}

template <typename T>
__device__ inline T load_ref(const T *__restrict__ v, Ref r)
{
    return r.s == 0 ? T(0) : (r.s > 0 ? v[r.idx] : -v[r.idx]);
}

// The same value through an unconditional load: a reference to a fixed
// zero still points at a valid entry (index 0), so every load of a row can
// be issued together and the sign is applied afterwards.
template <typename T>
__device__ inline T ld(const T *__restrict__ v, Ref r)
{
    const T x = v[r.idx];
    return r.s == 0 ? T(0) : (r.s > 0 ? x : -x);
}

// Ghost positions along axis d whose value is (sign x) the value at q: the
// inverse of resolve() for the positions the stencils read.  There are at
// most two, one caused by each end of the axis; slot 0 holds the image
// across the low end, slot 1 the one across the high end (sign 0: none).
struct AxisImages {
    int q[2];
    int s[2];
};

__host__ __device__ inline AxisImages images_of(const Grid &g, int d, int vert, int role, int q)
{
    const int n = g.n[d], bc = g.bc[d];
    AxisImages m{{0, 0}, {0, 0}};
    if (bc == AX_PERIODIC) {
        if (q == n - 1) { m.q[0] = -1; m.s[0] = 1; }
        if (q == 0) { m.q[1] = n; m.s[1] = 1; }
        return m;
    }
    if (!vert) {
        if (q == 0) { m.q[0] = -1; m.s[0] = role == ROLE_V ? -1 : 1; }
        if (q == n - 1) {
            int s = 1;
            if (role == ROLE_P && bc == AX_INOUT) s = -1;
            if (role == ROLE_V && bc == AX_WALLS) s = -1;
            m.q[1] = n;
            m.s[1] = s;
        }
        return m;
    }
    if (role == ROLE_C) {
        if (q == 1) { m.q[0] = -1; m.s[0] = 1; }
        if (q == n - 1) { m.q[1] = n + 1; m.s[1] = 1; }
        return m;
    }
    if (role == ROLE_V && bc == AX_INOUT && q == n - 1) { m.q[1] = n + 1; m.s[1] = 1; }
    return m;
}

// write v (times the reflection sign) to every ghost image of (i, j, k):
// each axis contributes the position itself or one of its images
template <typename T>
__host__ __device__ inline void write_images_any(const Grid &g, const AxisImages im[3], T *x, int i, int j, int k, T v)
{
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
                x[at(g, qa, qb, qc)] = sa * sb * sc > 0 ? v : -v;
            }
}

template <typename T>
__host__ __device__ inline void write_images(const Grid &g, int vmask, int role, T *x, int i, int j, int k, T v)
{
    const int q[3] = {i, j, k};
    AxisImages im[3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
        im[d] = d < g.D ? images_of(g, d, (vmask >> d) & 1, role, q[d]) : AxisImages{{0, 0}, {0, 0}};
    if ((im[0].s[0] | im[0].s[1] | im[1].s[0] | im[1].s[1] | im[2].s[0] | im[2].s[1]) == 0) return;
    // An axis with images at both ends only on the shortest lattices: there,
    // every combination of the two.
    if ((im[0].s[0] && im[0].s[1]) || (im[1].s[0] && im[1].s[1]) || (im[2].s[0] && im[2].s[1])) {
        write_images_any(g, im, x, i, j, k, v);
        return;
    }
    // Otherwise at most one image per axis: one write for each non-empty
    // set of the axes that have one (the same positions and values).
    int p[3], s[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        s[d] = im[d].s[0] ? im[d].s[0] : im[d].s[1];
        p[d] = im[d].s[0] ? im[d].q[0] : im[d].q[1];
    }
#pragma unroll
    for (int m = 1; m < 8; ++m) {
        if (((m & 1) && !s[0]) || ((m & 2) && !s[1]) || ((m & 4) && !s[2])) continue;
        const int sg = ((m & 1) ? s[0] : 1) * ((m & 2) ? s[1] : 1) * ((m & 4) ? s[2] : 1);
        x[at(g, (m & 1) ? p[0] : i, (m & 2) ? p[1] : j, (m & 4) ? p[2] : k)] = sg > 0 ? v : -v;
    }
}

// lattice masks
__host__ __device__ inline int face_mask(int a) { return 1 << a; }
__host__ __device__ inline int edge_mask(int D, int c) { return ((1 << D) - 1) & ~(1 << c); }

// The two regularised deltas of the paper's "Dirac Delta Approximation"
// section: kernel 0 the cosine phi_2, kernel 1 Peskin's four-point phi_1.
__device__ inline double phi_eval(int kernel, double r)
{
    double a = fabs(r);
    if (!(a < 2.0)) return 0.0;
    if (kernel == 1) {
        if (a <= 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) * 0.125;
        return (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a)) * 0.125;
    }
    return 0.25 * (1.0 + cos(1.5707963267948966 * a));
}

}  // namespace ibmg
