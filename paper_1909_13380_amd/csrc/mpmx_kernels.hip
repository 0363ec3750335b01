// mpmx_kernels.hip -- gfx950 kernels of the explicit MPM step.
//
// One explicit update-stress-first step (code overview: USF; introduction:
// nodal values reset every step, particle-to-node mapping and interpolation
// back with the same mapping functions), with node buffer b holding the
// step's nodal mass and momentum on entry:
//   sort      (only when flagged) counting sort of particles by brick-major
//             cell key, level-major inside each brick; rebuild the work list
//             of <= 512-particle chunks of one 4x4x4-cell brick; the last
//             workgroup then runs the step control (which scenes step, which
//             node buffer they use, work offsets)
//   stress    zero the other node buffer (the previous step's data); nodal
//             velocity with constraints into an LDS tile; velocity gradient,
//             strain increment, volume, elastic / Drucker-Prager stress;
//             internal + external nodal force through an LDS tile (FP64
//             accumulators), one global atomic per touched node and component
//   g2p_p2g   nodal acceleration and updated velocity with constraints into
//             LDS; FLIP/PIC particle velocity, FP64 position, new cell, drift
//             and error checks; the next step's nodal mass (FP64) and
//             momentum from the updated particle into the other buffer
// The first step of a call runs p2g alone to fill buffer b.  USL runs p2g_usl
// (mass, momentum and force from the old stress) and g2p_usl (particle
// update, then stress from the updated nodal velocity, and the clear of the
// other buffer).
//
// The item kernels are persistent: a fixed grid walks the flattened
// (scene, item) list whose offsets live in device memory, so a launch needs
// no host knowledge of how many items each scene has; each of the GPU's 8
// XCDs takes a contiguous range of the list.  Particle and node indices are
// 32-bit and every field is addressed from one scalar base with a 32-bit
// byte offset.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mpmx_dev.h"

#define GLOBAL __attribute__((address_space(1)))

namespace mpmx {

// ------------------------------------------------------------ helpers ----

template <typename T>
__device__ inline GLOBAL T *gp(T *p)
{
    return (GLOBAL T *)p;
}

template <typename T>
__device__ inline const GLOBAL T *gp(const T *p)
{
    return (const GLOBAL T *)p;
}

// Element b (0 or 1) of a two-buffer field of a scene descriptor.
template <typename T>
__device__ inline T pick(const T (&a)[2], int b)
{
    return b ? a[1] : a[0];
}

// Element i of a global array as a scalar base plus a 32-bit byte offset
// (every particle and node array component holds fewer than 2^32 bytes), so
// the address needs no 64-bit vector arithmetic.
template <typename T>
__device__ inline T ldg(const GLOBAL T *b, uint32_t i)
{
    return *(const GLOBAL T *)((const GLOBAL char *)b + i * (uint32_t)sizeof(T));
}

template <typename T>
__device__ inline void stg(GLOBAL T *b, uint32_t i, T v)
{
    *(GLOBAL T *)((GLOBAL char *)b + i * (uint32_t)sizeof(T)) = v;
}

template <typename T>
__device__ inline void addg(GLOBAL T *b, uint32_t i, T v)
{
    __hip_atomic_fetch_add((GLOBAL T *)((GLOBAL char *)b + i * (uint32_t)sizeof(T)), v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// One component of a structure-of-arrays field: the field's base and the
// component's first element.  All components share one scalar base, and an
// element's byte offset stays below 2^32 (the runtime bounds every field).
template <typename T>
struct Comp {
    GLOBAL T *base;
    uint32_t off;
};

template <typename T>
__device__ inline T ldg(const Comp<T> &c, uint32_t i)
{
    return ldg(c.base, c.off + i);
}

template <typename T>
__device__ inline void stg(const Comp<T> &c, uint32_t i, T v)
{
    stg(c.base, c.off + i, v);
}

template <typename T>
__device__ inline void addg(const Comp<T> &c, uint32_t i, T v)
{
    addg(c.base, c.off + i, v);
}

template <typename T>
__device__ inline int find_scene(const T *offs, int nscenes, int64_t g)
{
    // largest s with offs[s] <= g (offsets non-decreasing, offs[0] = 0)
    int lo = 0, hi = nscenes - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if ((int64_t)offs[mid] <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ inline uint32_t pack_cell(const int c[3])
{
    return (uint32_t)c[0] | ((uint32_t)c[1] << 11) | ((uint32_t)c[2] << 22);
}

__device__ inline void unpack_cell(uint32_t p, int c[3])
{
    c[0] = (int)(p & 2047u);
    c[1] = (int)((p >> 11) & 2047u);
    c[2] = (int)(p >> 22);
}

// Cells are grouped into bricks of 4^3 after a per-scene shift: brick
// coordinate (c + s) >> 2 per axis with s = (-cmin) & 3, cmin the smallest
// cell of the particles at creation, so that a block of particles starts a
// brick on its lower faces instead of leaving a row of underfilled bricks
// there.
__device__ inline int brick_shift(int cmin) { return (-cmin) & 3; }

__device__ inline void brick_origin(const SceneDev &S, uint32_t b, int o[3])
{
    o[0] = (int)(b % (uint32_t)S.nb[0]) * kBrick - brick_shift(S.cmin[0]);
    o[1] = (int)((b / (uint32_t)S.nb[0]) % (uint32_t)S.nb[1]) * kBrick - brick_shift(S.cmin[1]);
    o[2] = (int)(b / ((uint32_t)S.nb[0] * (uint32_t)S.nb[1])) * kBrick - brick_shift(S.cmin[2]);
}

// A per-scene constant in the state precision: the FP32 copy the host
// rounded once, or the FP64 value.
template <typename R>
__device__ inline R cst(double d, float f)
{
    if constexpr (sizeof(R) == 4)
        return f;
    else
        return (R)d;
}

// Cell of a position: floor((x - o) / h) with the IEEE FP64 quotient per
// axis.  The quotient is first estimated as (x - o) * (1/h), within a few ulp
// of it; only when the estimate lies that close to an integer (a cell face)
// is the division done, so the cell equals the one the exact quotient gives.
// Returns 0, ERR_OUT_OF_MESH or ERR_NONFINITE.
// With FRAC, also the position's local coordinate in its cell, (x - X_c)/h,
// as the estimate's fractional part (recomputed from X_c near a face).
template <bool FRAC = false>
__device__ inline uint32_t locate(const SceneDev &S, const double x[3], int c[3], double *frac = nullptr)
{
    if (!isfinite(x[0]) || !isfinite(x[1]) || !isfinite(x[2]))
        return ERR_NONFINITE;
    double d[3], t[3], f[3];
    bool near = false;
    for (int a = 0; a < 3; ++a) {
        d[a] = x[a] - S.origin[a];
        const double q = d[a] * S.inv_h;
        t[a] = floor(q);
        // the estimate is within 1e-12 of the quotient for |q| < 4096 (any
        // larger q is outside the mesh either way)
        f[a] = q - t[a];
        near = near || !(f[a] > 1e-11 && f[a] < 1.0 - 1e-11);
    }
    if (near)
        for (int a = 0; a < 3; ++a) {
            t[a] = floor(d[a] / S.h);
            if constexpr (FRAC)
                f[a] = (x[a] - (S.origin[a] + S.h * t[a])) * S.inv_h;
        }
    uint32_t out = 0;
    for (int a = 0; a < 3; ++a) {
        c[a] = (int)t[a];
        out |= (unsigned)c[a] >= (unsigned)S.n[a] ? 1u : 0u;
        if constexpr (FRAC)
            frac[a] = f[a];
    }
    return out ? ERR_OUT_OF_MESH : 0u;
}

// Node index (32-bit: the runtime bounds every node field below 2^32 bytes).
__device__ inline uint32_t node_id(const SceneDev &S, int i, int j, int k)
{
    const int g = S.ghost;
    return (uint32_t)((i + g) + S.N[0] * ((j + g) + S.N[1] * (k + g)));
}

__device__ inline bool node_in_mesh(const SceneDev &S, int i, int j, int k)
{
    const int g = S.ghost;
    return i >= -g && i <= S.n[0] + g && j >= -g && j <= S.n[1] + g && k >= -g && k <= S.n[2] + g;
}

// Components fixed by the face rules at node (i,j,k): bit a = component a.
__device__ inline uint32_t face_mask(const SceneDev &S, int i, int j, int k)
{
    const int idx[3] = {i, j, k};
    uint32_t m = 0;
    for (int b = 0; b < 3; ++b) {
        const uint32_t lo = idx[b] <= 0 ? (S.face_bits >> (4 * b)) & 3u : 0u;
        const uint32_t hi = idx[b] >= S.n[b] ? (S.face_bits >> (4 * b + 2)) & 3u : 0u;
        if (lo == 1u || hi == 1u)
            m = 7u;
        if (lo == 2u || hi == 2u)
            m |= 1u << b;
    }
    return m;
}

template <typename R>
struct alignas(4 * sizeof(R)) R4 {
    R x, y, z, w;
};

template <typename R>
struct alignas(2 * sizeof(R)) R2 {
    R s, t;
};

// Component arrays of one node buffer.
template <typename R>
struct NodeBuf {
    GLOBAL double *m;
    Comp<R> p[3];
    Comp<R> f[3];
};

template <typename R>
__device__ inline NodeBuf<R> node_buf(const SceneDev &S, int b)
{
    NodeBuf<R> nb;
    nb.m = gp(pick(S.nm, b));
    GLOBAL R *P = gp((R *)pick(S.np_, b));
    GLOBAL R *F = gp((R *)pick(S.nf, b));
    for (int a = 0; a < 3; ++a) {
        nb.p[a] = Comp<R>{P, (uint32_t)(a * S.nn)};
        nb.f[a] = Comp<R>{F, (uint32_t)(a * S.nn)};
    }
    return nb;
}

// Nodal velocity v = p / m (0 on void nodes) with velocity constraints, from
// the node's mass and momentum.
template <typename R>
__device__ inline void velocity_from_raw(const SceneDev &S, double m, const R p[3], int i, int j, int k, R v[3])
{
    const double inv = m > S.eps_m ? 1.0 / m : 0.0;   // void node: v = 0
    for (int a = 0; a < 3; ++a)
        v[a] = (R)((double)p[a] * inv);
    const uint32_t fm = face_mask(S, i, j, k);
    for (int a = 0; a < 3; ++a)
        if (fm & (1u << a))
            v[a] = (R)0;
    if (S.bc_mask) {
        const uint32_t I = node_id(S, i, j, k);
        const uint32_t em = gp(S.bc_mask)[I];
        for (int a = 0; a < 3; ++a)
            if (em & (1u << a))
                v[a] = (R)gp(S.bc_val)[3 * (size_t)I + a];
    }
}

template <typename R>
__device__ inline void node_velocity(const SceneDev &S, const NodeBuf<R> &nb, int i, int j, int k, R v[3])
{
    const uint32_t I = node_id(S, i, j, k);
    const R p[3] = {ldg(nb.p[0], I), ldg(nb.p[1], I), ldg(nb.p[2], I)};
    velocity_from_raw<R>(S, ldg(nb.m, I), p, i, j, k, v);
}

// Factor of the external nodal forces in the scene's current step n (the
// step control has counted it in CTL_STEPS): the smooth ramp u^2 (3 - 2u),
// u = n / force_ramp, and 1 from step force_ramp on.
__device__ inline double external_force_scale(const SceneDev &S)
{
    const int64_t n = (int64_t)__hip_atomic_load(&S.ctl[CTL_STEPS], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (S.force_ramp <= 0 || n >= S.force_ramp)
        return 1.0;
    const double u = (double)n / (double)S.force_ramp;
    return u * u * (3.0 - 2.0 * u);
}

// Nodal acceleration a = f / m and updated velocity vn = v + dt a, with the
// constraints applied to v (prescribed), a (zero) and vn (prescribed), from
// the node's mass, momentum and force.
template <typename R>
__device__ inline void update_from_raw(const SceneDev &S, double m, const R p[3], const R f[3], int i, int j, int k,
                                       R a[3], R vn[3])
{
    const double inv = m > S.eps_m ? 1.0 / m : 0.0;   // void node: v = a = 0
    uint32_t em = 0u;
    uint32_t I = 0u;
    if (S.bc_mask) {
        I = node_id(S, i, j, k);
        em = gp(S.bc_mask)[I];
    }
    // a node's external force (ramped over the scene's first steps) joins
    // the particles' sum before a = f / m; CTL_STEPS is the running step
    const double fs = (em & 8u) ? external_force_scale(S) : 0.0;
    R v[3];
    for (int c = 0; c < 3; ++c) {
        v[c] = (R)((double)p[c] * inv);
        const R fc = (em & 8u) ? f[c] + (R)(fs * gp(S.bc_force)[3 * (size_t)I + c]) : f[c];
        a[c] = (R)((double)fc * inv);
    }
    const uint32_t fm = face_mask(S, i, j, k);
    for (int c = 0; c < 3; ++c) {
        if (fm & (1u << c)) {
            v[c] = (R)0;
            a[c] = (R)0;
        }
        if (em & (1u << c)) {
            v[c] = (R)gp(S.bc_val)[3 * (size_t)I + c];
            a[c] = (R)0;
        }
    }
    const R dt = cst<R>(S.dt, S.f_dt);
    for (int c = 0; c < 3; ++c)
        vn[c] = v[c] + dt * a[c];
    for (int c = 0; c < 3; ++c) {
        if (fm & (1u << c))
            vn[c] = (R)0;
        if (em & (1u << c))
            vn[c] = (R)gp(S.bc_val)[3 * (size_t)I + c];
    }
}

template <typename R>
__device__ inline void node_update(const SceneDev &S, const NodeBuf<R> &nb, int i, int j, int k, R a[3], R vn[3])
{
    const uint32_t I = node_id(S, i, j, k);
    const R p[3] = {ldg(nb.p[0], I), ldg(nb.p[1], I), ldg(nb.p[2], I)};
    const R f[3] = {ldg(nb.f[0], I), ldg(nb.f[1], I), ldg(nb.f[2], I)};
    update_from_raw<R>(S, ldg(nb.m, I), p, f, i, j, k, a, vn);
}

// ------------------------------------------------------ shape functions --

// NS nodes per axis in a particle's support; a work item's node tile
// extends its cell box by lo nodes below and hi above; cap: tile nodes for a
// brick with one cell of drift on every side (7^3 linear, 9^3 GIMP).
template <int SH>
struct ShapeTraits;
template <>
struct ShapeTraits<0> {   // trilinear 8-node hexahedron
    static constexpr int NS = 2;
    static constexpr int lo = 0;
    static constexpr int hi = 1;
    static constexpr int cap = 343;
};
template <>
struct ShapeTraits<1> {   // uGIMP, particle half-length h/4, 27 nodes
    static constexpr int NS = 3;
    static constexpr int lo = 1;
    static constexpr int hi = 2;
    static constexpr int cap = 729;
};
template <>
struct ShapeTraits<2> {   // isoparametric trilinear 8-node hexahedron
    static constexpr int NS = 2;
    static constexpr int lo = 0;
    static constexpr int hi = 1;
    static constexpr int cap = 343;
};

// Shape function values w and one-axis derivatives dw of a particle's
// support nodes, per axis (tensor-product form).  Uniform linear and GIMP:
// dw is d/dx.  Isoparametric: the weights are those of the particle's local
// coordinates r in [0,1)^3 of its cell, dw is d/dr, and Ji = (dx/dr)^-1 at
// the particle turns d/dr into d/dx: dN/dx_b = sum_c dN/dr_c Ji[c][b].
template <typename R, int SH>
struct Support {
    int base[3];
    R w[3][ShapeTraits<SH>::NS];
    R dw[3][ShapeTraits<SH>::NS];
    R Ji[SH == 2 ? 3 : 1][SH == 2 ? 3 : 1];
};

// ------------------------------------------------ isoparametric cells --
// A cell of an isoparametric mesh (isoparametric-mesh section) is the
// trilinear image of its eight nodes over local coordinates r in [0,1]^3
// (r = (xi + 1) / 2 of the natural cube [-1,1]^3).  Relative to its first
// node o, x(r) = b1 r + b2 s + b3 t + b4 rs + b5 st + b6 rt + b7 rst
// (r, s, t the three local coordinates), in FP64.
struct IsoCell {
    double o[3];
    double b[7][3];
};

__device__ inline void iso_cell(const SceneDev &S, const int c[3], IsoCell &k)
{
    const uint32_t n0 = node_id(S, c[0], c[1], c[2]);
    const uint32_t ny = (uint32_t)S.N[0], nz = (uint32_t)(S.N[0] * S.N[1]), nn = (uint32_t)S.nn;
    const GLOBAL double *X = gp(S.X);
    double P[8][3];
    for (int q = 0; q < 8; ++q) {
        const uint32_t I = n0 + (uint32_t)(q & 1) + (uint32_t)((q >> 1) & 1) * ny + (uint32_t)(q >> 2) * nz;
        for (int a = 0; a < 3; ++a)
            P[q][a] = ldg(X, a * nn + I);
    }
    for (int a = 0; a < 3; ++a) {
        k.o[a] = P[0][a];
        const double p1 = P[1][a] - P[0][a], p2 = P[2][a] - P[0][a], p3 = P[3][a] - P[0][a];
        const double p4 = P[4][a] - P[0][a], p5 = P[5][a] - P[0][a], p6 = P[6][a] - P[0][a];
        const double p7 = P[7][a] - P[0][a];
        k.b[0][a] = p1;                       // r
        k.b[1][a] = p2;                       // s
        k.b[2][a] = p4;                       // t
        k.b[3][a] = p3 - p1 - p2;             // rs
        k.b[4][a] = p6 - p2 - p4;             // st
        k.b[5][a] = p5 - p1 - p4;             // rt
        k.b[6][a] = p7 - p3 - p5 - p6 + p1 + p2 + p4;   // rst
    }
}

// x(r) - o and the Jacobian J[a][c] = dx_a / dr_c.
__device__ inline void iso_eval(const IsoCell &k, const double r[3], double x[3], double J[3][3])
{
    const double rs = r[0] * r[1], st = r[1] * r[2], rt = r[0] * r[2];
    for (int a = 0; a < 3; ++a) {
        x[a] = k.b[0][a] * r[0] + k.b[1][a] * r[1] + k.b[2][a] * r[2] + k.b[3][a] * rs + k.b[4][a] * st +
               k.b[5][a] * rt + k.b[6][a] * rs * r[2];
        J[a][0] = k.b[0][a] + k.b[3][a] * r[1] + k.b[5][a] * r[2] + k.b[6][a] * st;
        J[a][1] = k.b[1][a] + k.b[3][a] * r[0] + k.b[4][a] * r[2] + k.b[6][a] * rt;
        J[a][2] = k.b[2][a] + k.b[4][a] * r[1] + k.b[5][a] * r[0] + k.b[6][a] * rs;
    }
}

__device__ inline void inverse3(const double M[3][3], double Mi[3][3])
{
    const double c00 = M[1][1] * M[2][2] - M[1][2] * M[2][1];
    const double c01 = M[1][2] * M[2][0] - M[1][0] * M[2][2];
    const double c02 = M[1][0] * M[2][1] - M[1][1] * M[2][0];
    const double id = 1.0 / (M[0][0] * c00 + M[0][1] * c01 + M[0][2] * c02);
    Mi[0][0] = c00 * id;
    Mi[1][0] = c01 * id;
    Mi[2][0] = c02 * id;
    Mi[0][1] = (M[0][2] * M[2][1] - M[0][1] * M[2][2]) * id;
    Mi[1][1] = (M[0][0] * M[2][2] - M[0][2] * M[2][0]) * id;
    Mi[2][1] = (M[0][1] * M[2][0] - M[0][0] * M[2][1]) * id;
    Mi[0][2] = (M[0][1] * M[1][2] - M[0][2] * M[1][1]) * id;
    Mi[1][2] = (M[0][2] * M[1][0] - M[0][0] * M[1][2]) * id;
    Mi[2][2] = (M[0][0] * M[1][1] - M[0][1] * M[1][0]) * id;
}

// Local coordinates r of the point o + y in the cell: Newton-Raphson on
// x(r) = y from the affine guess r0 = 1/2 + J(1/2)^-1 (y - x(1/2)), stopping
// after a correction of at most 5e-13 (1e-12 in natural coordinates; the
// error left is of the order of its square).  False if it broke down.
__device__ inline bool iso_local(const IsoCell &k, const double y[3], double r[3])
{
    double xm[3], J[3][3], Ji[3][3];
    const double c[3] = {0.5, 0.5, 0.5};
    iso_eval(k, c, xm, J);
    inverse3(J, Ji);
    for (int a = 0; a < 3; ++a)
        r[a] = 0.5 + Ji[a][0] * (y[0] - xm[0]) + Ji[a][1] * (y[1] - xm[1]) + Ji[a][2] * (y[2] - xm[2]);
    for (int it = 0; it < 50; ++it) {
        iso_eval(k, r, xm, J);
        inverse3(J, Ji);
        double dmax = 0.0;
        double d[3];
        for (int a = 0; a < 3; ++a)
            d[a] = Ji[a][0] * (xm[0] - y[0]) + Ji[a][1] * (xm[1] - y[1]) + Ji[a][2] * (xm[2] - y[2]);
        for (int a = 0; a < 3; ++a) {
            r[a] -= d[a];
            dmax = fmax(dmax, fabs(d[a]));
        }
        if (!(dmax > 5e-13))   // converged, or not a number (the check below fails)
            break;
    }
    return isfinite(r[0]) && isfinite(r[1]) && isfinite(r[2]);
}

// Cell of point x on an isoparametric mesh by a walk across cell faces from
// cell c (updated in place; the particle's previous cell, or a first guess)
// towards the point, at most `budget` cells: the cell whose local
// coordinates of x lie in [0,1)^3 (the uniform mesh's half-open rule), its
// geometry k and the local coordinates r.  A point that rounding leaves
// just past a face between two cells (by at most 5e-13, never past the
// mesh's outer faces) goes to the one it overshoots least.  Returns 0 or
// ERR_OUT_OF_MESH / ERR_NONFINITE.
__device__ inline uint32_t iso_locate(const SceneDev &S, const double x[3], int c[3], double r[3], IsoCell &k,
                                      int budget)
{
    if (!isfinite(x[0]) || !isfinite(x[1]) || !isfinite(x[2]))
        return ERR_NONFINITE;
    int best[3] = {-1, 0, 0}, prev[3] = {-1, -1, -1};
    double bover = 1.0, br[3] = {0.0, 0.0, 0.0};
    for (int m = 0; m < budget; ++m) {
        iso_cell(S, c, k);
        const double y[3] = {x[0] - k.o[0], x[1] - k.o[1], x[2] - k.o[2]};
        if (!iso_local(k, y, r))
            break;
        int d[3];
        bool in = true, outer = false;
        double over = -1.0;
        for (int a = 0; a < 3; ++a) {
            d[a] = r[a] < 0.0 ? -1 : (r[a] >= 1.0 ? 1 : 0);
            in = in && d[a] == 0;
            over = fmax(over, fmax(-r[a], r[a] - 1.0));
            outer = outer || (unsigned)(c[a] + d[a]) >= (unsigned)S.n[a];
        }
        if (in)
            return 0u;
        if (!outer && over <= 5e-13 && over < bover) {
            bover = over;
            for (int a = 0; a < 3; ++a) {
                best[a] = c[a];
                br[a] = r[a];
            }
        }
        if (outer)
            break;
        const int nx[3] = {c[0] + d[0], c[1] + d[1], c[2] + d[2]};
        if (nx[0] == prev[0] && nx[1] == prev[1] && nx[2] == prev[2])
            break;   // back and forth across one face
        for (int a = 0; a < 3; ++a) {
            prev[a] = c[a];
            c[a] = nx[a];
        }
    }
    if (best[0] < 0)
        return ERR_OUT_OF_MESH;
    for (int a = 0; a < 3; ++a) {
        c[a] = best[a];
        r[a] = br[a];
    }
    iso_cell(S, c, k);
    return 0u;
}

// ---------------------------------------- anchored GIMP scatter layout --
// A GIMP particle's 3-node support per axis starts at its cell c - 1 or c.
// Scattered as it stands, two lanes of a wavefront in neighbouring cells can
// add to the same node in the same LDS atomic (whenever one support starts
// at c and the other at c' - 1 = c), and the LDS unit serializes them.  The
// anchored form gives every particle the 4 nodes c - 1 .. c + 2 per axis
// (4^3 = 64 slots), with weight 0 at the end its support does not reach:
// the lanes of a level-major wavefront hold distinct cells, so for one slot
// they add to distinct nodes.  With the accumulators laid out at row and
// plane pitches of 12 and 108 entries (FP64) the adds are also free of bank
// conflicts.  Measured on a probe of this pattern: 8.3 cycles per
// wavefront-wide FP64 LDS add (2121 per 64 particles) against 31.5 (3407)
// for the 27-slot form.
// The rotated form keeps 27 slots and takes them in an order that mostly
// avoids the collisions: on each axis slots 0 and 1 are the nodes c and
// c + 1 for every lane, and slot 2 is c + 2 or c - 1 as the support
// requires.  Only slots 2 mix two translates: 16.7 cycles per add on the
// same layout (1806 per 64 particles), with 27/64 of the anchored form's
// arithmetic.  It suits the force scatter, whose anchored form is
// VALU-bound; two particles of one cell cannot share its adds.
constexpr int kAnchPX = 12, kAnchPXY = 108, kAnchCap = 972;   // 12 x 9 x 9 entries

// The 4 anchored weights (and their derivatives) of one axis from a 3-node
// support that starts at cell c (d = 1) or c - 1 (d = 0).
template <typename R>
__device__ inline void anchor4(const R w[3], const R dw[3], int d, R w4[4], R dw4[4])
{
    w4[0] = d ? (R)0 : w[0];
    w4[1] = d ? w[0] : w[1];
    w4[2] = d ? w[1] : w[2];
    w4[3] = d ? w[2] : (R)0;
    dw4[0] = d ? (R)0 : dw[0];
    dw4[1] = d ? dw[0] : dw[1];
    dw4[2] = d ? dw[1] : dw[2];
    dw4[3] = d ? dw[2] : (R)0;
}

// The rotated slot order of one axis (see kAnchPX) from a 3-node support
// that starts at cell c (up) or c - 1: weights and derivatives of the nodes
// c, c + 1, then c + 2 (up) or c - 1; returns the last slot's offset from
// node c - 1.
template <typename R>
__device__ inline int rotate3(const R w[3], const R dw[3], bool up, R wr[3], R dr[3])
{
    wr[0] = up ? w[0] : w[1];
    wr[1] = up ? w[1] : w[2];
    wr[2] = up ? w[2] : w[0];
    dr[0] = up ? dw[0] : dw[1];
    dr[1] = up ? dw[1] : dw[2];
    dr[2] = up ? dw[2] : dw[0];
    return up ? 3 : 0;
}

// Cells a per-step location walk may visit: a particle moves less than a
// cell per step (CFL), so it ends in its cell or a neighbour of it.
constexpr int kIsoWalk = 8;

// Support of a particle at local coordinates r of cell c (geometry k).
template <typename R>
__device__ inline void iso_support(const IsoCell &k, const int c[3], const double r[3], Support<R, 2> &sp)
{
    for (int a = 0; a < 3; ++a) {
        sp.base[a] = c[a];
        sp.w[a][0] = (R)(1.0 - r[a]);
        sp.w[a][1] = (R)r[a];
        sp.dw[a][0] = (R)-1;
        sp.dw[a][1] = (R)1;
    }
    double xm[3], J[3][3], Ji[3][3];
    iso_eval(k, r, xm, J);
    inverse3(J, Ji);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            sp.Ji[a][b] = (R)Ji[a][b];
}

// Gradient (d/dx) of a support node's shape function from its d/dr.
template <typename R, int SH>
__device__ inline void to_dx(const Support<R, SH> &sp, R &gx, R &gy, R &gz)
{
    if constexpr (SH == 2) {
        const R a = gx, b = gy, c = gz;
        gx = a * sp.Ji[0][0] + b * sp.Ji[1][0] + c * sp.Ji[2][0];
        gy = a * sp.Ji[0][1] + b * sp.Ji[1][1] + c * sp.Ji[2][1];
        gz = a * sp.Ji[0][2] + b * sp.Ji[1][2] + c * sp.Ji[2][2];
    }
}

// 1-D uGIMP weight for offset rho = (x_p - X_I)/h with lh = l/h = 1/4: the
// linear hat averaged over the particle's domain [x_p - l, x_p + l].
template <typename R>
__device__ inline void gimp1(R rho, R &S, R &dS)
{
    const R lh = (R)0.25;
    const R a = fabs(rho);
    const R s = rho < (R)0 ? (R)-1 : (R)1;
    if (a < lh) {
        S = (R)1 - (rho * rho + lh * lh) / ((R)2 * lh);
        dS = -rho / lh;
    } else if (a < (R)1 - lh) {
        S = (R)1 - a;
        dS = -s;
    } else if (a < (R)1 + lh) {
        const R d = (R)1 + lh - a;
        S = d * d / ((R)4 * lh);
        dS = -s * d / ((R)2 * lh);
    } else {
        S = (R)0;
        dS = (R)0;
    }
}

template <typename R, int SH>
__device__ inline void make_support(const SceneDev &S, const double x[3], const int c[3], Support<R, SH> &sp)
{
    const double h = S.h, ih = S.inv_h;
    const R inv_h = cst<R>(S.inv_h, S.f_inv_h);
    if constexpr (SH == 2) {
        IsoCell k;
        iso_cell(S, c, k);
        const double y[3] = {x[0] - k.o[0], x[1] - k.o[1], x[2] - k.o[2]};
        double r[3];
        iso_local(k, y, r);
        iso_support<R>(k, c, r, sp);
    } else if constexpr (SH == 0) {
        for (int a = 0; a < 3; ++a) {
            const R r = (R)((x[a] - (S.origin[a] + h * (double)c[a])) * ih);
            sp.base[a] = c[a];
            sp.w[a][0] = (R)1 - r;
            sp.w[a][1] = r;
            sp.dw[a][0] = -inv_h;
            sp.dw[a][1] = inv_h;
        }
    } else {
        const double l = 0.25 * h;
        for (int a = 0; a < 3; ++a) {
            // support starts at c-1 or c; the weight of the node it would
            // otherwise include is zero, so rounding here cannot matter
            const int i0 = (int)floor((x[a] - S.origin[a] - l) * ih);
            sp.base[a] = i0;
            for (int t = 0; t < 3; ++t) {
                const R rho = (R)((x[a] - (S.origin[a] + h * (double)(i0 + t))) * ih);
                R w, d;
                gimp1(rho, w, d);
                sp.w[a][t] = w;
                sp.dw[a][t] = d * inv_h;
            }
        }
    }
}

// --------------------------------------------------------- constitutive --

template <typename R>
__device__ inline void constitutive(const SceneDev &S, const R de[6], R sig[6])
{
    const R lam = cst<R>(S.lam, S.f_lam), G = cst<R>(S.G, S.f_G);
    const R tr = de[0] + de[1] + de[2];
    for (int a = 0; a < 3; ++a)
        sig[a] += lam * tr + (R)2 * G * de[a];
    for (int a = 3; a < 6; ++a)
        sig[a] += G * de[a];
    if (S.model != 1)
        return;
    // Drucker-Prager, perfectly plastic: f = sqrt(J2) + eta p - xi c.
    const R K = cst<R>(S.K, S.f_K), eta = cst<R>(S.eta, S.f_eta), etab = cst<R>(S.etab, S.f_etab);
    constexpr bool F32 = sizeof(R) == 4;
    const R p = F32 ? (sig[0] + sig[1] + sig[2]) * (R)(1.0 / 3.0) : (sig[0] + sig[1] + sig[2]) / (R)3;
    R s[6];
    for (int a = 0; a < 3; ++a)
        s[a] = sig[a] - p;
    for (int a = 3; a < 6; ++a)
        s[a] = sig[a];
    const R J2 = (R)0.5 * (s[0] * s[0] + s[1] * s[1] + s[2] * s[2]) + s[3] * s[3] + s[4] * s[4] + s[5] * s[5];
    // FP32: the hardware square root and reciprocal (about 1 ulp) in place
    // of the correctly rounded sequences
    R q;
    if constexpr (F32)
        q = __builtin_amdgcn_sqrtf(J2);
    else
        q = sqrt(J2);
    const R f = q + eta * p - cst<R>(S.xic, S.f_xic);
    if (!(f > (R)0))
        return;
    const R dgam = F32 ? f * cst<R>(S.inv_hard, S.f_inv_hard) : f / (G + K * eta * etab);
    if (q - G * dgam >= (R)0) {
        R scale;
        if constexpr (F32)
            scale = (R)1 - G * dgam * __builtin_amdgcn_rcpf(q);
        else
            scale = (R)1 - G * dgam / q;
        const R pn = p - K * etab * dgam;
        for (int a = 0; a < 3; ++a)
            sig[a] = scale * s[a] + pn;
        for (int a = 3; a < 6; ++a)
            sig[a] = scale * s[a];
    } else {
        const R pa = S.has_apex ? cst<R>(S.apex_p, S.f_apex) : p;
        for (int a = 0; a < 3; ++a)
            sig[a] = pa;
        for (int a = 3; a < 6; ++a)
            sig[a] = (R)0;
    }
}

// -------------------------------------------------------- scene lookup --

// Wave-uniform copies of values loaded through vector memory: the compiler
// then keeps them in scalar registers and forms addresses as a scalar base
// plus a 32-bit vector offset.
__device__ inline uint32_t uni(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

template <typename T>
__device__ inline T *uni(T *p)
{
    const uint64_t v = (uint64_t)p;
    return (T *)(((uint64_t)uni((uint32_t)(v >> 32)) << 32) | (uint64_t)uni((uint32_t)v));
}

// Load through the scalar cache: the address is wave-uniform and the data
// does not change during the kernel (written at creation or by an earlier
// kernel).
template <typename T>
__device__ inline T cld(const T *p)
{
    return *(const __attribute__((address_space(4))) T *)uni(p);
}

// The same for a plain struct, word by word.
template <typename T>
__device__ inline T cld_struct(const T *p)
{
    static_assert(sizeof(T) % 4 == 0, "word-sized struct");
    typedef const __attribute__((address_space(4))) uint32_t CWord;
    CWord *src = (CWord *)uni(p);
    T out;
    uint32_t *dst = (uint32_t *)&out;
    for (int w = 0; w < (int)(sizeof(T) / 4); ++w)
        dst[w] = src[w];
    return out;
}

// Largest s with offs[s] <= g for a wave-uniform g (offs non-decreasing),
// through the scalar cache: a work item's scene is found in a few scalar
// loads, not a chain of vector memory round trips.
template <typename T>
__device__ inline int find_scene_u(const T *offs, int nscenes, int64_t g)
{
    int lo = 0, hi = nscenes - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((int64_t)cld(&offs[mid]) <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Scene descriptor through the scalar cache: it is written once at creation
// and never changes afterwards.
__device__ inline SceneDev load_scene(const SceneDev *p)
{
    static_assert(sizeof(SceneDev) % 4 == 0, "word-sized struct");
    typedef const __attribute__((address_space(4))) uint32_t CWord;
    CWord *src = (CWord *)uni(p);
    SceneDev out;
    uint32_t *dst = (uint32_t *)&out;
    for (int w = 0; w < (int)(sizeof(SceneDev) / 4); ++w)
        dst[w] = src[w];
    return out;
}

struct ItemRef {
    const SceneDev *S;
    int it;
};

__device__ inline ItemRef item_ref(const uint32_t *offs, const BatchDev &B, int64_t g)
{
    const int s = find_scene_u(offs, B.nscenes, g);
    return {cld(&B.scenes[s]), (int)(uint32_t)(g - (int64_t)cld(&offs[s]))};
}

// The stage kernels after the step control test CTL_ACTIVE only: it is fixed
// for the whole step, whereas CTL_ERR may be raised by another workgroup of
// the same kernel, and every thread of a workgroup must take the same branch
// around its barriers.
__device__ inline bool scene_active(const SceneDev &S)
{
    return cld(&S.ctl[CTL_ACTIVE]) != 0u;
}

// Item order of the persistent grids.  Workgroup w runs on XCD w % 8, and
// each XCD has its own L2; the XCDs get contiguous ranges of the item list,
// so bricks that share node rows (consecutive items) are processed under one
// L2 rather than fetched into several.  A grid that is not a multiple of 8
// strides over the whole list.
struct ItemRange {
    int64_t first, step, end;
};

__device__ inline ItemRange item_range(int64_t total)
{
    const int nx = (gridDim.x % kXcds == 0) ? kXcds : 1;
    const int64_t per = gridDim.x / nx;
    const int64_t chunk = (total + nx - 1) / nx;
    const int64_t lo = (int64_t)(blockIdx.x % nx) * chunk;
    return {lo + blockIdx.x / nx, per, min(total, lo + chunk)};
}

template <int SH>
__device__ inline Tile tile_of_cells(const int lo[3], const int hi[3])
{
    Tile t;
    for (int a = 0; a < 3; ++a) {
        t.lo[a] = lo[a] - ShapeTraits<SH>::lo;
        t.dim[a] = hi[a] >= lo[a] ? hi[a] + ShapeTraits<SH>::hi - t.lo[a] + 1 : 0;
    }
    const int vol = t.dim[0] * t.dim[1] * t.dim[2];
    t.fits = vol <= ShapeTraits<SH>::cap ? 1 : 0;
    t.pad = 0;
    return t;
}

// LDS node tile of the next step's scatter in g2p_p2g: the nodes supporting
// the cells of the item's brick widened by one cell on every side (the
// reorder keeps every particle of the item there, except between a drift
// past it and the next reorder).
template <int SH>
__device__ inline Tile home_tile(const int o[3])
{
    Tile t;
    for (int a = 0; a < 3; ++a) {
        t.lo[a] = o[a] - 1 - ShapeTraits<SH>::lo;
        t.dim[a] = kBrick + 2 + ShapeTraits<SH>::lo + ShapeTraits<SH>::hi;
    }
    t.fits = 1;
    t.pad = 0;
    return t;
}

__device__ inline bool in_home(const int c[3], const int o[3])
{
    return c[0] >= o[0] - 1 && c[0] <= o[0] + kBrick && c[1] >= o[1] - 1 && c[1] <= o[1] + kBrick &&
           c[2] >= o[2] - 1 && c[2] <= o[2] + kBrick;
}

__device__ inline void tile_node(const Tile &t, int q, int &i, int &j, int &k)
{
    i = t.lo[0] + q % t.dim[0];
    j = t.lo[1] + (q / t.dim[0]) % t.dim[1];
    k = t.lo[2] + q / (t.dim[0] * t.dim[1]);
}

// Index of a particle's first support node in a tile and in the node array;
// corner (i,j,k) then adds i + j*sy + k*sz with the strides below.
struct Corners {
    int t0, ty, tz;   // tile
    uint32_t n0;
    int ny, nz;       // node array
};

__device__ inline Corners corners(const SceneDev &S, const Tile &t, const int base[3])
{
    Corners c;
    c.ty = t.dim[0];
    c.tz = t.dim[0] * t.dim[1];
    c.t0 = (base[0] - t.lo[0]) + c.ty * (base[1] - t.lo[1]) + c.tz * (base[2] - t.lo[2]);
    c.ny = S.N[0];
    c.nz = S.N[0] * S.N[1];
    c.n0 = node_id(S, base[0], base[1], base[2]);
    return c;
}

// ------------------------------------------------------ tile helpers --

// Node (i, j, k) of entry q < 2^20 of a tile, the quotients taken through a
// float reciprocal: (q + 0.5) / d lies at least 0.5 / d from an integer, and
// the float product is within 2^-21 q / d of it, so the truncation is exact.
__device__ inline void tile_node_small(const Tile &t, int q, int &i, int &j, int &k)
{
    const int dxy = t.dim[0] * t.dim[1];
    const int kq = (int)(((float)q + 0.5f) * __builtin_amdgcn_rcpf((float)dxy));
    const int r = q - kq * dxy;
    const int jq = (int)(((float)r + 0.5f) * __builtin_amdgcn_rcpf((float)t.dim[0]));
    i = t.lo[0] + r - jq * t.dim[0];
    j = t.lo[1] + jq;
    k = t.lo[2] + kq;
}

// Wave-wide min / max through DPP lane moves (every lane active); the result
// is wave-uniform.
template <bool MAX>
__device__ inline int wave_reduce(int v)
{
    auto op = [](int a, int b) { return MAX ? max(a, b) : min(a, b); };
    v = op(v, __builtin_amdgcn_update_dpp(v, v, 0xb1, 0xf, 0xf, false));    // quad_perm [1,0,3,2]
    v = op(v, __builtin_amdgcn_update_dpp(v, v, 0x4e, 0xf, 0xf, false));    // quad_perm [2,3,0,1]
    v = op(v, __builtin_amdgcn_update_dpp(v, v, 0x141, 0xf, 0xf, false));   // row_half_mirror
    v = op(v, __builtin_amdgcn_update_dpp(v, v, 0x140, 0xf, 0xf, false));   // row_mirror
    v = op(v, __builtin_amdgcn_update_dpp(v, v, 0x142, 0xa, 0xf, false));   // row_bcast:15
    v = op(v, __builtin_amdgcn_update_dpp(v, v, 0x143, 0xc, 0xf, false));   // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

// Workgroup-wide cell box of the threads' mn/mx (every thread calls it);
// red holds 6 words per wave.
template <int T>
__device__ inline void item_box(const int mn[3], const int mx[3], int *red, int lo[3], int hi[3])
{
    for (int a = 0; a < 3; ++a) {
        lo[a] = wave_reduce<false>(mn[a]);
        hi[a] = wave_reduce<true>(mx[a]);
    }
    if constexpr (T > 64) {
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0)
            for (int a = 0; a < 3; ++a) {
                red[6 * w + a] = lo[a];
                red[6 * w + 3 + a] = hi[a];
            }
        __syncthreads();
        for (int v = 0; v < T / 64; ++v)
            for (int a = 0; a < 3; ++a) {
                lo[a] = min(lo[a], red[6 * v + a]);
                hi[a] = max(hi[a], red[6 * v + 3 + a]);
            }
        __syncthreads();
    }
}

// Zero node buffer `buf` over the given node box.
template <typename R>
__device__ inline void clear_box(const SceneDev &S, const NodeBuf<R> &nb, const Tile &t)
{
    const int vol = t.dim[0] * t.dim[1] * t.dim[2];
    for (int q = threadIdx.x; q < vol; q += blockDim.x) {
        int i, j, k;
        if (t.fits)
            tile_node_small(t, q, i, j, k);
        else
            tile_node(t, q, i, j, k);
        const uint32_t I = node_id(S, i, j, k);
        stg(nb.m, I, 0.0);
        for (int a = 0; a < 3; ++a) {
            stg(nb.p[a], I, (R)0);
            stg(nb.f[a], I, (R)0);
        }
    }
}

// Zero the other node buffer of every active scene over the boxes recorded
// when it was filled (the previous step's data).
template <typename R>
__device__ inline void clear_previous(const BatchDev &B)
{
    const int64_t total = B.coffs[B.nscenes];
    const ItemRange ir = item_range(total);
    for (int64_t g = ir.first; g < ir.end; g += ir.step) {
        const ItemRef r = item_ref(B.coffs, B, g);
        const SceneDev S = load_scene(r.S);
        if (!scene_active(S))
            continue;
        const int other = (int)cld(&S.ctl[CTL_NBUF]) ^ 1;
        clear_box<R>(S, node_buf<R>(S, other), cld_struct(&pick(S.tiles, other)[r.it]));
    }
}

// MUSL: zero the remap array of every active MUSL scene over the boxes of
// the other node buffer's items, the only nodes the previous step's remap
// wrote.
template <typename R>
__device__ inline void clear_remap_previous(const BatchDev &B)
{
    const int64_t total = B.coffs[B.nscenes];
    const ItemRange ir = item_range(total);
    for (int64_t g = ir.first; g < ir.end; g += ir.step) {
        const ItemRef r = item_ref(B.coffs, B, g);
        const SceneDev S = load_scene(r.S);
        if (!scene_active(S) || !S.nr)
            continue;
        const int other = (int)cld(&S.ctl[CTL_NBUF]) ^ 1;
        const Tile t = cld_struct(&pick(S.tiles, other)[r.it]);
        GLOBAL R *NR = gp((R *)S.nr);
        const uint32_t nn = (uint32_t)S.nn;
        const int vol = t.dim[0] * t.dim[1] * t.dim[2];
        for (int q = threadIdx.x; q < vol; q += blockDim.x) {
            int i, j, k;
            if (t.fits)
                tile_node_small(t, q, i, j, k);
            else
                tile_node(t, q, i, j, k);
            const uint32_t I = node_id(S, i, j, k);
            for (int a = 0; a < 3; ++a)
                stg(NR, a * nn + I, (R)0);
        }
    }
}

// ----------------------------------------------------- load / read out --

// Inputs are row-major doubles (n x 3, n x 6, n); fills particle buffer 0,
// sets the identity permutation and each particle's cell.
template <typename R>
__global__ void k_load(SceneDev *Sd, const double *x, const double *v, const double *sig, const double *vol,
                       const double *mass)
{
    const SceneDev &S = *Sd;
    const int64_t n = S.np;
    double *X = S.x[0];
    R *V = (R *)S.v[0];
    R *SG = (R *)S.sig[0];
    R *VO = (R *)S.vol[0];
    R *M = (R *)S.mass[0];
    int mn[3] = {INT_MAX, INT_MAX, INT_MAX};
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        double xp[3];
        bool fin = true;
        for (int a = 0; a < 3; ++a) {
            xp[a] = x[3 * p + a];
            X[a * n + p] = xp[a];
            V[a * n + p] = (R)v[3 * p + a];
            fin = fin && isfinite(v[3 * p + a]);
        }
        for (int k = 0; k < 6; ++k) {
            const double s = sig ? sig[6 * p + k] : 0.0;
            SG[k * n + p] = (R)s;
            fin = fin && isfinite(s);
        }
        VO[p] = (R)vol[p];
        M[p] = (R)mass[p];
        fin = fin && isfinite(vol[p]) && isfinite(mass[p]);
        int c[3] = {0, 0, 0};
        uint32_t e;
        if (S.X) {
            // isoparametric: walk from the cell of the uniform grid (origin,
            // h) the mesh was made from, clamped to the mesh
            for (int a = 0; a < 3; ++a) {
                const double q = floor((xp[a] - S.origin[a]) * S.inv_h);
                c[a] = q < 0.0 ? 0 : (q >= (double)S.n[a] ? S.n[a] - 1 : (int)q);
            }
            double r[3];
            IsoCell k;
            e = iso_locate(S, xp, c, r, k, S.n[0] + S.n[1] + S.n[2] + kIsoWalk);
        } else {
            e = locate(S, xp, c);
        }
        if (!fin)
            e |= ERR_NONFINITE;
        if (e) {
            atomicOr(&S.ctl[CTL_ERR], e);
            c[0] = c[1] = c[2] = 0;
        }
        S.cell[0][p] = pack_cell(c);
        S.pid[0][p] = (uint32_t)p;
        if (!e)
            for (int a = 0; a < 3; ++a)
                mn[a] = min(mn[a], c[a]);
    }
    // the smallest cell per axis (sets the brick shift): one atomic per wave
    for (int a = 0; a < 3; ++a) {
        const int w = wave_reduce<false>(mn[a]);
        if ((threadIdx.x & 63) == 0 && w != INT_MAX)
            atomicMin(&Sd->cmin[a], w);
    }
}

// Particle state in original order (row-major doubles); any pointer may be null.
template <typename R>
__global__ void k_read_out(const SceneDev *Sd, double *x, double *v, double *sig, double *vol, int32_t *cell)
{
    const SceneDev &S = *Sd;
    const int64_t n = S.np;
    const int cur = (int)cld(&S.ctl[CTL_CUR]);
    const double *X = S.x[cur];
    const R *V = (const R *)S.v[cur];
    const R *SG = (const R *)S.sig[cur];
    const R *VO = (const R *)S.vol[cur];
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = S.pid[cur][p];
        if (x)
            for (int a = 0; a < 3; ++a)
                x[3 * o + a] = X[a * n + p];
        if (v)
            for (int a = 0; a < 3; ++a)
                v[3 * o + a] = (double)V[a * n + p];
        if (sig)
            for (int k = 0; k < 6; ++k)
                sig[6 * o + k] = (double)SG[k * n + p];
        if (vol)
            vol[o] = (double)VO[p];
        if (cell) {
            int c[3];
            unpack_cell(S.cell[cur][p], c);
            cell[o] = c[0] + S.n[0] * (c[1] + S.n[1] * c[2]);
        }
    }
}

__global__ void k_cell_counts(const SceneDev *Sd, uint32_t *counts)
{
    const SceneDev &S = *Sd;
    const int cur = (int)cld(&S.ctl[CTL_CUR]);
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < S.np; p += (int64_t)gridDim.x * blockDim.x) {
        int c[3];
        unpack_cell(S.cell[cur][p], c);
        atomicAdd(&counts[c[0] + (int64_t)S.n[0] * (c[1] + (int64_t)S.n[1] * c[2])], 1u);
    }
}

// Nodal fields of the last completed step (node buffer CTL_NBUF).
template <typename R>
__global__ void k_nodes_out(const SceneDev *Sd, double *m, double *p, double *f)
{
    const SceneDev &S = *Sd;
    const int b = (int)cld(&S.ctl[CTL_NBUF]);
    const R *P = (const R *)S.np_[b];
    const R *F = (const R *)S.nf[b];
    for (int64_t I = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; I < S.nn; I += (int64_t)gridDim.x * blockDim.x) {
        if (m)
            m[I] = S.nm[b][I];
        const bool ext = S.bc_mask && (S.bc_mask[I] & 8u);
        const double fs = ext ? external_force_scale(S) : 0.0;
        for (int a = 0; a < 3; ++a) {
            if (p)
                p[3 * I + a] = (double)P[a * S.nn + I];
            if (f)   // the particles' sum plus the node's external force, as the update uses it
                f[3 * I + a] = (double)(ext ? F[a * S.nn + I] + (R)(fs * S.bc_force[3 * I + a]) : F[a * S.nn + I]);
        }
    }
}

// ------------------------------------------------------- step control --

// Start of a call: steps to run per scene, and whether any scene starts with
// a reorder pending (a fresh scene always does).
__global__ void k_begin(BatchDev B, const int64_t *nsteps)
{
    __shared__ int any;
    if (threadIdx.x == 0)
        any = 0;
    __syncthreads();
    for (int s = threadIdx.x; s < B.nscenes; s += blockDim.x) {
        const int64_t k = nsteps[s];
        uint32_t *ctl = B.scenes[s]->ctl;
        ctl[CTL_REMAIN] = (uint32_t)(k < 0 ? 0 : (k > 0x7fffffff ? 0x7fffffff : k));
        if (ctl[CTL_NEED_SORT] && ctl[CTL_ERR] == 0u && k > 0)
            any = 1;
    }
    __syncthreads();
    for (int w = threadIdx.x; w < BF_WORDS; w += blockDim.x)
        B.flags[w] = (w == BF_ANY_SORT && any) ? 1u : 0u;
}

// Per-step control, run by one workgroup: apply a finished reorder, decide
// which scenes take part in this step, pick their node buffers, and write the
// offsets of this step's items (ioffs) and of the boxes to clear (coffs).
// Each thread handles one scene through one read and one write of its
// 64-byte control block (no other kernel runs meanwhile), so the work is a
// short chain of memory round trips whatever the number of scenes.
__device__ void step_control(const BatchDev &B)
{
    __shared__ uint32_t wi[kBlock / 64], wc[kBlock / 64];
    __shared__ uint32_t carry[2];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool fail = __hip_atomic_load(&B.flags[BF_SORT_FAIL], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
    if (threadIdx.x == 0) {
        carry[0] = carry[1] = 0u;
        B.ioffs[0] = 0;
        B.coffs[0] = 0;
    }
    __syncthreads();
    for (int base = 0; base < B.nscenes; base += blockDim.x) {
        const int s = base + threadIdx.x;
        uint32_t items = 0, clears = 0;
        if (s < B.nscenes) {
            uint4 *blk = (uint4 *)B.ctls[s];
            uint32_t c[CTL_WORDS];
            for (int q = 0; q < CTL_WORDS / 4; ++q) {
                const uint4 w = blk[q];
                c[4 * q] = w.x;
                c[4 * q + 1] = w.y;
                c[4 * q + 2] = w.z;
                c[4 * q + 3] = w.w;
            }
            bool go = c[CTL_ERR] == 0u && c[CTL_REMAIN] > 0u;
            if (go && c[CTL_NEED_SORT] && fail) {   // its reorder was abandoned
                c[CTL_ERR] |= ERR_SORT;
                go = false;
            }
            const bool sorted = go && c[CTL_NEED_SORT];   // the reorder phases moved it
            if (sorted) {
                c[CTL_CUR] ^= 1u;
                c[CTL_NEED_SORT] = 0u;
                c[CTL_N_SORTS] += 1u;
            }
            c[CTL_ACTIVE] = go ? 1u : 0u;
            if (go) {
                c[CTL_REMAIN] -= 1u;
                c[CTL_STEPS] += 1u;
                if (c[CTL_ALGO] == 0u) {        // USF: the previous g2p_p2g filled the other buffer
                    if (c[CTL_READY]) {
                        c[CTL_NBUF] ^= 1u;
                        c[CTL_READY] = 0u;
                        c[CTL_HAVE_P2G] = 1u;
                        // its boxes belong to the items it ran, valid unless
                        // this step reordered the particles
                        c[CTL_BOX_OK] = sorted ? 0u : 1u;
                    } else {
                        c[CTL_HAVE_P2G] = 0u;
                        c[CTL_BOX_OK] = 1u;   // p2g records them after the reorder
                    }
                } else {                        // USL: p2g_usl fills a fresh buffer every step
                    c[CTL_NBUF] ^= 1u;
                    c[CTL_HAVE_P2G] = 0u;
                    c[CTL_BOX_OK] = 0u;
                }
                items = c[CTL_N_ITEMS];
                clears = c[CTL_NBUF] ? c[CTL_ACC0] : c[CTL_ACC1];   // boxes of the other buffer
            }
            for (int q = 0; q < CTL_WORDS / 4; ++q)
                blk[q] = uint4{c[4 * q], c[4 * q + 1], c[4 * q + 2], c[4 * q + 3]};
        }
        // inclusive scan over the workgroup: waves, then wave totals
        uint32_t si = items, sc = clears;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t ti = __shfl_up(si, o), tc = __shfl_up(sc, o);
            if (lane >= o) {
                si += ti;
                sc += tc;
            }
        }
        if (lane == 63) {
            wi[wave] = si;
            wc[wave] = sc;
        }
        __syncthreads();
        uint32_t pi = carry[0], pc = carry[1];
        for (int v = 0; v < wave; ++v) {
            pi += wi[v];
            pc += wc[v];
        }
        if (s < B.nscenes) {
            B.ioffs[s + 1] = pi + si;
            B.coffs[s + 1] = pc + sc;
        }
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) {
            carry[0] = pi + si;
            carry[1] = pc + sc;
        }
        __syncthreads();
    }
}

// Clear the batch's reorder words for the next step (run by the first
// workgroup of the stage kernel after the reorder, when every reorder
// workgroup has finished).
__device__ inline void clear_reorder_flags(const BatchDev &B)
{
    if (blockIdx.x == 0)
        for (int w = threadIdx.x; w < BF_WORDS; w += blockDim.x)
            B.flags[w] = 0u;
}

// ----------------------------------------------------------------- sort --
// The reorder runs as one launch of one workgroup per compute unit, in
// five phases: per-cell counts; per-brick cell scan with each brick range's
// partial sums of the scan over bricks; the rest of that scan (the carried
// prefix, every brick's start, the list of non-empty bricks); the
// permutation; and the move of the non-empty bricks.  Steps that reorder no
// scene skip straight to the step control, so they pay a single launch.
//
// Each phase is split into chunks that workgroups claim from a counter, and
// a phase is complete when every chunk is done.  A workgroup waits only once
// no chunk is left to claim, that is for chunks that running workgroups
// hold, so the reorder completes with any number of its workgroups resident
// (another kernel may hold part of the device).
//
// Every wavefront works on one scene at a time, whose descriptor fields are
// read through the scalar cache; the particle phases keep kSortU particles
// per lane in flight, the brick phase kBrickU bricks per wavefront, and the
// move kMoveLevels levels of a brick (half as many in FP64).  One 1024-thread
// workgroup per CU: every workgroup's fences write back and invalidate its
// XCD's L2, so fewer, larger workgroups wait less.

constexpr int kBrickU = 8;
constexpr int kMoveLevels = 4;
constexpr uint32_t kScanBricks = 64;   // fewest bricks per chunk of the brick phases

// Bound of a phase wait (1 s of the 100 MHz wall clock).  The wait always
// ends (see above); a workgroup that still gives up raises BF_SORT_FAIL
// before it reports any later chunk done.
constexpr uint64_t kBarrierTicks = 100000000ull;

// phases of the reorder, which index the claim and done counters
enum : int { PH_COUNT = 0, PH_BRICKS = 1, PH_SCAN = 2, PH_PERM = 3, PH_MOVE = 4 };

// Claim and run chunks of `phase` until none is left (work(c) runs only if
// `go`), then publish them and count them done.  A chunk is claimed only
// once the previous one is finished: claiming ahead would let the first
// workgroups take two chunks each while others got none.
template <typename F>
__device__ void run_chunks(uint32_t *flags, int phase, uint32_t nchunks, bool go, int *sh, F work)
{
    uint32_t *claim = &flags[BF_CLAIM + 32 * phase];
    uint32_t mine = 0;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0)
            *sh = (int)atomicAdd(claim, 1u);
        __syncthreads();
        const uint32_t c = (uint32_t)*sh;
        if (c >= nchunks)
            break;
        if (go)
            work(c);
        ++mine;
    }
    __syncthreads();
    if (threadIdx.x == 0 && mine) {
        __threadfence();   // publish this workgroup's chunks
        if (atomicAdd(&flags[BF_DONE + 32 * phase], mine) + mine == nchunks) {
            // the phase's last chunk: release every group of waiting workgroups
            __threadfence();
            const uint32_t ng = min(gridDim.x, (uint32_t)kXcds);
            for (uint32_t q = 0; q < ng; ++q)
                __hip_atomic_store(&flags[BF_RELEASE + 32 * q], (uint32_t)phase + 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Wait until every chunk of `phase` is done; returns whether the reorder may
// go on (no workgroup gave up).  Workgroups poll one release word per group
// (blockIdx mod 8, the XCD a workgroup runs on), which the workgroup that
// finished the phase's last chunk writes.  The flag is read after the
// wait, so a workgroup that goes on has seen every chunk of the phase run.
__device__ bool phase_done(uint32_t *flags, int phase, int *sh)
{
    if (threadIdx.x == 0) {
        const uint32_t g = blockIdx.x % min(gridDim.x, (uint32_t)kXcds);
        const uint64_t t0 = wall_clock64();
        while (__hip_atomic_load(&flags[BF_RELEASE + 32 * g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <=
               (uint32_t)phase) {
            if (wall_clock64() - t0 > kBarrierTicks) {
                atomicOr(&flags[BF_SORT_FAIL], 1u);
                break;
            }
            __builtin_amdgcn_s_sleep(8);
        }
        __threadfence();   // see the other workgroups' chunks
        *sh = __hip_atomic_load(&flags[BF_SORT_FAIL], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u;
    }
    __syncthreads();
    return *sh != 0;
}


// The reorder state of one scene, in scalar registers.
struct SortView {
    const SceneDev *S;
    GLOBAL const uint32_t *cell;   // packed cells, current buffer
    GLOBAL uint32_t *cnt, *cstart, *rank, *perm;
    GLOBAL uint32_t *bcnt, *bitem, *bstart, *istart;
    GLOBAL Item *items;
    GLOBAL uint32_t *ctl;
    uint32_t nb0, nb1;
    int sh[3];      // brick shift per axis
    uint32_t bo;    // flattened index of the scene's brick 0
    int cur;
    bool sorting;   // the scene reorders in the coming step
    __device__ uint32_t key(uint32_t packed) const
    {
        int c[3];
        unpack_cell(packed, c);
        for (int a = 0; a < 3; ++a)
            c[a] += sh[a];
        const uint32_t b = (uint32_t)(c[0] >> 2) + nb0 * ((uint32_t)(c[1] >> 2) + nb1 * (uint32_t)(c[2] >> 2));
        return b * 64u + (uint32_t)((c[0] & 3) + 4 * ((c[1] & 3) + 4 * (c[2] & 3)));
    }
};

__device__ inline SortView sort_view(const BatchDev &B, int s)
{
    SortView v;
    const SceneDev *S = cld(&B.scenes[s]);
    v.S = S;
    uint32_t *ctl = cld(&S->ctl);
    v.ctl = gp(ctl);
    v.cur = (int)cld(&ctl[CTL_CUR]);
    v.sorting = cld(&ctl[CTL_ERR]) == 0u && cld(&ctl[CTL_REMAIN]) > 0u && cld(&ctl[CTL_NEED_SORT]) != 0u;
    v.cell = gp((const uint32_t *)cld(&S->cell[v.cur]));
    v.cnt = gp(cld(&S->cnt));
    v.cstart = gp(cld(&S->cstart));
    v.rank = gp(cld(&S->rank));
    v.perm = gp(cld(&S->perm));
    v.bcnt = gp(cld(&S->bcnt));
    v.bitem = gp(cld(&S->bitem));
    v.bstart = gp(cld(&S->bstart));
    v.istart = gp(cld(&S->istart));
    v.items = gp(cld(&S->items));
    v.nb0 = (uint32_t)cld(&S->nb[0]);
    v.nb1 = (uint32_t)cld(&S->nb[1]);
    for (int a = 0; a < 3; ++a)
        v.sh[a] = brick_shift(cld(&S->cmin[a]));
    v.bo = (uint32_t)cld(&B.boffs[s]);
    return v;
}


// The particle phases: the flattened batch is cut into spans of 64 * kSortU
// consecutive particles, and chunk c of n takes spans c, c + n, c + 2n, ...
// (so the wavefronts running at one time work on distinct bricks, whose
// count atomics and slot stores then do not meet).  Each wavefront takes
// one span per pass and calls f(view, first, lo, hi, off) once per
// reordering scene the span meets; lane l's particles are
// first + u * 64 + l (u < kSortU), those in [lo, hi) belong to the scene,
// whose particle 0 is flattened index off.
constexpr int64_t kSpan = 64 * kSortU;

template <typename F>
__device__ inline void particle_spans(const BatchDev &B, uint32_t chunk, uint32_t nchunks, F f)
{
    const int64_t wave = uni(threadIdx.x >> 6), nw = blockDim.x >> 6;
    for (int64_t first = (chunk + nchunks * wave) * kSpan; first < B.total_particles; first += nchunks * nw * kSpan) {
        const int64_t end = min(first + kSpan, B.total_particles);
        int s = find_scene_u(B.poffs, B.nscenes, first);
        for (int64_t lo = first; lo < end; ++s) {
            const int64_t off = cld(&B.poffs[s]), hi = min(end, cld(&B.poffs[s + 1]));
            if (hi <= lo)
                continue;
            const SortView v = sort_view(B, s);
            if (v.sorting)
                f(v, first, lo, hi, off);
            lo = hi;
        }
    }
}

// rank[p] = arrival order of p among the particles of its cell.
__device__ void sort_count(const BatchDev &B, uint32_t chunk, uint32_t nchunks)
{
    const int lane = threadIdx.x & 63;
    particle_spans(B, chunk, nchunks, [&](const SortView &v, int64_t first, int64_t lo, int64_t hi, int64_t off) {
        // loads for every lane (an idle lane reads particle 0 of the scene),
        // so all of them are in flight together
        uint32_t p[kSortU], key[kSortU];
        bool act[kSortU];
        for (int u = 0; u < kSortU; ++u) {
            const int64_t g = first + u * 64 + lane;
            act[u] = g >= lo && g < hi;
            p[u] = act[u] ? (uint32_t)(g - off) : 0u;
        }
        for (int u = 0; u < kSortU; ++u)
            key[u] = v.cell[p[u]];
        for (int u = 0; u < kSortU; ++u)
            if (act[u])
                v.rank[p[u]] = atomicAdd((uint32_t *)&v.cnt[v.key(key[u])], 1u);
    });
}

// --- scan over the bricks of every reordering scene (segmented by scene) --
// Chunk j is a contiguous range of the flattened brick list; each thread of
// the workgroup running it takes a contiguous run of that range.

// Particle and item sums after the last scene start of a run (f: a scene
// starts inside the run), and the run's count of non-empty bricks of
// reordering scenes (not reset at scene starts: it numbers the batch's list
// of such bricks); join(a, b) is the run a followed by the run b.
struct Seg {
    uint32_t p, i, f, n;
};

__device__ inline Seg seg_join(const Seg &a, const Seg &b)
{
    return b.f ? Seg{b.p, b.i, 1u, a.n + b.n} : Seg{a.p + b.p, a.i + b.i, a.f, a.n + b.n};
}

struct BrickRun {
    uint32_t lo, hi;   // flattened brick indices [lo, hi)
};

// A thread's contiguous run of the brick range [b0, b1).
__device__ inline BrickRun thread_run(uint32_t b0, uint32_t b1)
{
    const uint32_t per = (b1 - b0 + blockDim.x - 1) / blockDim.x;
    const uint32_t lo = min(b0 + threadIdx.x * per, b1);
    return {lo, min(lo + per, b1)};
}

// A thread's walk over its run, scene by scene (vector loads: neighbouring
// threads may be in different scenes).  f(scene, sorting, flattened brick,
// brick in scene, first brick of its scene, last brick of its scene).
template <typename F>
__device__ inline void walk_run(const BatchDev &B, const BrickRun &r, F f)
{
    if (r.lo >= r.hi)
        return;
    int s = find_scene(B.boffs, B.nscenes, (int64_t)r.lo);
    uint32_t s_lo = (uint32_t)B.boffs[s], s_hi = (uint32_t)B.boffs[s + 1];
    const SceneDev *S = B.scenes[s];
    bool sorting = S->ctl[CTL_ERR] == 0u && S->ctl[CTL_REMAIN] > 0u && S->ctl[CTL_NEED_SORT] != 0u;
    for (uint32_t gb = r.lo; gb < r.hi; ++gb) {
        while (gb >= s_hi) {
            ++s;
            s_lo = s_hi;
            s_hi = (uint32_t)B.boffs[s + 1];
            S = B.scenes[s];
            sorting = S->ctl[CTL_ERR] == 0u && S->ctl[CTL_REMAIN] > 0u && S->ctl[CTL_NEED_SORT] != 0u;
        }
        f(S, sorting, gb, gb - s_lo, gb == s_lo, gb + 1 == s_hi);
    }
}

// One wavefront per brick, over a contiguous run of chunk j's range [b0, b1)
// of the flattened brick list (kBrickU bricks per pass): the brick's
// particle count, its work-item count and the cell-major start of every
// cell inside the brick (written for non-empty bricks only: nothing reads
// the others).  The workgroup then writes the range's partial sums for the
// brick scan into B.scan[4 j].
__device__ void sort_bricks(const BatchDev &B, uint32_t j, uint32_t b0, uint32_t b1)
{
    __shared__ Seg wseg[kBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint32_t per_wave = (b1 - b0 + nw - 1) / nw;
    const uint32_t w0 = uni(min(b0 + wave * per_wave, b1)), w1 = uni(min(w0 + per_wave, b1));
    Seg acc{0u, 0u, 0u, 0u};
    if (w0 < w1) {
        int s = find_scene_u(B.boffs, B.nscenes, w0);
        uint32_t s_hi = (uint32_t)cld(&B.boffs[s + 1]);
        SortView v = sort_view(B, s);
        for (uint32_t gb = w0; gb < w1;) {
            while (gb >= s_hi) {
                ++s;
                s_hi = (uint32_t)cld(&B.boffs[s + 1]);
                v = sort_view(B, s);
            }
            const uint32_t n = min(min(w1, s_hi) - gb, (uint32_t)kBrickU);
            const uint32_t bb = gb - v.bo;   // brick of the scene
            if (bb == 0)
                acc = Seg{0u, 0u, 1u, acc.n};
            if (v.sorting) {
                uint32_t c[kBrickU];
                for (int u = 0; u < kBrickU; ++u)
                    c[u] = (uint32_t)u < n ? v.cnt[(bb + u) * 64 + lane] : 0u;
                for (int u = 0; u < kBrickU; ++u) {
                    if ((uint32_t)u >= n)
                        break;
                    uint32_t inc = c[u];
                    for (int o = 1; o < 64; o <<= 1) {
                        const uint32_t t = __shfl_up(inc, o);
                        if (lane >= o)
                            inc += t;
                    }
                    const uint32_t tot = uni((uint32_t)__shfl(inc, 63));
                    const uint32_t items = (tot + kChunk - 1) / kChunk;
                    if (tot)
                        v.cstart[(bb + u) * 64 + lane] = inc - c[u];   // cell-major start inside the brick
                    if (lane == 0) {
                        v.bcnt[bb + u] = tot;
                        v.bitem[bb + u] = items;
                    }
                    acc.p += tot;
                    acc.i += items;
                    acc.n += tot ? 1u : 0u;
                }
            }
            gb += n;
        }
    }
    if (lane == 0)
        wseg[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        Seg agg{0u, 0u, 0u, 0u};
        for (int w = 0; w < nw; ++w)
            agg = seg_join(agg, wseg[w]);
        gp(B.scan)[4 * j] = agg.p;
        gp(B.scan)[4 * j + 1] = agg.i;
        gp(B.scan)[4 * j + 2] = agg.f;
        gp(B.scan)[4 * j + 3] = agg.n;
    }
    __syncthreads();   // wseg is reused by the workgroup's next chunk
}

// Workgroup-wide inclusive scan of Seg values with seg_join.
__device__ inline Seg block_seg_scan(Seg v)
{
    __shared__ Seg sv[kBlock];
    sv[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < (int)blockDim.x; o <<= 1) {
        Seg a{0u, 0u, 0u, 0u};
        const bool has = threadIdx.x >= (unsigned)o;
        if (has)
            a = sv[threadIdx.x - o];
        __syncthreads();
        if (has)
            v = seg_join(a, v);
        sv[threadIdx.x] = v;
        __syncthreads();
    }
    return v;
}

// Rest of the scan for chunk j (range [b0, b1)): the carried prefix from the
// earlier chunks' sums (back to the last one in which a scene starts; the
// brick count from all of them), then every brick's exclusive particle and
// item start, each scene's totals, and the batch's list of non-empty bricks
// in brick order.
__device__ void scan_finish(const BatchDev &B, uint32_t j, uint32_t b0, uint32_t b1)
{
    __shared__ uint32_t red[kBlock / 64][3];
    __shared__ uint32_t carry[3];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const GLOBAL uint32_t *P = gp(B.scan);
    // nearest earlier chunk whose range holds a scene start
    int k0 = 0;
    for (int k = threadIdx.x; k < (int)j; k += blockDim.x)
        if (P[4 * k + 2])
            k0 = max(k0, k);
    k0 = wave_reduce<true>(k0);
    if (lane == 0)
        red[wave][0] = (uint32_t)k0;
    __syncthreads();
    k0 = 0;
    for (int w = 0; w < nw; ++w)
        k0 = max(k0, (int)red[w][0]);
    __syncthreads();
    uint32_t cp = 0, ci = 0, cn = 0;
    for (int k = k0 + threadIdx.x; k < (int)j; k += blockDim.x) {
        cp += P[4 * k];
        ci += P[4 * k + 1];
    }
    for (int k = threadIdx.x; k < (int)j; k += blockDim.x)
        cn += P[4 * k + 3];
    for (int o = 32; o > 0; o >>= 1) {
        cp += __shfl_xor(cp, o);
        ci += __shfl_xor(ci, o);
        cn += __shfl_xor(cn, o);
    }
    if (lane == 0) {
        red[wave][0] = cp;
        red[wave][1] = ci;
        red[wave][2] = cn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = 0, c = 0, m = 0;
        for (int w = 0; w < nw; ++w) {
            a += red[w][0];
            c += red[w][1];
            m += red[w][2];
        }
        carry[0] = a;
        carry[1] = c;
        carry[2] = m;
    }
    __syncthreads();
    // this thread's run sums, then its start within the workgroup
    const BrickRun r = thread_run(b0, b1);
    Seg mine{0u, 0u, 0u, 0u};
    walk_run(B, r, [&](const SceneDev *S, bool sorting, uint32_t, uint32_t b, bool first, bool) {
        if (first)
            mine = Seg{0u, 0u, 1u, mine.n};
        if (sorting) {
            const uint32_t bc = gp(S->bcnt)[b];
            mine.p += bc;
            mine.i += gp(S->bitem)[b];
            mine.n += bc ? 1u : 0u;
        }
    });
    const Seg inc = block_seg_scan(mine);
    // exclusive start of the run: carried prefix joined with the earlier threads
    __shared__ Seg xs[kBlock];
    xs[threadIdx.x] = inc;
    __syncthreads();
    Seg run{carry[0], carry[1], 0u, carry[2]};
    if (threadIdx.x > 0)
        run = seg_join(run, xs[threadIdx.x - 1]);
    __syncthreads();
    walk_run(B, r, [&](const SceneDev *S, bool sorting, uint32_t gb, uint32_t b, bool first, bool last) {
        if (first)
            run = Seg{0u, 0u, 1u, run.n};
        if (!sorting)
            return;
        const uint32_t bc = gp(S->bcnt)[b], bi = gp(S->bitem)[b];
        gp(S->bstart)[b] = run.p;
        gp(S->istart)[b] = run.i;
        if (bc)
            gp(B.bricks)[run.n++] = gb;
        run.p += bc;
        run.i += bi;
        if (last) {
            gp(S->bstart)[b + 1] = run.p;
            gp(S->istart)[b + 1] = run.i;
            gp(S->ctl)[CTL_N_ITEMS] = run.i;
        }
    });
    if (r.lo < r.hi && r.hi == (uint32_t)B.total_bricks)   // the batch's last brick
        B.flags[BF_NBRICKS] = run.n;
    __syncthreads();   // shared arrays are reused by the workgroup's next chunk
}

// perm lists the particles cell-major: slot bstart[brick] + cstart[key] +
// rank holds p.  The particle that opens a 512-slot chunk of its brick
// writes that work item.
__device__ void sort_perm(const BatchDev &B, uint32_t chunk, uint32_t nchunks)
{
    const int lane = threadIdx.x & 63;
    particle_spans(B, chunk, nchunks, [&](const SortView &v, int64_t first, int64_t lo, int64_t hi, int64_t off) {
        // loads for every lane (an idle lane reads particle 0 of the scene),
        // so all of them are in flight together
        uint32_t p[kSortU], key[kSortU], local[kSortU], bs[kSortU];
        bool act[kSortU];
        for (int u = 0; u < kSortU; ++u) {
            const int64_t g = first + u * 64 + lane;
            act[u] = g >= lo && g < hi;
            p[u] = act[u] ? (uint32_t)(g - off) : 0u;
        }
        for (int u = 0; u < kSortU; ++u)
            key[u] = v.cell[p[u]];
        for (int u = 0; u < kSortU; ++u)
            key[u] = v.key(key[u]);
        for (int u = 0; u < kSortU; ++u) {
            local[u] = v.cstart[key[u]] + v.rank[p[u]];
            bs[u] = v.bstart[key[u] >> 6];
        }
        for (int u = 0; u < kSortU; ++u) {
            if (!act[u])
                continue;
            v.perm[bs[u] + local[u]] = p[u];
            if (local[u] % kChunk == 0) {
                const uint32_t b = key[u] >> 6;
                Item it;
                it.start = bs[u] + local[u];
                it.count = min((uint32_t)kChunk, v.bcnt[b] - local[u]);
                it.brick = b;
                it.pad = 0;
                ((Item *)v.items)[v.istart[b] + local[u] / kChunk] = it;
            }
        }
    });
}

// Particle arrays of one buffer for the move: one scalar base per field.
template <typename R>
struct MoveBuf {
    GLOBAL double *x;
    GLOBAL R *v, *sig, *vol, *mass;
    GLOBAL uint32_t *cell, *pid;
};

template <typename R>
__device__ inline MoveBuf<R> move_buf(const SceneDev *S, int b)
{
    MoveBuf<R> m;
    m.x = gp(cld(&S->x[b]));
    m.v = gp((R *)cld(&S->v[b]));
    m.sig = gp((R *)cld(&S->sig[b]));
    m.vol = gp((R *)cld(&S->vol[b]));
    m.mass = gp((R *)cld(&S->mass[b]));
    m.cell = gp(cld(&S->cell[b]));
    m.pid = gp(cld(&S->pid[b]));
    return m;
}

// One particle's state in registers.
template <typename R>
struct MoveRec {
    double x[3];
    R v[3], sig[6], vol, mass;
    uint32_t cell, pid;
};

// One wavefront per listed (non-empty) brick, lane = cell: write the
// brick's particles to the other buffer in level-major order -- the first
// particle of every occupied cell, then the second of every cell holding two
// or more, and so on.  A wavefront of consecutive particles then spans
// distinct cells, so the scatter kernels' LDS atomics for one node corner do
// not collide.  Each pass reads kMoveLevels levels before it writes any.
// Resets the brick's per-cell counts for the next sort.
// A chunk is the listed bricks [i0, i1).
template <typename R>
__device__ void sort_move(const BatchDev &B, uint32_t i0, uint32_t i1)
{
    const int lane = threadIdx.x & 63;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint32_t nw = blockDim.x >> 6;
    for (uint32_t i = i0 + uni(threadIdx.x >> 6); i < i1; i += nw) {
        const uint32_t gb = uni(gp(B.bricks)[i]);
        const int s = find_scene_u(B.boffs, B.nscenes, gb);
        const SortView sv = sort_view(B, s);
        const uint32_t n = (uint32_t)cld(&sv.S->np);
        const MoveBuf<R> src = move_buf<R>(sv.S, sv.cur), dst = move_buf<R>(sv.S, sv.cur ^ 1);
        const uint32_t b = gb - sv.bo;
        const uint32_t nc = sv.cnt[b * 64 + lane];
        const uint32_t bs = uni(sv.bstart[b]);
        const uint32_t cs = bs + sv.cstart[b * 64 + lane];
        sv.cnt[b * 64 + lane] = 0u;
        uint32_t levels = nc;
        for (int o = 32; o > 0; o >>= 1)
            levels = max(levels, (uint32_t)__shfl_xor(levels, o));
        levels = uni(levels);
        uint32_t base = bs;
        constexpr int ML = sizeof(R) == 4 ? kMoveLevels : kMoveLevels / 2;   // within 128 VGPRs
        for (uint32_t j0 = 0; j0 < levels; j0 += ML) {
            MoveRec<R> r[ML];
            uint32_t d[ML];
            bool act[ML];
            for (int l = 0; l < ML; ++l) {
                act[l] = j0 + l < nc;
                const uint64_t m = __ballot(act[l]);
                d[l] = base + (uint32_t)__popcll(m & below);
                base += (uint32_t)__popcll(m);
                if (!act[l])
                    continue;
                const uint32_t p = sv.perm[cs + j0 + l];
                for (int a = 0; a < 3; ++a) {
                    r[l].x[a] = ldg(src.x, a * n + p);
                    r[l].v[a] = ldg(src.v, a * n + p);
                }
                for (int k = 0; k < 6; ++k)
                    r[l].sig[k] = ldg(src.sig, k * n + p);
                r[l].vol = ldg(src.vol, p);
                r[l].mass = ldg(src.mass, p);
                r[l].cell = ldg(src.cell, p);
                r[l].pid = ldg(src.pid, p);
            }
            for (int l = 0; l < ML; ++l) {
                if (!act[l])
                    continue;
                const uint32_t q = d[l];
                for (int a = 0; a < 3; ++a) {
                    stg(dst.x, a * n + q, r[l].x[a]);
                    stg(dst.v, a * n + q, r[l].v[a]);
                }
                for (int k = 0; k < 6; ++k)
                    stg(dst.sig, k * n + q, r[l].sig[k]);
                stg(dst.vol, q, r[l].vol);
                stg(dst.mass, q, r[l].mass);
                stg(dst.cell, q, r[l].cell);
                stg(dst.pid, q, r[l].pid);
            }
        }
    }
}

// Reorder of the flagged scenes, then the step control in the last
// workgroup to leave.  Chunk sizes grow with the batch so that there are
// about as many chunks in every phase as workgroups.  A phase
// runs only if no workgroup gave up waiting for the one before; the step
// control then fails the reordering scenes (ERR_SORT) and keeps their
// particles where they were.  The counters are cleared by the next stage
// kernel (and at the start of every call), after every workgroup of this
// launch has finished.
template <typename R>
__global__ void __launch_bounds__(kBlock) k_reorder(BatchDev B)
{
    __shared__ int sh;
    if (!B.flags[BF_ANY_SORT]) {
        // nothing moves: the first workgroup runs the step control alone
        if (blockIdx.x == 0)
            step_control(B);
        return;
    }
    uint32_t *F = B.flags;
    const int64_t np = B.total_particles;
    const uint32_t nb = (uint32_t)B.total_bricks;
    // chunks per phase aimed at: one per workgroup, so that with every
    // workgroup resident the phases split as evenly as a static assignment
    const int64_t target = gridDim.x;
    // particle chunks: about `target` of them, each a whole number of
    // wavefront passes of the workgroup
    const int64_t pass = kSpan * (blockDim.x >> 6);
    const uint32_t npc = (uint32_t)max((int64_t)1, min(target, (np + pass - 1) / pass));
    // brick chunks of the scan: at most kScanChunks of them
    const uint32_t bch = max(max(kScanBricks, (nb + kScanChunks - 1) / kScanChunks),
                             (uint32_t)((nb + gridDim.x - 1) / gridDim.x));
    const uint32_t nbc = max(1u, (nb + bch - 1) / bch);
    bool go = true;
    run_chunks(F, PH_COUNT, npc, go, &sh, [&](uint32_t c) { sort_count(B, c, npc); });
    go = phase_done(F, PH_COUNT, &sh);
    run_chunks(F, PH_BRICKS, nbc, go, &sh,
               [&](uint32_t c) { sort_bricks(B, c, min(c * bch, nb), min((c + 1) * bch, nb)); });
    go = phase_done(F, PH_BRICKS, &sh);
    run_chunks(F, PH_SCAN, nbc, go, &sh,
               [&](uint32_t c) { scan_finish(B, c, min(c * bch, nb), min((c + 1) * bch, nb)); });
    go = phase_done(F, PH_SCAN, &sh);
    run_chunks(F, PH_PERM, npc, go, &sh, [&](uint32_t c) { sort_perm(B, c, npc); });
    go = phase_done(F, PH_PERM, &sh);
    // move chunks: listed bricks, one per wavefront per pass
    const uint32_t nbr = uni(__hip_atomic_load(&F[BF_NBRICKS], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    const uint32_t mpass = blockDim.x >> 6;
    const uint32_t mch = max(1u, (nbr + mpass * (uint32_t)target - 1) / (mpass * (uint32_t)target)) * mpass;
    const uint32_t nmc = max(1u, (nbr + mch - 1) / mch);
    run_chunks(F, PH_MOVE, nmc, go, &sh, [&](uint32_t c) { sort_move<R>(B, c * mch, min((c + 1) * mch, nbr)); });
    // the last workgroup to leave runs the step control
    if (threadIdx.x == 0) {
        __threadfence();
        sh = atomicAdd(&F[BF_EXIT], 1u) == gridDim.x - 1 ? 1 : 0;
    }
    __syncthreads();
    if (!sh)
        return;
    __threadfence();
    step_control(B);
}

// ------------------------------------------------------- item kernels --
// One workgroup per work item.  Particles are taken 256 at a time in storage
// (level-major) order, so one instruction's lanes belong to distinct cells.
// Scatters accumulate in FP64 in the workgroup's LDS node tile (an LDS add
// of doubles is far cheaper than one of floats on gfx950) and are flushed
// with one global atomic per touched node and component.

// Particle arrays of one buffer: one scalar base per field.
template <typename R>
struct Parts {
    Comp<double> x[3];
    Comp<R> v[3];
    Comp<R> sig[6];
    GLOBAL R *vol;
    GLOBAL R *mass;
    GLOBAL uint32_t *cell;
};

template <typename R>
__device__ inline Parts<R> parts(const SceneDev &S, int cur)
{
    Parts<R> P;
    const uint32_t n = (uint32_t)S.np;
    for (int a = 0; a < 3; ++a) {
        P.x[a] = Comp<double>{gp(pick(S.x, cur)), a * n};
        P.v[a] = Comp<R>{gp((R *)pick(S.v, cur)), a * n};
    }
    for (int k = 0; k < 6; ++k)
        P.sig[k] = Comp<R>{gp((R *)pick(S.sig, cur)), k * n};
    P.vol = gp((R *)pick(S.vol, cur));
    P.mass = gp((R *)pick(S.mass, cur));
    P.cell = gp(pick(S.cell, cur));
    return P;
}

// GIMP P2G of one work item (k_p2g): the item's particles' mass and momentum
// into the node box t, flushed to node buffer nb; with force, a second pass
// of the nodal force (internal from the current stress and volume, and
// gravity) through the same LDS accumulators.  When the box fits the
// anchored layout (kAnchPX), each particle adds its mass and momentum to the
// 4 x 4 x 4 anchored slots of its cell, a thread's two particles in one cell
// (successive particles of the cell in level-major order) sharing one set of
// adds, and its force to its 27 support nodes in rotated order; otherwise
// each particle adds to its 27-node support at the box's pitches.
template <typename R, bool WITH_FORCE, int T>
__device__ __attribute__((always_inline)) inline void p2g_gimp_item(const SceneDev &S, const Parts<R> &P, const NodeBuf<R> &nb, const Item &item,
                                     const Tile &t, double (*acc)[kAnchCap], R gx, R gy, R gz)
{
    constexpr int KP = kChunk / T;
    const int tv = t.dim[0] * t.dim[1] * t.dim[2];
    const bool anch = t.dim[0] <= kAnchPX && t.dim[1] <= 9 && t.dim[2] <= 9;
    const int px = anch ? kAnchPX : t.dim[0], pxy = anch ? kAnchPXY : t.dim[0] * t.dim[1];
    auto entry = [&](int i, int j, int k) { return (i - t.lo[0]) + px * (j - t.lo[1]) + pxy * (k - t.lo[2]); };
    uint32_t pc[KP];
#pragma unroll
    for (int rr = 0; rr < KP; ++rr) {
        const uint32_t q = threadIdx.x + rr * T;
        pc[rr] = q < item.count ? ldg(P.cell, item.start + q) : 0xffffffffu;
    }
    for (int q = threadIdx.x; q < tv; q += T) {
        int i, j, k;
        tile_node_small(t, q, i, j, k);
        const int e = entry(i, j, k);
        acc[0][e] = acc[1][e] = acc[2][e] = acc[3][e] = 0.0;
    }
    __syncthreads();
    // support of the thread's particle rr (cell c), anchored weights
    auto support = [&](int rr, const int c[3], R w4[3][4], R dw4[3][4], Support<R, 1> &sq) {
        const uint32_t p = item.start + threadIdx.x + rr * T;
        const double xp[3] = {ldg(P.x[0], p), ldg(P.x[1], p), ldg(P.x[2], p)};
        make_support<R, 1>(S, xp, c, sq);
        for (int a = 0; a < 3; ++a)
            anchor4<R>(sq.w[a], sq.dw[a], sq.base[a] == c[a] ? 1 : 0, w4[a], dw4[a]);
    };
    // pass 1: mass and momentum of particle ra, and of rb (>= 0) in its cell
    auto mass_momentum = [&](int ra, int rb) {
        int c[3];
        unpack_cell(pc[ra], c);
        const int np_ = rb >= 0 ? 2 : 1;
        R w4[2][3][4], dw4[3][4], m[2], mv[2][3];
        Support<R, 1> sq[2];
        for (int u = 0; u < np_; ++u) {
            const int rq = u ? rb : ra;
            const uint32_t p = item.start + threadIdx.x + rq * T;
            support(rq, c, w4[u], dw4, sq[u]);
            m[u] = ldg(P.mass, p);
            for (int a = 0; a < 3; ++a)
                mv[u][a] = m[u] * ldg(P.v[a], p);
        }
        if (anch) {
            const int a0 = entry(c[0] - 1, c[1] - 1, c[2] - 1);
            for (int k = 0; k < 4; ++k)
                for (int j = 0; j < 4; ++j) {
                    R y[2];
                    for (int u = 0; u < np_; ++u)
                        y[u] = w4[u][1][j] * w4[u][2][k];
                    for (int i = 0; i < 4; ++i) {
                        R sm = (R)0, s0 = (R)0, s1 = (R)0, s2 = (R)0;
                        for (int u = 0; u < np_; ++u) {
                            const R N = w4[u][0][i] * y[u];
                            sm += N * m[u];
                            s0 += N * mv[u][0];
                            s1 += N * mv[u][1];
                            s2 += N * mv[u][2];
                        }
                        const int li = a0 + i + kAnchPX * j + kAnchPXY * k;
                        atomicAdd(&acc[0][li], (double)sm);
                        atomicAdd(&acc[1][li], (double)s0);
                        atomicAdd(&acc[2][li], (double)s1);
                        atomicAdd(&acc[3][li], (double)s2);
                    }
                    __builtin_amdgcn_sched_barrier(0);   // one row of LDS adds in flight
                }
        } else {
            const Support<R, 1> &sp = sq[0];
            const int b0 = entry(sp.base[0], sp.base[1], sp.base[2]);
            for (int k = 0; k < 3; ++k)
                for (int j = 0; j < 3; ++j)
                    for (int i = 0; i < 3; ++i) {
                        const R N = sp.w[0][i] * sp.w[1][j] * sp.w[2][k];
                        const int li = b0 + i + px * j + pxy * k;
                        atomicAdd(&acc[0][li], (double)(N * m[0]));
                        atomicAdd(&acc[1][li], (double)(N * mv[0][0]));
                        atomicAdd(&acc[2][li], (double)(N * mv[0][1]));
                        atomicAdd(&acc[3][li], (double)(N * mv[0][2]));
                    }
        }
    };
    // pass 2: internal and external force of particle rr: f_a = A_a0 dN/dx +
    // A_a1 dN/dy + A_a2 dN/dz + N m g_a with A = -V sigma; on a support row
    // (j, k), dN/dx = dw_i P1, dN/dy = w_i P2, dN/dz = w_i P3 and N = w_i P1.
    // In the anchored layout the 27 slots go in rotated order (see kAnchPX):
    // the pass is VALU-bound, and a pair's 64 shared slots cost more
    // arithmetic than they save in LDS adds
    auto forces = [&](int rr, int) {
        int c[3];
        unpack_cell(pc[rr], c);
        const uint32_t p = item.start + threadIdx.x + rr * T;
        const double xp[3] = {ldg(P.x[0], p), ldg(P.x[1], p), ldg(P.x[2], p)};
        Support<R, 1> sp;
        make_support<R, 1>(S, xp, c, sp);
        const R mq = ldg(P.mass, p), vq = ldg(P.vol, p);
        R A[6];
        for (int k = 0; k < 6; ++k)
            A[k] = -vq * ldg(P.sig[k], p);
        const R mg[3] = {mq * gx, mq * gy, mq * gz};
        if (anch) {
            R wr[3][3], dr[3][3];
            int e[3];
            for (int a = 0; a < 3; ++a)
                e[a] = rotate3<R>(sp.w[a], sp.dw[a], sp.base[a] == c[a], wr[a], dr[a]);
            const int a0 = entry(c[0] - 1, c[1] - 1, c[2] - 1);
            const int ox[3] = {1, 2, e[0]}, oy[3] = {kAnchPX, 2 * kAnchPX, kAnchPX * e[1]},
                      oz[3] = {kAnchPXY, 2 * kAnchPXY, kAnchPXY * e[2]};
            for (int k = 0; k < 3; ++k)
                for (int j = 0; j < 3; ++j) {
                    const R P1 = wr[1][j] * wr[2][k], P2 = dr[1][j] * wr[2][k], P3 = wr[1][j] * dr[2][k];
                    const R X[3] = {A[0] * P1, A[3] * P1, A[5] * P1};
                    const R Y[3] = {A[3] * P2 + A[5] * P3 + mg[0] * P1, A[1] * P2 + A[4] * P3 + mg[1] * P1,
                                    A[4] * P2 + A[2] * P3 + mg[2] * P1};
                    const int rb = a0 + oy[j] + oz[k];
                    for (int i = 0; i < 3; ++i) {
                        const int li = rb + ox[i];
                        atomicAdd(&acc[0][li], (double)(dr[0][i] * X[0] + wr[0][i] * Y[0]));
                        atomicAdd(&acc[1][li], (double)(dr[0][i] * X[1] + wr[0][i] * Y[1]));
                        atomicAdd(&acc[2][li], (double)(dr[0][i] * X[2] + wr[0][i] * Y[2]));
                    }
                    __builtin_amdgcn_sched_barrier(0);   // one row of LDS adds in flight
                }
        } else {
            const int b0 = entry(sp.base[0], sp.base[1], sp.base[2]);
            for (int k = 0; k < 3; ++k)
                for (int j = 0; j < 3; ++j)
                    for (int i = 0; i < 3; ++i) {
                        const R P1 = sp.w[1][j] * sp.w[2][k], P2 = sp.dw[1][j] * sp.w[2][k],
                                P3 = sp.w[1][j] * sp.dw[2][k];
                        const R dx = sp.dw[0][i] * P1, dy = sp.w[0][i] * P2, dz = sp.w[0][i] * P3,
                                N = sp.w[0][i] * P1;
                        const int li = b0 + i + px * j + pxy * k;
                        atomicAdd(&acc[0][li], (double)(A[0] * dx + A[3] * dy + A[5] * dz + N * mg[0]));
                        atomicAdd(&acc[1][li], (double)(A[3] * dx + A[1] * dy + A[4] * dz + N * mg[1]));
                        atomicAdd(&acc[2][li], (double)(A[5] * dx + A[4] * dy + A[2] * dz + N * mg[2]));
                    }
        }
    };
    // each particle of the thread; with pairs, successive particles rr,
    // rr + 1 of one cell together
    auto each = [&](auto &&fn, bool pairs) {
#pragma unroll
        for (int rr = 0; rr < KP; rr += 2) {
            if (threadIdx.x + rr * T >= item.count)
                break;
            const bool has1 = rr + 1 < KP && threadIdx.x + (rr + 1) * T < item.count;
            if (pairs && anch && has1 && pc[rr] == pc[rr + 1]) {
                fn(rr, rr + 1);
                continue;
            }
            fn(rr, -1);
            if (has1)
                fn(rr + 1, -1);
        }
    };
    each(mass_momentum, true);
    __syncthreads();
    for (int q = threadIdx.x; q < tv; q += T) {
        int i, j, k;
        tile_node_small(t, q, i, j, k);
        const int e = entry(i, j, k);
        const double m = acc[0][e];
        if (m != 0.0) {
            const uint32_t I = node_id(S, i, j, k);
            addg(nb.m, I, m);
            for (int a = 0; a < 3; ++a)
                addg(nb.p[a], I, (R)acc[1 + a][e]);
        }
        if constexpr (WITH_FORCE)
            acc[0][e] = acc[1][e] = acc[2][e] = 0.0;
    }
    __syncthreads();
    if constexpr (WITH_FORCE) {
        each(forces, false);
        __syncthreads();
        for (int q = threadIdx.x; q < tv; q += T) {
            int i, j, k;
            tile_node_small(t, q, i, j, k);
            const int e = entry(i, j, k);
            const R f0 = (R)acc[0][e], f1 = (R)acc[1][e], f2 = (R)acc[2][e];
            if (f0 == (R)0 && f1 == (R)0 && f2 == (R)0)
                continue;
            const uint32_t I = node_id(S, i, j, k);
            addg(nb.f[0], I, f0);
            addg(nb.f[1], I, f1);
            addg(nb.f[2], I, f2);
        }
        __syncthreads();
    }
}

// Nodal mass and momentum into the step's node buffer (first step of a call;
// USF scenes whose buffer is already filled skip it); with WITH_FORCE also
// the nodal force from the current stress and volume (USL and MUSL, every
// step); with REMAP (MUSL) it also zeroes the previous step's remap.
template <typename R, int SH, bool WITH_FORCE, int T, bool REMAP = false>
__global__ void __launch_bounds__(T) k_p2g(BatchDev B)
{
    constexpr int NS = ShapeTraits<SH>::NS;
    constexpr int CAP = ShapeTraits<SH>::cap;
    constexpr int NACC = WITH_FORCE ? 7 : 4;
    // GIMP: mass and momentum, then (with force) the force, in two passes
    // over one set of four accumulators, laid out at the anchored pitches
    // when the item's box fits them
    constexpr int ACC_N = SH == 1 ? 4 : NACC;
    constexpr int ACC_CAP = SH == 1 ? kAnchCap : CAP;
    __shared__ double acc[ACC_N][ACC_CAP];
    __shared__ int red[6 * (T / 64)];
    clear_reorder_flags(B);
    if constexpr (REMAP)
        clear_remap_previous<R>(B);
    const int64_t total = B.ioffs[B.nscenes];
    const ItemRange ir = item_range(total);
    for (int64_t g = ir.first; g < ir.end; g += ir.step) {
        const ItemRef r = item_ref(B.ioffs, B, g);
        const SceneDev S = load_scene(r.S);
        if (!scene_active(S) || (!WITH_FORCE && S.ctl[CTL_HAVE_P2G]))
            continue;
        const Item item = cld_struct(&S.items[r.it]);
        const int cur = (int)cld(&S.ctl[CTL_CUR]);
        const int buf = (int)cld(&S.ctl[CTL_NBUF]);
        const Parts<R> P = parts<R>(S, cur);
        const NodeBuf<R> nb = node_buf<R>(S, buf);
        Tile t;
        {
            int mn[3] = {1 << 30, 1 << 30, 1 << 30}, mx[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
            for (uint32_t q = threadIdx.x; q < item.count; q += T) {
                int c[3];
                unpack_cell(ldg(P.cell, item.start + q), c);
                for (int a = 0; a < 3; ++a) {
                    mn[a] = min(mn[a], c[a]);
                    mx[a] = max(mx[a], c[a]);
                }
            }
            int lo[3], hi[3];
            item_box<T>(mn, mx, red, lo, hi);
            t = tile_of_cells<SH>(lo, hi);
        }
        if (threadIdx.x == 0) {
            pick(S.tiles, buf)[r.it] = t;
            if (r.it == 0)
                S.ctl[CTL_ACC0 + buf] = S.ctl[CTL_N_ITEMS];
        }
        if (!t.fits) {
            if (threadIdx.x == 0)
                atomicOr(&S.ctl[CTL_ERR], ERR_TILE);
            continue;
        }
        const int tv = t.dim[0] * t.dim[1] * t.dim[2];
        const R gx = cst<R>(S.g[0], S.f_g[0]), gy = cst<R>(S.g[1], S.f_g[1]), gz = cst<R>(S.g[2], S.f_g[2]);
        if constexpr (SH == 1) {
            p2g_gimp_item<R, WITH_FORCE, T>(S, P, nb, item, t, acc, gx, gy, gz);
            continue;
        } else {
        for (int q = threadIdx.x; q < tv; q += blockDim.x)
            for (int c = 0; c < NACC; ++c)
                acc[c][q] = 0.0;
        __syncthreads();
        // a work item holds at most kChunk particles: a fixed trip count the
        // compiler unrolls, keeping the next particle's loads in flight
#pragma unroll
        for (int rr = 0; rr < kChunk / T; ++rr) {
            const uint32_t q = threadIdx.x + rr * T;
            if (q >= item.count)
                break;
            const uint32_t p = item.start + q;
            const double xp[3] = {ldg(P.x[0], p), ldg(P.x[1], p), ldg(P.x[2], p)};
            int c[3];
            unpack_cell(ldg(P.cell, p), c);
            Support<R, SH> sp;
            make_support<R, SH>(S, xp, c, sp);
            const Corners cn = corners(S, t, sp.base);
            const R mp = ldg(P.mass, p);
            const R mv[3] = {mp * ldg(P.v[0], p), mp * ldg(P.v[1], p), mp * ldg(P.v[2], p)};
            R sg[6], vol = (R)0;
            if constexpr (WITH_FORCE) {
                for (int k = 0; k < 6; ++k)
                    sg[k] = ldg(P.sig[k], p);
                vol = ldg(P.vol, p);
            }
            for (int k = 0; k < NS; ++k)
                for (int j = 0; j < NS; ++j)
                    for (int i = 0; i < NS; ++i) {
                        const R wyz = sp.w[1][j] * sp.w[2][k];
                        const R N = sp.w[0][i] * wyz;
                        const int li = cn.t0 + i + j * cn.ty + k * cn.tz;
                        atomicAdd(&acc[0][li], (double)(N * mp));
                        atomicAdd(&acc[1][li], (double)(N * mv[0]));
                        atomicAdd(&acc[2][li], (double)(N * mv[1]));
                        atomicAdd(&acc[3][li], (double)(N * mv[2]));
                        if constexpr (WITH_FORCE) {
                            R gxN = sp.dw[0][i] * wyz;
                            R gyN = sp.w[0][i] * sp.dw[1][j] * sp.w[2][k];
                            R gzN = sp.w[0][i] * sp.w[1][j] * sp.dw[2][k];
                            to_dx<R, SH>(sp, gxN, gyN, gzN);
                            const R fx = -vol * (sg[0] * gxN + sg[3] * gyN + sg[5] * gzN) + N * mp * gx;
                            const R fy = -vol * (sg[3] * gxN + sg[1] * gyN + sg[4] * gzN) + N * mp * gy;
                            const R fz = -vol * (sg[5] * gxN + sg[4] * gyN + sg[2] * gzN) + N * mp * gz;
                            atomicAdd(&acc[4][li], (double)fx);
                            atomicAdd(&acc[5][li], (double)fy);
                            atomicAdd(&acc[6][li], (double)fz);
                        }
                    }
        }
        __syncthreads();
        for (int q = threadIdx.x; q < tv; q += blockDim.x) {
            const double m = acc[0][q];
            if (m == 0.0)
                continue;
            int i, j, k;
            tile_node_small(t, q, i, j, k);
            const uint32_t I = node_id(S, i, j, k);
            addg(nb.m, I, m);
            for (int a = 0; a < 3; ++a)
                addg(nb.p[a], I, (R)acc[1 + a][q]);
            if constexpr (WITH_FORCE)
                for (int a = 0; a < 3; ++a)
                    addg(nb.f[a], I, (R)acc[4 + a][q]);
        }
        __syncthreads();
        }
    }
}

// Per-thread support cache of the item kernels.  With T threads per item,
// thread t takes the item's particles t, t + T, t + 2T, ...; in level-major
// order these are successive particles of one cell, so with linear shape
// functions they share one support.  The thread then gathers that support's
// nodal values from LDS once and sums its particles' scatter contributions
// in registers, touching LDS again only when the support changes.  GIMP
// supports differ between particles of a cell, so GIMP gathers and scatters
// per particle.
template <int SH, bool G, bool S>
struct Cache {
    static constexpr bool gather = SH != 1 && G;
    static constexpr bool scatter = SH != 1 && S;
    static constexpr int gnodes = gather ? 8 : 1;
    static constexpr int snodes = scatter ? 8 : 1;
};

// Make the compiler produce the G2P sums where they are written: without
// this it sinks a sum into the branch that needs it (the PIC/FLIP choice,
// the stress update after the position), which keeps every gathered node
// value live to the end of the support (the GIMP g2p_usl and musl_g2p took
// 238-256 VGPRs; 113 and 92 with it).  An empty statement, no code.
template <typename R>
__device__ inline void pin_sums(R (&a)[3], R (&b)[3])
{
    asm volatile("" : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(b[0]), "+v"(b[1]), "+v"(b[2]));
}

template <typename R>
__device__ inline void pin_grad(R (&L)[3][3])
{
    asm volatile("" : "+v"(L[0][0]), "+v"(L[0][1]), "+v"(L[0][2]), "+v"(L[1][0]), "+v"(L[1][1]), "+v"(L[1][2]),
                 "+v"(L[2][0]), "+v"(L[2][1]), "+v"(L[2][2]));
}

// Keep loaded particle values at their loads: a value that one branch alone
// uses (FLIP's old velocity) is otherwise loaded inside that branch, one more
// memory round trip per particle.  An empty statement, no code.
template <typename R>
__device__ inline void pin_loaded(const R (&v)[3])
{
    asm volatile("" ::"v"(v[0]), "v"(v[1]), "v"(v[2]));
}

__device__ inline bool same_base(const int a[3], const int b[3])
{
    return a[0] == b[0] && a[1] == b[1] && a[2] == b[2];
}

// USF: zero the previous step's node buffer; nodal velocity, strain
// increment, volume and stress update, nodal internal + external force.
template <typename R, int SH, int T>
__global__ void __launch_bounds__(T) k_stress(BatchDev B)
{
    constexpr int NS = ShapeTraits<SH>::NS;
    constexpr int CAP = ShapeTraits<SH>::cap;
    constexpr int KP = kChunk / T;
    using C = Cache<SH, kStressCacheGather, kStressCacheScatter>;
    constexpr bool GC = C::gather, SC = C::scatter;
    constexpr int GN = C::gnodes, SN = C::snodes;
    // GIMP force accumulators in the anchored layout (12 x 9 x 9) when the
    // item's node box fits it, else in the box's own layout
    constexpr int FCAP = SH == 1 ? kAnchCap : CAP;
    // nodal velocity tile, 12 bytes per node (FP32): x, y in lvxy, z in lvz
    __shared__ R2<R> lvxy[CAP];
    __shared__ R lvz[CAP];
    __shared__ double lf[3][FCAP];
    __shared__ int red[6 * (T / 64)];
    clear_reorder_flags(B);
    clear_previous<R>(B);
    const int64_t total = B.ioffs[B.nscenes];
    const ItemRange ir = item_range(total);
    for (int64_t g = ir.first; g < ir.end; g += ir.step) {
        const ItemRef r = item_ref(B.ioffs, B, g);
        const SceneDev S = load_scene(r.S);
        if (!scene_active(S))
            continue;
        const Item item = cld_struct(&S.items[r.it]);
        const int cur = (int)cld(&S.ctl[CTL_CUR]);
        const int buf = (int)cld(&S.ctl[CTL_NBUF]);
        const Parts<R> P = parts<R>(S, cur);
        const NodeBuf<R> nb = node_buf<R>(S, buf);
        uint32_t pcell[KP];
        int mn[3] = {1 << 30, 1 << 30, 1 << 30}, mx[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
#pragma unroll
        for (int rr = 0; rr < KP; ++rr) {
            const uint32_t q = threadIdx.x + rr * T;
            if (q >= item.count)
                continue;
            pcell[rr] = ldg(P.cell, item.start + q);
            int c[3];
            unpack_cell(pcell[rr], c);
            for (int a = 0; a < 3; ++a) {
                mn[a] = min(mn[a], c[a]);
                mx[a] = max(mx[a], c[a]);
            }
        }
        // the node box: recorded by the kernel that filled this node buffer
        // when the items are unchanged since, else reduced here
        Tile t;
        if (cld(&S.ctl[CTL_BOX_OK])) {
            t = cld_struct(&pick(S.tiles, buf)[r.it]);
        } else {
            int blo[3], bhi[3];
            item_box<T>(mn, mx, red, blo, bhi);
            t = tile_of_cells<SH>(blo, bhi);
        }
        if (threadIdx.x == 0)
            S.tstep[r.it] = t;
        if (!t.fits) {
            if (threadIdx.x == 0)
                atomicOr(&S.ctl[CTL_ERR], ERR_TILE);
            __syncthreads();
            continue;
        }
        const int tv = t.dim[0] * t.dim[1] * t.dim[2];
        // anchored GIMP scatter: every anchored node of the item's particles
        // (cells lo..hi, nodes lo - 1 .. hi + 2) lies in the box, whose edges
        // must fit the anchored layout
        const bool anch = SH == 1 && t.dim[0] <= kAnchPX && t.dim[1] <= 9 && t.dim[2] <= 9;
        auto fidx = [&](int q, int i, int j, int k) {
            return anch ? (i - t.lo[0]) + kAnchPX * (j - t.lo[1]) + kAnchPXY * (k - t.lo[2]) : q;
        };
        for (int q = threadIdx.x; q < tv; q += blockDim.x) {
            int i, j, k;
            tile_node_small(t, q, i, j, k);
            R v[3];
            node_velocity<R>(S, nb, i, j, k, v);
            lvxy[q] = R2<R>{v[0], v[1]};
            lvz[q] = v[2];
            const int fq = fidx(q, i, j, k);
            lf[0][fq] = lf[1][fq] = lf[2][fq] = 0.0;
        }
        __syncthreads();
        const R dt = cst<R>(S.dt, S.f_dt);
        const R gx = cst<R>(S.g[0], S.f_g[0]), gy = cst<R>(S.g[1], S.f_g[1]), gz = cst<R>(S.g[2], S.f_g[2]);
        uint32_t bad = 0;
        int kb[3] = {-(1 << 30), 0, 0};   // support base held in the gather cache
        int fb[3] = {-(1 << 30), 0, 0};   // support base of the force accumulators
        Corners kc{};
        R cv[GN][3], fa[SN][3];
        auto flush = [&]() {
            for (int n = 0; n < SN; ++n) {
                const int li = kc.t0 + (n & 1) + ((n >> 1) & 1) * kc.ty + (n >> 2) * kc.tz;
                for (int a = 0; a < 3; ++a)
                    atomicAdd(&lf[a][li], (double)fa[n][a]);
            }
        };
#pragma unroll
        for (int rr = 0; rr < KP; ++rr) {
            const uint32_t q = threadIdx.x + rr * T;
            if (q >= item.count)
                break;
            const uint32_t p = item.start + q;
            const double xp[3] = {ldg(P.x[0], p), ldg(P.x[1], p), ldg(P.x[2], p)};
            // every input of the particle in one round trip, except on
            // isoparametric cells, whose inverse Jacobian leaves no registers
            // for them (one wavefront per SIMD fewer, measured slower)
            R vol0 = 0, sg[6] = {0, 0, 0, 0, 0, 0}, mp = 0;
            if constexpr (SH != 2) {
                vol0 = ldg(P.vol, p);
                for (int k = 0; k < 6; ++k)
                    sg[k] = ldg(P.sig[k], p);
                mp = ldg(P.mass, p);
            }
            __builtin_amdgcn_sched_barrier(0);   // the particle's loads in one round trip
            int c[3];
            unpack_cell(pcell[rr], c);
            Support<R, SH> sp;
            make_support<R, SH>(S, xp, c, sp);
            const Corners cn = corners(S, t, sp.base);
            if constexpr (GC) {
                if (!same_base(sp.base, kb)) {
                    for (int a = 0; a < 3; ++a)
                        kb[a] = sp.base[a];
                    for (int n = 0; n < GN; ++n) {
                        const int li = cn.t0 + (n & 1) + ((n >> 1) & 1) * cn.ty + (n >> 2) * cn.tz;
                        const R2<R> v = lvxy[li];
                        cv[n][0] = v.s;
                        cv[n][1] = v.t;
                        cv[n][2] = lvz[li];
                    }
                }
            }
            if constexpr (SC) {
                if (!same_base(sp.base, fb)) {
                    if (fb[0] != -(1 << 30))
                        flush();
                    for (int a = 0; a < 3; ++a)
                        fb[a] = sp.base[a];
                    kc = cn;
                    for (int n = 0; n < SN; ++n)
                        fa[n][0] = fa[n][1] = fa[n][2] = (R)0;
                }
            }
            R L[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
            // linear shape functions: dN/dx_a is +-1/h times the product of the
            // other two axes' weights (pair products below, shared with the
            // force), so the gradient is a weighted sum of nodal differences
            R Pyz[4], Pxz[4], Pxy[4];
            if constexpr (SH != 1) {
                for (int u = 0; u < 2; ++u)
                    for (int w = 0; w < 2; ++w) {
                        Pyz[u + 2 * w] = sp.w[1][u] * sp.w[2][w];
                        Pxz[u + 2 * w] = sp.w[0][u] * sp.w[2][w];
                        Pxy[u + 2 * w] = sp.w[0][u] * sp.w[1][w];
                    }
                R v8[8][3];
                for (int n = 0; n < 8; ++n) {
                    if constexpr (GC) {
                        v8[n][0] = cv[n][0];
                        v8[n][1] = cv[n][1];
                        v8[n][2] = cv[n][2];
                    } else {
                        const int li = cn.t0 + (n & 1) + ((n >> 1) & 1) * cn.ty + (n >> 2) * cn.tz;
                        const R2<R> w = lvxy[li];
                        v8[n][0] = w.s;
                        v8[n][1] = w.t;
                        v8[n][2] = lvz[li];
                    }
                }
                const R ih = cst<R>(S.inv_h, S.f_inv_h);
                for (int e = 0; e < 3; ++e) {
                    R gx = 0, gy = 0, gz = 0;
                    for (int u = 0; u < 2; ++u)
                        for (int w = 0; w < 2; ++w) {
                            gx += Pyz[u + 2 * w] * (v8[1 + 2 * u + 4 * w][e] - v8[2 * u + 4 * w][e]);
                            gy += Pxz[u + 2 * w] * (v8[u + 2 + 4 * w][e] - v8[u + 4 * w][e]);
                            gz += Pxy[u + 2 * w] * (v8[u + 2 * w + 4][e] - v8[u + 2 * w][e]);
                        }
                    if constexpr (SH == 2) {   // d/dr to d/dx through (dx/dr)^-1
                        for (int b = 0; b < 3; ++b)
                            L[e][b] = gx * sp.Ji[0][b] + gy * sp.Ji[1][b] + gz * sp.Ji[2][b];
                    } else {
                        L[e][0] = ih * gx;
                        L[e][1] = ih * gy;
                        L[e][2] = ih * gz;
                    }
                }
            } else {
            // GIMP, row by row of the support: dN/dx = dw_i P1, dN/dy = w_i P2,
            // dN/dz = w_i P3 with the row's (j, k) factors, so each row sums
            // v dw_i and v w_i over i first
            for (int k = 0; k < NS; ++k)
                for (int j = 0; j < NS; ++j) {
                    const R P1 = sp.w[1][j] * sp.w[2][k], P2 = sp.dw[1][j] * sp.w[2][k],
                            P3 = sp.w[1][j] * sp.dw[2][k];
                    R Sx[3] = {0, 0, 0}, Sw[3] = {0, 0, 0};
                    for (int i = 0; i < NS; ++i) {
                        const int li = cn.t0 + i + j * cn.ty + k * cn.tz;
                        const R2<R> w = lvxy[li];
                        const R v[3] = {w.s, w.t, lvz[li]};
                        for (int e = 0; e < 3; ++e) {
                            Sx[e] += v[e] * sp.dw[0][i];
                            Sw[e] += v[e] * sp.w[0][i];
                        }
                    }
                    for (int e = 0; e < 3; ++e) {
                        L[e][0] += Sx[e] * P1;
                        L[e][1] += Sw[e] * P2;
                        L[e][2] += Sw[e] * P3;
                    }
                    __builtin_amdgcn_sched_barrier(0);   // one support row of LDS reads in flight
                }
            }
            const R de[6] = {dt * L[0][0], dt * L[1][1], dt * L[2][2], dt * (L[0][1] + L[1][0]),
                             dt * (L[1][2] + L[2][1]), dt * (L[0][2] + L[2][0])};
            if constexpr (SH == 2) {
                vol0 = ldg(P.vol, p);
                for (int k = 0; k < 6; ++k)
                    sg[k] = ldg(P.sig[k], p);
            }
            const R vol = vol0 * ((R)1 + de[0] + de[1] + de[2]);
            constitutive<R>(S, de, sg);
            for (int k = 0; k < 6; ++k) {
                stg(P.sig[k], p, sg[k]);
                if (!isfinite(sg[k]))
                    bad = ERR_NONFINITE;
            }
            stg(P.vol, p, vol);
            if constexpr (SH == 2)
                mp = ldg(P.mass, p);
            auto deposit = [&](int i, int j, int k, R f0, R f1, R f2) {
                if constexpr (SC) {
                    const int n = i + 2 * j + 4 * k;
                    fa[n][0] += f0;
                    fa[n][1] += f1;
                    fa[n][2] += f2;
                } else {
                    const int li = cn.t0 + i + j * cn.ty + k * cn.tz;
                    atomicAdd(&lf[0][li], (double)f0);
                    atomicAdd(&lf[1][li], (double)f1);
                    atomicAdd(&lf[2][li], (double)f2);
                }
            };
            if constexpr (SH != 1) {
                // f_I = -V sigma . grad N_I + N_I m g with grad N_I = (1/h) (sx Pyz,
                // sy Pxz, sz Pxy), s = -1 for the lower node of an axis; on an
                // isoparametric cell grad N_I = Ji^T (sx Pyz, sy Pxz, sz Pxy), so
                // f_Ia = sum_c B_ac dN_I/dr_c with B = -V sigma Ji^T
                R B[3][3];
                if constexpr (SH == 2) {
                    const R sm[3][3] = {{sg[0], sg[3], sg[5]}, {sg[3], sg[1], sg[4]}, {sg[5], sg[4], sg[2]}};
                    for (int a = 0; a < 3; ++a)
                        for (int c2 = 0; c2 < 3; ++c2)
                            B[a][c2] = -vol * (sm[a][0] * sp.Ji[c2][0] + sm[a][1] * sp.Ji[c2][1] +
                                               sm[a][2] * sp.Ji[c2][2]);
                } else {
                    const R c = -vol * cst<R>(S.inv_h, S.f_inv_h);
                    B[0][0] = c * sg[0];
                    B[1][1] = c * sg[1];
                    B[2][2] = c * sg[2];
                    B[0][1] = B[1][0] = c * sg[3];
                    B[1][2] = B[2][1] = c * sg[4];
                    B[0][2] = B[2][0] = c * sg[5];
                }
                const R mg0 = mp * gx, mg1 = mp * gy, mg2 = mp * gz;
                for (int k = 0; k < 2; ++k)
                    for (int j = 0; j < 2; ++j)
                        for (int i = 0; i < 2; ++i) {
                            const R yz = Pyz[j + 2 * k], xz = Pxz[i + 2 * k], xy = Pxy[i + 2 * j];
                            const R ax = i ? yz : -yz, ay = j ? xz : -xz, az = k ? xy : -xy;
                            const R N = sp.w[0][i] * yz;
                            deposit(i, j, k, N * mg0 + B[0][0] * ax + B[0][1] * ay + B[0][2] * az,
                                    N * mg1 + B[1][0] * ax + B[1][1] * ay + B[1][2] * az,
                                    N * mg2 + B[2][0] * ax + B[2][1] * ay + B[2][2] * az);
                        }
            } else if (anch) {
                // the 27 support nodes in rotated order (see kAnchPX): on each
                // axis slots 0 and 1 are the nodes c and c + 1, slot 2 the
                // node c + 2 (support from c) or c - 1 (support from c - 1), so
                // a wavefront's lanes mostly add to one translate of their
                // cells.  f_a = A_a0 dN/dx + A_a1 dN/dy + A_a2 dN/dz + N m g_a
                // with A = -V sigma, dN/dx = dw_i P1, dN/dy = w_i P2,
                // dN/dz = w_i P3, N = w_i P1: the row's (j, k) factors once,
                // then two terms per slot
                R wr[3][3], dr[3][3];
                int e[3];
                for (int a = 0; a < 3; ++a)
                    e[a] = rotate3<R>(sp.w[a], sp.dw[a], sp.base[a] == c[a], wr[a], dr[a]);
                R A[6];
                for (int k = 0; k < 6; ++k)
                    A[k] = -vol * sg[k];
                const R mg[3] = {mp * gx, mp * gy, mp * gz};
                const int a0 = (c[0] - 1 - t.lo[0]) + kAnchPX * (c[1] - 1 - t.lo[1]) + kAnchPXY * (c[2] - 1 - t.lo[2]);
                const int ox[3] = {1, 2, e[0]}, oy[3] = {kAnchPX, 2 * kAnchPX, kAnchPX * e[1]},
                          oz[3] = {kAnchPXY, 2 * kAnchPXY, kAnchPXY * e[2]};
                for (int k = 0; k < 3; ++k)
                    for (int j = 0; j < 3; ++j) {
                        const R P1 = wr[1][j] * wr[2][k], P2 = dr[1][j] * wr[2][k], P3 = wr[1][j] * dr[2][k];
                        const R X[3] = {A[0] * P1, A[3] * P1, A[5] * P1};
                        const R Y[3] = {A[3] * P2 + A[5] * P3 + mg[0] * P1, A[1] * P2 + A[4] * P3 + mg[1] * P1,
                                        A[4] * P2 + A[2] * P3 + mg[2] * P1};
                        const int rb = a0 + oy[j] + oz[k];
                        for (int i = 0; i < 3; ++i) {
                            const int li = rb + ox[i];
                            atomicAdd(&lf[0][li], (double)(dr[0][i] * X[0] + wr[0][i] * Y[0]));
                            atomicAdd(&lf[1][li], (double)(dr[0][i] * X[1] + wr[0][i] * Y[1]));
                            atomicAdd(&lf[2][li], (double)(dr[0][i] * X[2] + wr[0][i] * Y[2]));
                        }
                        __builtin_amdgcn_sched_barrier(0);   // one row of LDS adds in flight
                    }
            } else {
            for (int k = 0; k < NS; ++k)
                for (int j = 0; j < NS; ++j)
                    for (int i = 0; i < NS; ++i) {
                        const R wyz = sp.w[1][j] * sp.w[2][k];
                        const R N = sp.w[0][i] * wyz;
                        const R gxN = sp.dw[0][i] * wyz;
                        const R gyN = sp.w[0][i] * sp.dw[1][j] * sp.w[2][k];
                        const R gzN = sp.w[0][i] * sp.w[1][j] * sp.dw[2][k];
                        const R f0 = -vol * (sg[0] * gxN + sg[3] * gyN + sg[5] * gzN) + N * mp * gx;
                        const R f1 = -vol * (sg[3] * gxN + sg[1] * gyN + sg[4] * gzN) + N * mp * gy;
                        const R f2 = -vol * (sg[5] * gxN + sg[4] * gyN + sg[2] * gzN) + N * mp * gz;
                        deposit(i, j, k, f0, f1, f2);
                        if constexpr (SH == 1)
                            if (i == NS - 1)
                                __builtin_amdgcn_sched_barrier(0);   // one support layer of LDS reads in flight
                    }
            }
        }
        if constexpr (SC)
            if (fb[0] != -(1 << 30))
                flush();
        if (bad)
            atomicOr(&S.ctl[CTL_ERR], bad);
        __syncthreads();
        for (int q = threadIdx.x; q < tv; q += blockDim.x) {
            int i, j, k;
            tile_node_small(t, q, i, j, k);
            const int fq = fidx(q, i, j, k);
            const R f0 = (R)lf[0][fq], f1 = (R)lf[1][fq], f2 = (R)lf[2][fq];
            if (f0 == (R)0 && f1 == (R)0 && f2 == (R)0)
                continue;
            const uint32_t I = node_id(S, i, j, k);
            addg(nb.f[0], I, f0);
            addg(nb.f[1], I, f1);
            addg(nb.f[2], I, f2);
        }
        __syncthreads();
    }
}

// Load the acceleration and updated velocity of the item's node tile.
template <typename R>
__device__ inline void load_update_tile(const SceneDev &S, const NodeBuf<R> &nb, const Tile &t, R4<R> *la,
                                        R4<R> *lvn)
{
    const int tv = t.dim[0] * t.dim[1] * t.dim[2];
    for (int q = threadIdx.x; q < tv; q += blockDim.x) {
        int i, j, k;
        tile_node_small(t, q, i, j, k);
        R a[3], vn[3];
        node_update<R>(S, nb, i, j, k, a, vn);
        la[q] = R4<R>{a[0], a[1], a[2], (R)0};
        lvn[q] = R4<R>{vn[0], vn[1], vn[2], (R)0};
    }
}

// Load the acceleration and updated velocity of the item's node tile into
// 24 bytes per node (FP32): a and vn.x in la, vn.y and vn.z in lyz.
template <typename R>
__device__ inline void load_update_tile_packed(const SceneDev &S, const NodeBuf<R> &nb, const Tile &t, R4<R> *la,
                                               R2<R> *lyz)
{
    const int tv = t.dim[0] * t.dim[1] * t.dim[2];
    for (int q = threadIdx.x; q < tv; q += blockDim.x) {
        int i, j, k;
        tile_node_small(t, q, i, j, k);
        R a[3], vn[3];
        node_update<R>(S, nb, i, j, k, a, vn);
        la[q] = R4<R>{a[0], a[1], a[2], vn[0]};
        lyz[q] = R2<R>{vn[1], vn[2]};
    }
}

// USF: particle velocity (FLIP/PIC) and position from the nodal acceleration
// and updated velocity; new cell, error and reorder flags; then the next
// step's nodal mass and momentum from the updated particle into the other
// (zeroed) node buffer, through an LDS tile over the item's home region
// (particles that drifted past it add to global memory directly).
template <typename R, int SH, int T>
__global__ void __launch_bounds__(T) k_g2p_p2g(BatchDev B)
{
    constexpr int NS = ShapeTraits<SH>::NS;
    constexpr int CAP = ShapeTraits<SH>::cap;
    constexpr int KP = kChunk / T;
    using C = Cache<SH, kG2PCacheGather, kG2PCacheScatter>;
    constexpr bool GC = C::gather, SC = C::scatter;
    constexpr int GN = C::gnodes, SN = C::snodes;
    // GIMP: the gather tile and the scatter accumulators share LDS (all
    // particles are updated before the scatter starts), which admits one
    // more workgroup per CU
    constexpr bool OVERLAY = SH == 1;
    // home-tile accumulators: edge HD, at row and plane pitches APX, APXY
    // (GIMP: the anchored layout, see kAnchPX)
    constexpr int HD = kBrick + 2 + ShapeTraits<SH>::lo + ShapeTraits<SH>::hi;   // home tile edge
    constexpr int APX = SH == 1 ? kAnchPX : HD, APXY = SH == 1 ? kAnchPXY : HD * HD;
    constexpr int ACAP = APXY * HD;
    static_assert(SH != 1 || (HD == 9 && ACAP == kAnchCap), "anchored layout holds the GIMP home tile");
    // the gather tile packs a node's acceleration and updated velocity in
    // 24 bytes (FP32), which leaves room for one more workgroup per CU
    constexpr int TILE_BYTES = CAP * (int)(sizeof(R4<R>) + sizeof(R2<R>)), ACC_BYTES = 4 * ACAP * (int)sizeof(double);
    static_assert((CAP * sizeof(R4<R>)) % alignof(R2<R>) == 0 && TILE_BYTES % alignof(double) == 0, "tile alignment");
    __shared__ __attribute__((aligned(16))) char lds[OVERLAY ? (TILE_BYTES > ACC_BYTES ? TILE_BYTES : ACC_BYTES)
                                                             : TILE_BYTES + ACC_BYTES];
    R4<R> *la = (R4<R> *)lds;
    R2<R> *lyz = (R2<R> *)(lds + CAP * sizeof(R4<R>));
    double (*acc)[ACAP] = (double (*)[ACAP])(lds + (OVERLAY ? 0 : TILE_BYTES));
    __shared__ int red[6 * (T / 64)];
    // the accumulators start at zero, and each item's flush leaves them so
    // (with OVERLAY the tile overwrites them, so every item zeroes them)
    if constexpr (!OVERLAY)
        for (int q = threadIdx.x; q < ACAP; q += blockDim.x)
            acc[0][q] = acc[1][q] = acc[2][q] = acc[3][q] = 0.0;
    const int64_t total = B.ioffs[B.nscenes];
    const ItemRange ir = item_range(total);
    for (int64_t g = ir.first; g < ir.end; g += ir.step) {
        const ItemRef r = item_ref(B.ioffs, B, g);
        const SceneDev S = load_scene(r.S);
        if (!scene_active(S))
            continue;
        const Item item = cld_struct(&S.items[r.it]);
        const Tile t = cld_struct(&S.tstep[r.it]);
        if (!t.fits)
            continue;
        const int cur = (int)cld(&S.ctl[CTL_CUR]);
        const int buf = (int)cld(&S.ctl[CTL_NBUF]), nbuf = buf ^ 1;
        const Parts<R> P = parts<R>(S, cur);
        const NodeBuf<R> nb = node_buf<R>(S, buf);
        const NodeBuf<R> nn = node_buf<R>(S, nbuf);
        int o[3];
        brick_origin(S, item.brick, o);
        const Tile ht = home_tile<SH>(o);
        load_update_tile_packed<R>(S, nb, t, la, lyz);
        __syncthreads();
        const R dt = cst<R>(S.dt, S.f_dt);
        const int pic = S.vel_update == 1;
        uint32_t err = 0, drift = 0, lost = 0;
        int mn[3] = {1 << 30, 1 << 30, 1 << 30}, mx[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
        // gather cache (old support) and scatter cache (new support)
        int gb[3] = {-(1 << 30), 0, 0}, sb[3] = {-(1 << 30), 0, 0};
        R ca[GN][3], cu[GN][3], sp_[SN][3], sm[SN];
        Corners sc{};
        bool s_in = true;
        // the moved particles awaiting the scatter (OVERLAY)
        struct Moved {
            double x[3];
            R m, mv[3];
            int c[3];
            bool ok, in;
        };
        Moved mvd[OVERLAY ? KP : 1];
        if constexpr (OVERLAY)
            for (int rr = 0; rr < KP; ++rr)
                mvd[rr].ok = false;
        // next step's mass and momentum of one particle with support sp:
        // into the home tile's accumulators, or (drifted) global memory
        auto scatter = [&](const Support<R, SH> &sq, const int cq[3], bool inh, R m, const R mvq[3]) {
            const Corners hq = corners(S, ht, sq.base);
            if (SH == 1 && inh) {
                // anchored 4 x 4 x 4 slots (see kAnchPX); home-tile coordinates
                // of node c - 1 are c - o + 1 in [0, 5] for a cell in the home region
                R w4[3][4], dw4[3][4];
                for (int a = 0; a < 3; ++a)
                    anchor4<R>(sq.w[a], sq.dw[a], sq.base[a] == cq[a] ? 1 : 0, w4[a], dw4[a]);
                const int a0 = (cq[0] - 1 - ht.lo[0]) + APX * (cq[1] - 1 - ht.lo[1]) + APXY * (cq[2] - 1 - ht.lo[2]);
                for (int k = 0; k < 4; ++k)
                    for (int j = 0; j < 4; ++j) {
                        const R wyz = w4[1][j] * w4[2][k];
                        for (int i = 0; i < 4; ++i) {
                            const R N = w4[0][i] * wyz;
                            const int li = a0 + i + APX * j + APXY * k;
                            atomicAdd(&acc[0][li], (double)(N * m));
                            atomicAdd(&acc[1][li], (double)(N * mvq[0]));
                            atomicAdd(&acc[2][li], (double)(N * mvq[1]));
                            atomicAdd(&acc[3][li], (double)(N * mvq[2]));
                        }
                        __builtin_amdgcn_sched_barrier(0);   // one row of LDS adds in flight
                    }
            } else if (inh) {
                for (int k = 0; k < NS; ++k)
                    for (int j = 0; j < NS; ++j)
                        for (int i = 0; i < NS; ++i) {
                            const R N = sq.w[0][i] * sq.w[1][j] * sq.w[2][k];
                            const int li = hq.t0 + i + j * hq.ty + k * hq.tz;
                            atomicAdd(&acc[0][li], (double)(N * m));
                            atomicAdd(&acc[1][li], (double)(N * mvq[0]));
                            atomicAdd(&acc[2][li], (double)(N * mvq[1]));
                            atomicAdd(&acc[3][li], (double)(N * mvq[2]));
                        }
            } else {
                for (int k = 0; k < NS; ++k)
                    for (int j = 0; j < NS; ++j)
                        for (int i = 0; i < NS; ++i) {
                            const R N = sq.w[0][i] * sq.w[1][j] * sq.w[2][k];
                            const uint32_t I = hq.n0 + (uint32_t)(i + j * hq.ny + k * hq.nz);
                            addg(nn.m, I, (double)(N * m));
                            for (int a = 0; a < 3; ++a)
                                addg(nn.p[a], I, N * mvq[a]);
                        }
            }
        };
        // two particles in one home cell (GIMP): one set of anchored adds
        // carries the sum of their contributions
        auto scatter_pair = [&](const Support<R, SH> &sa, const Support<R, SH> &sb, const int cq[3], R ma,
                                const R mva[3], R mb, const R mvb[3]) {
            R wa[3][4], wb[3][4], unused[4];
            for (int a = 0; a < 3; ++a) {
                anchor4<R>(sa.w[a], sa.dw[a], sa.base[a] == cq[a] ? 1 : 0, wa[a], unused);
                anchor4<R>(sb.w[a], sb.dw[a], sb.base[a] == cq[a] ? 1 : 0, wb[a], unused);
            }
            const int a0 = (cq[0] - 1 - ht.lo[0]) + APX * (cq[1] - 1 - ht.lo[1]) + APXY * (cq[2] - 1 - ht.lo[2]);
            for (int k = 0; k < 4; ++k)
                for (int j = 0; j < 4; ++j) {
                    const R ya = wa[1][j] * wa[2][k], yb = wb[1][j] * wb[2][k];
                    for (int i = 0; i < 4; ++i) {
                        const R Na = wa[0][i] * ya, Nb = wb[0][i] * yb;
                        const int li = a0 + i + APX * j + APXY * k;
                        atomicAdd(&acc[0][li], (double)(Na * ma + Nb * mb));
                        atomicAdd(&acc[1][li], (double)(Na * mva[0] + Nb * mvb[0]));
                        atomicAdd(&acc[2][li], (double)(Na * mva[1] + Nb * mvb[1]));
                        atomicAdd(&acc[3][li], (double)(Na * mva[2] + Nb * mvb[2]));
                    }
                    __builtin_amdgcn_sched_barrier(0);   // one row of LDS adds in flight
                }
        };
        auto flush = [&]() {
            for (int n = 0; n < SN; ++n) {
                const int di = n & 1, dj = (n >> 1) & 1, dk = n >> 2;
                if (s_in) {
                    const int li = sc.t0 + di + dj * sc.ty + dk * sc.tz;
                    atomicAdd(&acc[0][li], (double)sm[n]);
                    for (int a = 0; a < 3; ++a)
                        atomicAdd(&acc[1 + a][li], (double)sp_[n][a]);
                } else {
                    const uint32_t I = sc.n0 + (uint32_t)(di + dj * sc.ny + dk * sc.nz);
                    addg(nn.m, I, (double)sm[n]);
                    for (int a = 0; a < 3; ++a)
                        addg(nn.p[a], I, sp_[n][a]);
                }
            }
        };
#pragma unroll
        for (int rr = 0; rr < KP; ++rr) {
            const uint32_t q = threadIdx.x + rr * T;
            if (q >= item.count)
                break;
            const uint32_t p = item.start + q;
            double xp[3] = {ldg(P.x[0], p), ldg(P.x[1], p), ldg(P.x[2], p)};
            const R pv[3] = {ldg(P.v[0], p), ldg(P.v[1], p), ldg(P.v[2], p)};
            const R mp = ldg(P.mass, p);
            const uint32_t pc = ldg(P.cell, p);
            __builtin_amdgcn_sched_barrier(0);   // the particle's loads in one round trip
            int c[3];
            unpack_cell(pc, c);
            Support<R, SH> sp;
            make_support<R, SH>(S, xp, c, sp);
            pin_loaded(pv);
            const Corners cn = corners(S, t, sp.base);
            if constexpr (GC) {
                if (!same_base(sp.base, gb)) {
                    for (int a = 0; a < 3; ++a)
                        gb[a] = sp.base[a];
                    for (int n = 0; n < GN; ++n) {
                        const int li = cn.t0 + (n & 1) + ((n >> 1) & 1) * cn.ty + (n >> 2) * cn.tz;
                        const R4<R> a4 = la[li];
                        const R2<R> u2 = lyz[li];
                        ca[n][0] = a4.x;
                        ca[n][1] = a4.y;
                        ca[n][2] = a4.z;
                        cu[n][0] = a4.w;
                        cu[n][1] = u2.s;
                        cu[n][2] = u2.t;
                    }
                }
            }
            R dv[3] = {0, 0, 0}, vp[3] = {0, 0, 0};
            for (int k = 0; k < NS; ++k)
                for (int j = 0; j < NS; ++j)
                    for (int i = 0; i < NS; ++i) {
                        const R N = sp.w[0][i] * sp.w[1][j] * sp.w[2][k];
                        R a[3], u[3];
                        if constexpr (GC) {
                            const int n = i + 2 * j + 4 * k;
                            for (int e = 0; e < 3; ++e) {
                                a[e] = ca[n][e];
                                u[e] = cu[n][e];
                            }
                        } else {
                            const int li = cn.t0 + i + j * cn.ty + k * cn.tz;
                            const R4<R> a4 = la[li];
                            const R2<R> u2 = lyz[li];
                            a[0] = a4.x;
                            a[1] = a4.y;
                            a[2] = a4.z;
                            u[0] = a4.w;
                            u[1] = u2.s;
                            u[2] = u2.t;
                        }
                        for (int e = 0; e < 3; ++e) {
                            dv[e] += N * a[e];
                            vp[e] += N * u[e];
                        }
                        if constexpr (SH == 1)
                            if (i == NS - 1)
                                __builtin_amdgcn_sched_barrier(0);   // one support layer of LDS reads in flight
                    }
            R nv[3];
            for (int a = 0; a < 3; ++a) {
                nv[a] = pic ? vp[a] : pv[a] + dt * dv[a];
                stg(P.v[a], p, nv[a]);
                xp[a] += S.dt * (double)vp[a];
                stg(P.x[a], p, xp[a]);
                if (!isfinite(nv[a]))
                    err |= ERR_NONFINITE;
            }
            int nc[3];
            double fr[3];
            uint32_t e;
            if constexpr (SH == 2) {   // walk from the old cell; fr: local coordinates in the new one
                IsoCell k;
                for (int a = 0; a < 3; ++a)
                    nc[a] = c[a];
                e = iso_locate(S, xp, nc, fr, k, kIsoWalk);
            } else {
                e = locate<SH == 0>(S, xp, nc, fr);
            }
            if (e) {
                err |= e;   // keep the old cell; the scene stops after this step
                lost += (e & ERR_OUT_OF_MESH) ? 1u : 0u;
                continue;
            }
            stg(P.cell, p, pack_cell(nc));
            for (int a = 0; a < 3; ++a) {
                mn[a] = min(mn[a], nc[a]);
                mx[a] = max(mx[a], nc[a]);
            }
            const bool in = in_home(nc, o);
            drift |= in ? 0u : 1u;
            if constexpr (OVERLAY) {
                Moved &mq = mvd[rr];
                for (int a = 0; a < 3; ++a) {
                    mq.x[a] = xp[a];
                    mq.c[a] = nc[a];
                    mq.mv[a] = mp * nv[a];
                }
                mq.m = mp;
                mq.in = in;
                mq.ok = true;
                continue;
            }
            // the next step's P2G from the updated particle (trilinear: the
            // local coordinate is the cell search's fractional part, or the
            // isoparametric walk's local coordinates)
            if constexpr (SH != 1) {
                const R ih = cst<R>(S.inv_h, S.f_inv_h);
                for (int a = 0; a < 3; ++a) {
                    const R r = (R)fr[a];
                    sp.base[a] = nc[a];
                    sp.w[a][0] = (R)1 - r;
                    sp.w[a][1] = r;
                    sp.dw[a][0] = -ih;
                    sp.dw[a][1] = ih;
                }
            } else {
                make_support<R, SH>(S, xp, nc, sp);
            }
            const Corners hn = corners(S, ht, sp.base);
            const R mv[3] = {mp * nv[0], mp * nv[1], mp * nv[2]};
            if constexpr (SC) {
                if (!same_base(sp.base, sb)) {
                    if (sb[0] != -(1 << 30))
                        flush();
                    for (int a = 0; a < 3; ++a)
                        sb[a] = sp.base[a];
                    sc = hn;
                    s_in = in;
                    for (int n = 0; n < SN; ++n) {
                        sm[n] = (R)0;
                        sp_[n][0] = sp_[n][1] = sp_[n][2] = (R)0;
                    }
                }
            }
            if constexpr (SC) {
                for (int k = 0; k < NS; ++k)
                    for (int j = 0; j < NS; ++j)
                        for (int i = 0; i < NS; ++i) {
                            const R N = sp.w[0][i] * sp.w[1][j] * sp.w[2][k];
                            const int n = i + 2 * j + 4 * k;
                            sm[n] += N * mp;
                            for (int a = 0; a < 3; ++a)
                                sp_[n][a] += N * mv[a];
                        }
            } else {
                scatter(sp, nc, in, mp, mv);
            }
        }
        if constexpr (OVERLAY) {
            // every gather from the tile is done: the same LDS now accumulates
            __syncthreads();
            for (int q = threadIdx.x; q < ACAP; q += blockDim.x)
                acc[0][q] = acc[1][q] = acc[2][q] = acc[3][q] = 0.0;
            __syncthreads();
            // particles rr and rr + 1 of a thread are successive particles of
            // one cell in level-major order, and most stay in it: such a pair
            // shares one set of anchored adds (half the LDS atomics)
#pragma unroll
            for (int rr = 0; rr < KP; rr += 2) {
                if (rr + 1 < KP && mvd[rr].ok && mvd[rr + 1].ok && mvd[rr].in && mvd[rr + 1].in &&
                    same_base(mvd[rr].c, mvd[rr + 1].c)) {
                    Support<R, SH> sa, sb;
                    make_support<R, SH>(S, mvd[rr].x, mvd[rr].c, sa);
                    make_support<R, SH>(S, mvd[rr + 1].x, mvd[rr + 1].c, sb);
                    scatter_pair(sa, sb, mvd[rr].c, mvd[rr].m, mvd[rr].mv, mvd[rr + 1].m, mvd[rr + 1].mv);
                    continue;
                }
#pragma unroll
                for (int r2 = rr; r2 < rr + 2 && r2 < KP; ++r2)
                    if (mvd[r2].ok) {
                        Support<R, SH> sq;
                        make_support<R, SH>(S, mvd[r2].x, mvd[r2].c, sq);
                        scatter(sq, mvd[r2].c, mvd[r2].in, mvd[r2].m, mvd[r2].mv);
                    }
            }
        }
        if constexpr (SC)
            if (sb[0] != -(1 << 30))
                flush();
        if (err)
            atomicOr(&S.ctl[CTL_ERR], err);
        if (lost)
            atomicAdd(&S.ctl[CTL_LOST], lost);
        if (drift || (S.sort_always && threadIdx.x == 0)) {
            S.ctl[CTL_NEED_SORT] = 1u;
            B.flags[BF_ANY_SORT] = 1u;
        }
        int blo[3], bhi[3];
        item_box<T>(mn, mx, red, blo, bhi);
        if (threadIdx.x == 0) {
            pick(S.tiles, nbuf)[r.it] = tile_of_cells<SH>(blo, bhi);
            if (r.it == 0) {
                S.ctl[CTL_ACC0 + nbuf] = S.ctl[CTL_N_ITEMS];
                S.ctl[CTL_READY] = 1u;
            }
        }
        // flush the home-tile entries the moved particles can have touched
        // (their cells' node box), zeroing them for the next item
        const Tile nbx = tile_of_cells<SH>(blo, bhi);
        Tile fb;   // nbx within the home tile, in home-tile coordinates
        for (int a = 0; a < 3; ++a) {
            fb.lo[a] = max(nbx.lo[a], ht.lo[a]) - ht.lo[a];
            fb.dim[a] = max(min(nbx.lo[a] + nbx.dim[a], ht.lo[a] + HD) - ht.lo[a] - fb.lo[a], 0);
        }
        const int fv = fb.dim[0] * fb.dim[1] * fb.dim[2];
        for (int q = threadIdx.x; q < fv; q += blockDim.x) {
            int a, b, c;
            tile_node_small(fb, q, a, b, c);
            const int li = a + APX * b + APXY * c;
            const double m = acc[0][li];
            const int i = ht.lo[0] + a, j = ht.lo[1] + b, k = ht.lo[2] + c;
            if (m != 0.0 && node_in_mesh(S, i, j, k)) {
                const uint32_t I = node_id(S, i, j, k);
                addg(nn.m, I, m);
                for (int e = 0; e < 3; ++e)
                    addg(nn.p[e], I, (R)acc[1 + e][li]);
            }
            if constexpr (!OVERLAY)
                acc[0][li] = acc[1][li] = acc[2][li] = acc[3][li] = 0.0;
        }
        __syncthreads();
    }
}

// USL: particle velocity and position, then the strain increment from the
// updated nodal velocity and the stress update; zeroes the previous step's
// node buffer.
template <typename R, int SH, int T>
__global__ void __launch_bounds__(T) k_g2p_usl(BatchDev B)
{
    constexpr int NS = ShapeTraits<SH>::NS;
    constexpr int CAP = ShapeTraits<SH>::cap;
    __shared__ R4<R> la[CAP];
    __shared__ R4<R> lvn[CAP];
    clear_previous<R>(B);
    const int64_t total = B.ioffs[B.nscenes];
    const ItemRange ir = item_range(total);
    for (int64_t g = ir.first; g < ir.end; g += ir.step) {
        const ItemRef r = item_ref(B.ioffs, B, g);
        const SceneDev S = load_scene(r.S);
        if (!scene_active(S))
            continue;
        const Item item = cld_struct(&S.items[r.it]);
        const int buf = (int)cld(&S.ctl[CTL_NBUF]);
        const Tile t = pick(S.tiles, buf)[r.it];
        if (!t.fits)
            continue;
        const int cur = (int)cld(&S.ctl[CTL_CUR]);
        const Parts<R> P = parts<R>(S, cur);
        const NodeBuf<R> nb = node_buf<R>(S, buf);
        int o[3];
        brick_origin(S, item.brick, o);
        load_update_tile<R>(S, nb, t, la, lvn);
        __syncthreads();
        const R dt = cst<R>(S.dt, S.f_dt);
        const int pic = S.vel_update == 1;
        uint32_t err = 0, drift = 0, lost = 0;
        for (uint32_t q = threadIdx.x; q < item.count; q += blockDim.x) {
            const uint32_t p = item.start + q;
            double xp[3] = {ldg(P.x[0], p), ldg(P.x[1], p), ldg(P.x[2], p)};
            const R pv[3] = {ldg(P.v[0], p), ldg(P.v[1], p), ldg(P.v[2], p)};
            // volume and stress with the position, except under GIMP, whose
            // support sums leave no registers for them (one wavefront per
            // SIMD fewer, measured slower)
            R vol0 = 0, sg[6] = {0, 0, 0, 0, 0, 0};
            if constexpr (SH != 1) {
                vol0 = ldg(P.vol, p);
                for (int k = 0; k < 6; ++k)
                    sg[k] = ldg(P.sig[k], p);
            }
            const uint32_t pc = ldg(P.cell, p);
            __builtin_amdgcn_sched_barrier(0);   // the particle's loads in one round trip
            int c[3];
            unpack_cell(pc, c);
            Support<R, SH> sp;
            make_support<R, SH>(S, xp, c, sp);
            pin_loaded(pv);
            const Corners cn = corners(S, t, sp.base);
            R dv[3] = {0, 0, 0}, vp[3] = {0, 0, 0};
            R L[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
            for (int k = 0; k < NS; ++k)
                for (int j = 0; j < NS; ++j)
                    for (int i = 0; i < NS; ++i) {
                        const R wyz = sp.w[1][j] * sp.w[2][k];
                        const R N = sp.w[0][i] * wyz;
                        R gxN = sp.dw[0][i] * wyz;
                        R gyN = sp.w[0][i] * sp.dw[1][j] * sp.w[2][k];
                        R gzN = sp.w[0][i] * sp.w[1][j] * sp.dw[2][k];
                        to_dx<R, SH>(sp, gxN, gyN, gzN);
                        const int li = cn.t0 + i + j * cn.ty + k * cn.tz;
                        const R4<R> a = la[li];
                        const R4<R> u = lvn[li];
                        dv[0] += N * a.x;
                        dv[1] += N * a.y;
                        dv[2] += N * a.z;
                        vp[0] += N * u.x;
                        vp[1] += N * u.y;
                        vp[2] += N * u.z;
                        L[0][0] += u.x * gxN;
                        L[0][1] += u.x * gyN;
                        L[0][2] += u.x * gzN;
                        L[1][0] += u.y * gxN;
                        L[1][1] += u.y * gyN;
                        L[1][2] += u.y * gzN;
                        L[2][0] += u.z * gxN;
                        L[2][1] += u.z * gyN;
                        L[2][2] += u.z * gzN;
                        if constexpr (SH == 1)
                            if (i == NS - 1)
                                __builtin_amdgcn_sched_barrier(0);   // one support layer of LDS reads in flight
                    }
            pin_sums<R>(dv, vp);
            pin_grad<R>(L);
            for (int a = 0; a < 3; ++a) {
                const R nva = pic ? vp[a] : pv[a] + dt * dv[a];
                stg(P.v[a], p, nva);
                xp[a] += S.dt * (double)vp[a];
                stg(P.x[a], p, xp[a]);
                if (!isfinite(nva))
                    err |= ERR_NONFINITE;
            }
            const R de[6] = {dt * L[0][0], dt * L[1][1], dt * L[2][2], dt * (L[0][1] + L[1][0]),
                             dt * (L[1][2] + L[2][1]), dt * (L[0][2] + L[2][0])};
            if constexpr (SH == 1) {
                vol0 = ldg(P.vol, p);
                for (int k = 0; k < 6; ++k)
                    sg[k] = ldg(P.sig[k], p);
            }
            stg(P.vol, p, vol0 * ((R)1 + de[0] + de[1] + de[2]));
            constitutive<R>(S, de, sg);
            for (int k = 0; k < 6; ++k) {
                stg(P.sig[k], p, sg[k]);
                if (!isfinite(sg[k]))
                    err |= ERR_NONFINITE;
            }
            int nc[3];
            uint32_t e;
            if constexpr (SH == 2) {
                double rr[3];
                IsoCell k;
                for (int a = 0; a < 3; ++a)
                    nc[a] = c[a];
                e = iso_locate(S, xp, nc, rr, k, kIsoWalk);
            } else {
                e = locate(S, xp, nc);
            }
            if (e) {
                err |= e;
                lost += (e & ERR_OUT_OF_MESH) ? 1u : 0u;
                continue;
            }
            stg(P.cell, p, pack_cell(nc));
            drift |= in_home(nc, o) ? 0u : 1u;
        }
        if (err)
            atomicOr(&S.ctl[CTL_ERR], err);
        if (lost)
            atomicAdd(&S.ctl[CTL_LOST], lost);
        if (drift || (S.sort_always && threadIdx.x == 0)) {
            S.ctl[CTL_NEED_SORT] = 1u;
            B.flags[BF_ANY_SORT] = 1u;
        }
        __syncthreads();
    }
}

// GIMP k_musl_g2p for one work item (the gather tile loaded, the block
// synchronized): each particle's velocity from the tile; then, over the same
// LDS, the remap of the updated momenta with the start-of-step weights into
// the anchored slots of each particle's cell, a thread's two particles in
// one cell sharing one set of adds (the 27-slot form at the box's pitches
// when the box does not fit the anchored layout); flushed to the remap array.
template <typename R, int T>
__device__ __attribute__((always_inline)) inline void musl_g2p_gimp_item(const SceneDev &S, const Parts<R> &P,
                                                                         const Item &item, const Tile &t,
                                                                         const R4<R> *la, const R4<R> *lvn,
                                                                         double (*acc)[kAnchCap])
{
    constexpr int NS = ShapeTraits<1>::NS;
    constexpr int KP = kChunk / T;
    const int tv = t.dim[0] * t.dim[1] * t.dim[2];
    const R dt = cst<R>(S.dt, S.f_dt);
    const int pic = S.vel_update == 1;
    uint32_t err = 0;
    R mvs[KP][3];
    uint32_t pcl[KP];
    bool ok[KP];
#pragma unroll
    for (int rr = 0; rr < KP; ++rr) {
        ok[rr] = false;
        pcl[rr] = 0xffffffffu;
        const uint32_t q = threadIdx.x + rr * T;
        if (q >= item.count)
            continue;
        const uint32_t p = item.start + q;
        const double xp[3] = {ldg(P.x[0], p), ldg(P.x[1], p), ldg(P.x[2], p)};
        pcl[rr] = ldg(P.cell, p);
        int c[3];
        unpack_cell(pcl[rr], c);
        Support<R, 1> sp;
        make_support<R, 1>(S, xp, c, sp);
        const Corners cn = corners(S, t, sp.base);
        R dv[3] = {0, 0, 0}, vp[3] = {0, 0, 0};
        for (int k = 0; k < NS; ++k)
            for (int j = 0; j < NS; ++j)
                for (int i = 0; i < NS; ++i) {
                    const R N = sp.w[0][i] * sp.w[1][j] * sp.w[2][k];
                    const int li = cn.t0 + i + j * cn.ty + k * cn.tz;
                    const R4<R> a = la[li];
                    const R4<R> u = lvn[li];
                    dv[0] += N * a.x;
                    dv[1] += N * a.y;
                    dv[2] += N * a.z;
                    vp[0] += N * u.x;
                    vp[1] += N * u.y;
                    vp[2] += N * u.z;
                    if (i == NS - 1)
                        __builtin_amdgcn_sched_barrier(0);   // one support layer of LDS reads in flight
                }
        pin_sums<R>(dv, vp);
        const R mp = ldg(P.mass, p);
        for (int a = 0; a < 3; ++a) {
            const R nva = pic ? vp[a] : ldg(P.v[a], p) + dt * dv[a];
            stg(P.v[a], p, nva);
            mvs[rr][a] = mp * nva;
            if (!isfinite(nva))
                err |= ERR_NONFINITE;
        }
        ok[rr] = true;
    }
    if (err)
        atomicOr(&S.ctl[CTL_ERR], err);
    // every gather from the tile is done: the same LDS now accumulates
    __syncthreads();
    const bool anch = t.dim[0] <= kAnchPX && t.dim[1] <= 9 && t.dim[2] <= 9;
    const int px = anch ? kAnchPX : t.dim[0], pxy = anch ? kAnchPXY : t.dim[0] * t.dim[1];
    auto entry = [&](int i, int j, int k) { return (i - t.lo[0]) + px * (j - t.lo[1]) + pxy * (k - t.lo[2]); };
    for (int q = threadIdx.x; q < tv; q += T) {
        int i, j, k;
        tile_node_small(t, q, i, j, k);
        const int e = entry(i, j, k);
        acc[0][e] = acc[1][e] = acc[2][e] = 0.0;
    }
    __syncthreads();
    // the updated momenta of particle ra, and of rb (>= 0) in its cell
    auto remap = [&](int ra, int rb) {
        int c[3];
        unpack_cell(pcl[ra], c);
        const int np_ = rb >= 0 ? 2 : 1;
        R w4[2][3][4], unused[4];
        Support<R, 1> sq[2];
        for (int u = 0; u < np_; ++u) {
            const uint32_t p = item.start + threadIdx.x + (u ? rb : ra) * T;
            const double xp[3] = {ldg(P.x[0], p), ldg(P.x[1], p), ldg(P.x[2], p)};
            make_support<R, 1>(S, xp, c, sq[u]);
            for (int a = 0; a < 3; ++a)
                anchor4<R>(sq[u].w[a], sq[u].dw[a], sq[u].base[a] == c[a] ? 1 : 0, w4[u][a], unused);
        }
        if (anch) {
            const int a0 = entry(c[0] - 1, c[1] - 1, c[2] - 1);
            for (int k = 0; k < 4; ++k)
                for (int j = 0; j < 4; ++j) {
                    R y[2];
                    for (int u = 0; u < np_; ++u)
                        y[u] = w4[u][1][j] * w4[u][2][k];
                    for (int i = 0; i < 4; ++i) {
                        R s0 = (R)0, s1 = (R)0, s2 = (R)0;
                        for (int u = 0; u < np_; ++u) {
                            const R N = w4[u][0][i] * y[u];
                            const int ru = u ? rb : ra;
                            s0 += N * mvs[ru][0];
                            s1 += N * mvs[ru][1];
                            s2 += N * mvs[ru][2];
                        }
                        const int li = a0 + i + kAnchPX * j + kAnchPXY * k;
                        atomicAdd(&acc[0][li], (double)s0);
                        atomicAdd(&acc[1][li], (double)s1);
                        atomicAdd(&acc[2][li], (double)s2);
                    }
                    __builtin_amdgcn_sched_barrier(0);   // one row of LDS adds in flight
                }
        } else {
            const Support<R, 1> &sp = sq[0];
            const int b0 = entry(sp.base[0], sp.base[1], sp.base[2]);
            for (int k = 0; k < NS; ++k)
                for (int j = 0; j < NS; ++j)
                    for (int i = 0; i < NS; ++i) {
                        const R N = sp.w[0][i] * sp.w[1][j] * sp.w[2][k];
                        const int li = b0 + i + px * j + pxy * k;
                        atomicAdd(&acc[0][li], (double)(N * mvs[ra][0]));
                        atomicAdd(&acc[1][li], (double)(N * mvs[ra][1]));
                        atomicAdd(&acc[2][li], (double)(N * mvs[ra][2]));
                    }
        }
    };
#pragma unroll
    for (int rr = 0; rr < KP; rr += 2) {
        const bool has1 = rr + 1 < KP && ok[rr + 1];
        if (anch && ok[rr] && has1 && pcl[rr] == pcl[rr + 1]) {
            remap(rr, rr + 1);
            continue;
        }
        if (ok[rr])
            remap(rr, -1);
        if (has1)
            remap(rr + 1, -1);
    }
    __syncthreads();
    GLOBAL R *NR = gp((R *)S.nr);
    const uint32_t nn = (uint32_t)S.nn;
    for (int q = threadIdx.x; q < tv; q += T) {
        int i, j, k;
        tile_node_small(t, q, i, j, k);
        const int e = entry(i, j, k);
        const double r0 = acc[0][e], r1 = acc[1][e], r2 = acc[2][e];
        if (r0 == 0.0 && r1 == 0.0 && r2 == 0.0)
            continue;
        const uint32_t I = node_id(S, i, j, k);
        addg(NR, I, (R)r0);
        addg(NR, nn + I, (R)r1);
        addg(NR, 2 * nn + I, (R)r2);
    }
    __syncthreads();
}

// MUSL, after p2g_usl: particle velocity (FLIP or PIC) from the nodal
// acceleration and updated velocity, then the updated particle momenta back
// to the nodes through the same start-of-step shape functions, summed in the
// scene's remap array.  Positions move in k_musl_stress, which evaluates
// the same shape functions again.
template <typename R, int SH, int T>
__global__ void __launch_bounds__(T) k_musl_g2p(BatchDev B)
{
    constexpr int NS = ShapeTraits<SH>::NS;
    constexpr int CAP = ShapeTraits<SH>::cap;
    // GIMP: the remap's accumulators, in the anchored layout, overlay the
    // gather tile (every particle is gathered before the remap starts)
    constexpr bool OV = SH == 1;
    constexpr int ACC_CAP = OV ? kAnchCap : CAP;
    constexpr int TILE_BYTES = 2 * CAP * (int)sizeof(R4<R>), ACC_BYTES = 3 * ACC_CAP * (int)sizeof(double);
    __shared__ __attribute__((aligned(16))) char lds[OV ? (TILE_BYTES > ACC_BYTES ? TILE_BYTES : ACC_BYTES)
                                                        : TILE_BYTES + ACC_BYTES];
    R4<R> *la = (R4<R> *)lds;
    R4<R> *lvn = la + CAP;
    double (*acc)[ACC_CAP] = (double (*)[ACC_CAP])(lds + (OV ? 0 : TILE_BYTES));
    const int64_t total = B.ioffs[B.nscenes];
    const ItemRange ir = item_range(total);
    for (int64_t g = ir.first; g < ir.end; g += ir.step) {
        const ItemRef r = item_ref(B.ioffs, B, g);
        const SceneDev S = load_scene(r.S);
        if (!scene_active(S))
            continue;
        const Item item = cld_struct(&S.items[r.it]);
        const int buf = (int)cld(&S.ctl[CTL_NBUF]);
        const Tile t = pick(S.tiles, buf)[r.it];
        if (!t.fits)
            continue;
        const int cur = (int)cld(&S.ctl[CTL_CUR]);
        const Parts<R> P = parts<R>(S, cur);
        const NodeBuf<R> nb = node_buf<R>(S, buf);
        const int tv = t.dim[0] * t.dim[1] * t.dim[2];
        load_update_tile<R>(S, nb, t, la, lvn);
        if constexpr (OV) {
            __syncthreads();
            musl_g2p_gimp_item<R, T>(S, P, item, t, la, lvn, acc);
            continue;
        } else {
        for (int q = threadIdx.x; q < tv; q += blockDim.x)
            acc[0][q] = acc[1][q] = acc[2][q] = 0.0;
        __syncthreads();
        const R dt = cst<R>(S.dt, S.f_dt);
        const int pic = S.vel_update == 1;
        uint32_t err = 0;
        for (uint32_t q = threadIdx.x; q < item.count; q += blockDim.x) {
            const uint32_t p = item.start + q;
            const double xp[3] = {ldg(P.x[0], p), ldg(P.x[1], p), ldg(P.x[2], p)};
            const R pv[3] = {ldg(P.v[0], p), ldg(P.v[1], p), ldg(P.v[2], p)};
            const R mp = ldg(P.mass, p);
            const uint32_t pc = ldg(P.cell, p);
            __builtin_amdgcn_sched_barrier(0);   // the particle's loads in one round trip
            int c[3];
            unpack_cell(pc, c);
            Support<R, SH> sp;
            make_support<R, SH>(S, xp, c, sp);
            pin_loaded(pv);
            const Corners cn = corners(S, t, sp.base);
            R dv[3] = {0, 0, 0}, vp[3] = {0, 0, 0};
            for (int k = 0; k < NS; ++k)
                for (int j = 0; j < NS; ++j)
                    for (int i = 0; i < NS; ++i) {
                        const R N = sp.w[0][i] * sp.w[1][j] * sp.w[2][k];
                        const int li = cn.t0 + i + j * cn.ty + k * cn.tz;
                        const R4<R> a = la[li];
                        const R4<R> u = lvn[li];
                        dv[0] += N * a.x;
                        dv[1] += N * a.y;
                        dv[2] += N * a.z;
                        vp[0] += N * u.x;
                        vp[1] += N * u.y;
                        vp[2] += N * u.z;
                        if constexpr (SH == 1)
                            if (i == NS - 1)
                                __builtin_amdgcn_sched_barrier(0);   // one support layer of LDS reads in flight
                    }
            pin_sums<R>(dv, vp);
            R mv[3];
            for (int a = 0; a < 3; ++a) {
                const R nva = pic ? vp[a] : pv[a] + dt * dv[a];
                stg(P.v[a], p, nva);
                mv[a] = mp * nva;
                if (!isfinite(nva))
                    err |= ERR_NONFINITE;
            }
            for (int k = 0; k < NS; ++k)
                for (int j = 0; j < NS; ++j)
                    for (int i = 0; i < NS; ++i) {
                        const R N = sp.w[0][i] * sp.w[1][j] * sp.w[2][k];
                        const int li = cn.t0 + i + j * cn.ty + k * cn.tz;
                        atomicAdd(&acc[0][li], (double)(N * mv[0]));
                        atomicAdd(&acc[1][li], (double)(N * mv[1]));
                        atomicAdd(&acc[2][li], (double)(N * mv[2]));
                    }
        }
        if (err)
            atomicOr(&S.ctl[CTL_ERR], err);
        __syncthreads();
        GLOBAL R *NR = gp((R *)S.nr);
        const uint32_t nn = (uint32_t)S.nn;
        for (int q = threadIdx.x; q < tv; q += blockDim.x) {
            const double r0 = acc[0][q], r1 = acc[1][q], r2 = acc[2][q];
            if (r0 == 0.0 && r1 == 0.0 && r2 == 0.0)
                continue;
            int i, j, k;
            tile_node_small(t, q, i, j, k);
            const uint32_t I = node_id(S, i, j, k);
            addg(NR, I, (R)r0);
            addg(NR, nn + I, (R)r1);
            addg(NR, 2 * nn + I, (R)r2);
        }
        __syncthreads();
        }
    }
}

// MUSL, after k_musl_g2p: the nodal velocity of the remapped momenta (over
// the step's nodal mass, with the velocity constraints) gives the strain
// increment, volume and stress update; the position moves by the
// interpolated updated nodal velocity of the grid update; new cell, error
// and reorder flags.  Zeroes the previous step's node buffer.
template <typename R, int SH, int T>
__global__ void __launch_bounds__(T) k_musl_stress(BatchDev B)
{
    constexpr int NS = ShapeTraits<SH>::NS;
    constexpr int CAP = ShapeTraits<SH>::cap;
    __shared__ R4<R> lvn[CAP];
    __shared__ R4<R> lvr[CAP];
    clear_previous<R>(B);
    const int64_t total = B.ioffs[B.nscenes];
    const ItemRange ir = item_range(total);
    for (int64_t g = ir.first; g < ir.end; g += ir.step) {
        const ItemRef r = item_ref(B.ioffs, B, g);
        const SceneDev S = load_scene(r.S);
        if (!scene_active(S))
            continue;
        const Item item = cld_struct(&S.items[r.it]);
        const int buf = (int)cld(&S.ctl[CTL_NBUF]);
        const Tile t = pick(S.tiles, buf)[r.it];
        if (!t.fits)
            continue;
        const int cur = (int)cld(&S.ctl[CTL_CUR]);
        const Parts<R> P = parts<R>(S, cur);
        const NodeBuf<R> nb = node_buf<R>(S, buf);
        int o[3];
        brick_origin(S, item.brick, o);
        {
            const GLOBAL R *NR = gp((const R *)S.nr);
            const uint32_t nn = (uint32_t)S.nn;
            const int tv = t.dim[0] * t.dim[1] * t.dim[2];
            for (int q = threadIdx.x; q < tv; q += blockDim.x) {
                int i, j, k;
                tile_node_small(t, q, i, j, k);
                const uint32_t I = node_id(S, i, j, k);
                R a[3], vn[3], vr[3];
                node_update<R>(S, nb, i, j, k, a, vn);
                const R pr[3] = {ldg(NR, I), ldg(NR, nn + I), ldg(NR, 2 * nn + I)};
                velocity_from_raw<R>(S, ldg(nb.m, I), pr, i, j, k, vr);
                lvn[q] = R4<R>{vn[0], vn[1], vn[2], (R)0};
                lvr[q] = R4<R>{vr[0], vr[1], vr[2], (R)0};
            }
        }
        __syncthreads();
        const R dt = cst<R>(S.dt, S.f_dt);
        uint32_t err = 0, drift = 0, lost = 0;
        for (uint32_t q = threadIdx.x; q < item.count; q += blockDim.x) {
            const uint32_t p = item.start + q;
            double xp[3] = {ldg(P.x[0], p), ldg(P.x[1], p), ldg(P.x[2], p)};
            const R vol0 = ldg(P.vol, p);
            R sg[6];
            for (int k = 0; k < 6; ++k)
                sg[k] = ldg(P.sig[k], p);
            const uint32_t pc = ldg(P.cell, p);
            __builtin_amdgcn_sched_barrier(0);   // the particle's loads in one round trip
            int c[3];
            unpack_cell(pc, c);
            Support<R, SH> sp;
            make_support<R, SH>(S, xp, c, sp);
            const Corners cn = corners(S, t, sp.base);
            R vp[3] = {0, 0, 0};
            R L[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
            for (int k = 0; k < NS; ++k)
                for (int j = 0; j < NS; ++j)
                    for (int i = 0; i < NS; ++i) {
                        const R wyz = sp.w[1][j] * sp.w[2][k];
                        const R N = sp.w[0][i] * wyz;
                        R gxN = sp.dw[0][i] * wyz;
                        R gyN = sp.w[0][i] * sp.dw[1][j] * sp.w[2][k];
                        R gzN = sp.w[0][i] * sp.w[1][j] * sp.dw[2][k];
                        to_dx<R, SH>(sp, gxN, gyN, gzN);
                        const int li = cn.t0 + i + j * cn.ty + k * cn.tz;
                        const R4<R> u = lvn[li];
                        const R4<R> w = lvr[li];
                        vp[0] += N * u.x;
                        vp[1] += N * u.y;
                        vp[2] += N * u.z;
                        L[0][0] += w.x * gxN;
                        L[0][1] += w.x * gyN;
                        L[0][2] += w.x * gzN;
                        L[1][0] += w.y * gxN;
                        L[1][1] += w.y * gyN;
                        L[1][2] += w.y * gzN;
                        L[2][0] += w.z * gxN;
                        L[2][1] += w.z * gyN;
                        L[2][2] += w.z * gzN;
                        if constexpr (SH == 1)
                            if (i == NS - 1)
                                __builtin_amdgcn_sched_barrier(0);   // one support layer of LDS reads in flight
                    }
            pin_grad<R>(L);
            for (int a = 0; a < 3; ++a) {
                xp[a] += S.dt * (double)vp[a];
                stg(P.x[a], p, xp[a]);
            }
            const R de[6] = {dt * L[0][0], dt * L[1][1], dt * L[2][2], dt * (L[0][1] + L[1][0]),
                             dt * (L[1][2] + L[2][1]), dt * (L[0][2] + L[2][0])};
            stg(P.vol, p, vol0 * ((R)1 + de[0] + de[1] + de[2]));
            constitutive<R>(S, de, sg);
            for (int k = 0; k < 6; ++k) {
                stg(P.sig[k], p, sg[k]);
                if (!isfinite(sg[k]))
                    err |= ERR_NONFINITE;
            }
            int nc[3];
            uint32_t e;
            if constexpr (SH == 2) {
                double rr[3];
                IsoCell k;
                for (int a = 0; a < 3; ++a)
                    nc[a] = c[a];
                e = iso_locate(S, xp, nc, rr, k, kIsoWalk);
            } else {
                e = locate(S, xp, nc);
            }
            if (e) {
                err |= e;
                lost += (e & ERR_OUT_OF_MESH) ? 1u : 0u;
                continue;
            }
            stg(P.cell, p, pack_cell(nc));
            drift |= in_home(nc, o) ? 0u : 1u;
        }
        if (err)
            atomicOr(&S.ctl[CTL_ERR], err);
        if (lost)
            atomicAdd(&S.ctl[CTL_LOST], lost);
        if (drift || (S.sort_always && threadIdx.x == 0)) {
            S.ctl[CTL_NEED_SORT] = 1u;
            B.flags[BF_ANY_SORT] = 1u;
        }
        __syncthreads();
    }
}

}  // namespace mpmx

// --------------------------------------------------- host launch table --

#include "mpmx_launch.h"

namespace mpmx {

template <typename R, int SH, int TI>
static void set_items(KernelSet &k)
{
    constexpr int T = kItemThreadChoices[TI];
    k.p2g[TI] = (const void *)&k_p2g<R, SH, false, T>;
    k.stress[TI] = (const void *)&k_stress<R, SH, T>;
    k.g2p_p2g[TI] = (const void *)&k_g2p_p2g<R, SH, T>;
    k.p2g_usl[TI] = (const void *)&k_p2g<R, SH, true, T>;
    k.g2p_usl[TI] = (const void *)&k_g2p_usl<R, SH, T>;
    k.p2g_musl[TI] = (const void *)&k_p2g<R, SH, true, T, true>;
    k.musl_g2p[TI] = (const void *)&k_musl_g2p<R, SH, T>;
    k.musl_stress[TI] = (const void *)&k_musl_stress<R, SH, T>;
}

template <typename R, int SH>
static KernelSet make_set()
{
    KernelSet k;
    k.load = (const void *)&k_load<R>;
    k.read_out = (const void *)&k_read_out<R>;
    k.nodes_out = (const void *)&k_nodes_out<R>;
    k.reorder = (const void *)&k_reorder<R>;
    set_items<R, SH, 0>(k);
    set_items<R, SH, 1>(k);
    set_items<R, SH, 2>(k);
    return k;
}

const KernelSet &kernel_set(int prec, int shape)
{
    static const KernelSet sets[2][3] = {{make_set<float, 0>(), make_set<float, 1>(), make_set<float, 2>()},
                                         {make_set<double, 0>(), make_set<double, 1>(), make_set<double, 2>()}};
    return sets[prec ? 1 : 0][shape < 0 || shape > 2 ? 0 : shape];
}

const CommonKernels &common_kernels()
{
    static const CommonKernels c = {(const void *)&k_begin, (const void *)&k_cell_counts};
    return c;
}

}  // namespace mpmx
