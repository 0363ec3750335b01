// mpmx_kernels.hip -- gfx950 kernels of the explicit MPM step.
//
// One explicit update-stress-first step (code overview: USF; introduction:
// nodal values reset every step, particle-to-node mapping and interpolation
// back with the same mapping functions):
//   clear    zero the nodal mass, momentum and force the last step touched
//   sort     (only when needed) counting sort of particles by brick-major
//            cell key; rebuild the work list of <= 512-particle chunks of
//            one 4x4x4-cell brick
//   p2g      nodal mass (FP64) and momentum, accumulated in an LDS node tile
//            per work item and flushed with one global atomic per touched
//            node and component
//   stress   nodal velocity (with constraints) into LDS, velocity gradient,
//            strain increment, volume, elastic / Drucker-Prager stress,
//            internal + external nodal force through an LDS tile
//   g2p      nodal acceleration and updated velocity (with constraints) into
//            LDS, FLIP/PIC particle velocity, FP64 position, new cell key,
//            drift / error checks
// USL replaces p2g+stress+g2p with p2g_usl (mass, momentum and force from the
// old stress) and g2p_usl (particle update, then stress from the updated
// nodal velocity).
//
// Every per-item kernel is persistent: a fixed grid strides over the
// flattened (scene, item) list whose offsets live in device memory, so a
// launch needs no host knowledge of how many items each scene has.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mpmx_dev.h"

namespace mpmx {

// ------------------------------------------------------------ helpers ----

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

__device__ inline int wave_min(int v)
{
    for (int o = 32; o > 0; o >>= 1)
        v = min(v, __shfl_xor(v, o));
    return v;
}

__device__ inline int wave_max(int v)
{
    for (int o = 32; o > 0; o >>= 1)
        v = max(v, __shfl_xor(v, o));
    return v;
}

__device__ inline uint32_t wave_sum(uint32_t v)
{
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o);
    return v;
}

__device__ inline void key_to_cell(const SceneDev &S, uint32_t key, int c[3])
{
    uint32_t b = key >> 6, l = key & 63u;
    uint32_t bx = b % (uint32_t)S.nb[0];
    uint32_t t = b / (uint32_t)S.nb[0];
    uint32_t by = t % (uint32_t)S.nb[1];
    uint32_t bz = t / (uint32_t)S.nb[1];
    c[0] = (int)(bx * 4 + (l & 3u));
    c[1] = (int)(by * 4 + ((l >> 2) & 3u));
    c[2] = (int)(bz * 4 + (l >> 4));
}

__device__ inline uint32_t cell_to_key(const SceneDev &S, const int c[3])
{
    uint32_t b = (uint32_t)(c[0] >> 2) +
                 (uint32_t)S.nb[0] * ((uint32_t)(c[1] >> 2) + (uint32_t)S.nb[1] * (uint32_t)(c[2] >> 2));
    return b * 64u + (uint32_t)((c[0] & 3) + 4 * ((c[1] & 3) + 4 * (c[2] & 3)));
}

// Cell of a position: floor((x - o) / h) in IEEE FP64 per axis.  Returns 0,
// ERR_OUT_OF_MESH or ERR_NONFINITE.
__device__ inline uint32_t locate(const SceneDev &S, const double x[3], int c[3])
{
    for (int a = 0; a < 3; ++a) {
        if (!isfinite(x[a]))
            return ERR_NONFINITE;
        double t = floor((x[a] - S.origin[a]) / S.h);
        if (!(t >= 0.0 && t < (double)S.n[a]))
            return ERR_OUT_OF_MESH;
        c[a] = (int)t;
    }
    return 0;
}

__device__ inline int64_t node_id(const SceneDev &S, int i, int j, int k)
{
    const int g = S.ghost;
    return (int64_t)(i + g) + (int64_t)S.N[0] * ((int64_t)(j + g) + (int64_t)S.N[1] * (int64_t)(k + g));
}

// Components fixed by the face rules at node (i,j,k): bit a = component a.
__device__ inline uint32_t face_mask(const SceneDev &S, int i, int j, int k)
{
    const int idx[3] = {i, j, k};
    uint32_t m = 0;
    for (int b = 0; b < 3; ++b) {
        uint32_t lo = idx[b] <= 0 ? (S.face_bits >> (4 * b)) & 3u : 0u;
        uint32_t hi = idx[b] >= S.n[b] ? (S.face_bits >> (4 * b + 2)) & 3u : 0u;
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

// Nodal velocity v = p / m (0 on void nodes) with velocity constraints.
template <typename R>
__device__ inline void node_velocity(const SceneDev &S, int i, int j, int k, R v[3])
{
    const int64_t I = node_id(S, i, j, k);
    const double m = S.nm[I];
    const R *P = (const R *)S.np_;
    for (int a = 0; a < 3; ++a)
        v[a] = m > S.eps_m ? (R)((double)P[a * S.nn + I] / m) : (R)0;
    uint32_t fm = face_mask(S, i, j, k);
    for (int a = 0; a < 3; ++a)
        if (fm & (1u << a))
            v[a] = (R)0;
    if (S.bc_mask) {
        uint32_t em = S.bc_mask[I];
        for (int a = 0; a < 3; ++a)
            if (em & (1u << a))
                v[a] = (R)S.bc_val[3 * I + a];
    }
}

// Nodal acceleration a = f / m and updated velocity vn = v + dt a, with the
// constraints applied to v (prescribed), a (zero) and vn (prescribed).
template <typename R>
__device__ inline void node_update(const SceneDev &S, int i, int j, int k, R a[3], R vn[3])
{
    const int64_t I = node_id(S, i, j, k);
    const double m = S.nm[I];
    const R *P = (const R *)S.np_;
    const R *F = (const R *)S.nf;
    R v[3];
    for (int c = 0; c < 3; ++c) {
        v[c] = m > S.eps_m ? (R)((double)P[c * S.nn + I] / m) : (R)0;
        a[c] = m > S.eps_m ? (R)((double)F[c * S.nn + I] / m) : (R)0;
    }
    uint32_t fm = face_mask(S, i, j, k);
    uint32_t em = S.bc_mask ? (uint32_t)S.bc_mask[I] : 0u;
    for (int c = 0; c < 3; ++c) {
        if (fm & (1u << c)) {
            v[c] = (R)0;
            a[c] = (R)0;
        }
        if (em & (1u << c)) {
            v[c] = (R)S.bc_val[3 * I + c];
            a[c] = (R)0;
        }
    }
    const R dt = (R)S.dt;
    for (int c = 0; c < 3; ++c)
        vn[c] = v[c] + dt * a[c];
    for (int c = 0; c < 3; ++c) {
        if (fm & (1u << c))
            vn[c] = (R)0;
        if (em & (1u << c))
            vn[c] = (R)S.bc_val[3 * I + c];
    }
}

// ------------------------------------------------------ shape functions --

template <int SH>
struct ShapeTraits;
template <>
struct ShapeTraits<0> {   // trilinear 8-node hexahedron
    static constexpr int NS = 2;
    static constexpr int lo = 0;   // node tile extends cells [lo, hi] by
    static constexpr int hi = 1;   // -lo .. +hi nodes
};
template <>
struct ShapeTraits<1> {   // uGIMP, particle half-length h/4, 27 nodes
    static constexpr int NS = 3;
    static constexpr int lo = 1;
    static constexpr int hi = 2;
};

template <typename R, int SH>
struct Support {
    int base[3];
    R w[3][ShapeTraits<SH>::NS];
    R dw[3][ShapeTraits<SH>::NS];
};

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
    const double h = S.h;
    const R inv_h = (R)(1.0 / h);
    if constexpr (SH == 0) {
        for (int a = 0; a < 3; ++a) {
            const R r = (R)((x[a] - (S.origin[a] + h * (double)c[a])) / h);
            sp.base[a] = c[a];
            sp.w[a][0] = (R)1 - r;
            sp.w[a][1] = r;
            sp.dw[a][0] = -inv_h;
            sp.dw[a][1] = inv_h;
        }
    } else {
        const double l = 0.25 * h;
        for (int a = 0; a < 3; ++a) {
            const int i0 = (int)floor((x[a] - S.origin[a] - l) / h);
            sp.base[a] = i0;
            for (int t = 0; t < 3; ++t) {
                const R rho = (R)((x[a] - (S.origin[a] + h * (double)(i0 + t))) / h);
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
    const R lam = (R)S.lam, G = (R)S.G;
    const R tr = de[0] + de[1] + de[2];
    for (int a = 0; a < 3; ++a)
        sig[a] += lam * tr + (R)2 * G * de[a];
    for (int a = 3; a < 6; ++a)
        sig[a] += G * de[a];
    if (S.model != 1)
        return;
    // Drucker-Prager, perfectly plastic: f = sqrt(J2) + eta p - xi c.
    const R K = (R)S.K, eta = (R)S.eta, etab = (R)S.etab;
    const R p = (sig[0] + sig[1] + sig[2]) / (R)3;
    R s[6];
    for (int a = 0; a < 3; ++a)
        s[a] = sig[a] - p;
    for (int a = 3; a < 6; ++a)
        s[a] = sig[a];
    const R J2 = (R)0.5 * (s[0] * s[0] + s[1] * s[1] + s[2] * s[2]) + s[3] * s[3] + s[4] * s[4] + s[5] * s[5];
    const R q = sqrt(J2);
    const R f = q + eta * p - (R)S.xic;
    if (!(f > (R)0))
        return;
    const R dgam = f / (G + K * eta * etab);
    if (q - G * dgam >= (R)0) {
        const R scale = (R)1 - G * dgam / q;
        const R pn = p - K * etab * dgam;
        for (int a = 0; a < 3; ++a)
            sig[a] = scale * s[a] + pn;
        for (int a = 3; a < 6; ++a)
            sig[a] = scale * s[a];
    } else {
        const R pa = S.has_apex ? (R)S.apex_p : p;
        for (int a = 0; a < 3; ++a)
            sig[a] = pa;
        for (int a = 3; a < 6; ++a)
            sig[a] = (R)0;
    }
}

// -------------------------------------------------------- scene lookup --

struct ItemRef {
    const SceneDev *S;
    int it;
};

__device__ inline ItemRef item_ref(const BatchDev &B, int64_t g)
{
    const int s = find_scene(B.ioffs, B.nscenes, g);
    return {B.scenes[s], (int)(g - (int64_t)B.ioffs[s])};
}

// A scene takes part in the coming step: not stopped by an error and with
// steps left.  Read by the clear and sort kernels, during which neither
// word changes.
__device__ inline bool scene_pending(const SceneDev &S)
{
    return S.ctl[CTL_ERR] == 0u && S.ctl[CTL_REMAIN] > 0u;
}

// The stage kernels after step_control test CTL_ACTIVE only: it is fixed for
// the whole step, whereas CTL_ERR may be raised by another workgroup of the
// same kernel, and every thread of a workgroup must take the same branch
// around its barriers.
__device__ inline bool scene_active(const SceneDev &S)
{
    return S.ctl[CTL_ACTIVE] != 0u;
}

// ----------------------------------------------------- load / read out --

// Inputs are row-major doubles (n x 3, n x 6, n); fills buffer 0, sets the
// identity permutation and each particle's key.
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
        uint32_t e = locate(S, xp, c);
        if (!fin)
            e |= ERR_NONFINITE;
        if (e) {
            atomicOr(&S.ctl[CTL_ERR], e);
            c[0] = c[1] = c[2] = 0;
        }
        S.key[0][p] = cell_to_key(S, c);
        S.pid[0][p] = (uint32_t)p;
    }
}

// Particle state in original order (row-major doubles); any pointer may be null.
template <typename R>
__global__ void k_read_out(const SceneDev *Sd, double *x, double *v, double *sig, double *vol, int32_t *cell)
{
    const SceneDev &S = *Sd;
    const int64_t n = S.np;
    const int cur = (int)S.ctl[CTL_CUR];
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
            key_to_cell(S, S.key[cur][p], c);
            cell[o] = c[0] + S.n[0] * (c[1] + S.n[1] * c[2]);
        }
    }
}

__global__ void k_cell_counts(const SceneDev *Sd, uint32_t *counts)
{
    const SceneDev &S = *Sd;
    const int cur = (int)S.ctl[CTL_CUR];
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < S.np; p += (int64_t)gridDim.x * blockDim.x) {
        int c[3];
        key_to_cell(S, S.key[cur][p], c);
        atomicAdd(&counts[c[0] + (int64_t)S.n[0] * (c[1] + (int64_t)S.n[1] * c[2])], 1u);
    }
}

template <typename R>
__global__ void k_nodes_out(const SceneDev *Sd, double *m, double *p, double *f)
{
    const SceneDev &S = *Sd;
    const R *P = (const R *)S.np_;
    const R *F = (const R *)S.nf;
    for (int64_t I = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; I < S.nn; I += (int64_t)gridDim.x * blockDim.x) {
        if (m)
            m[I] = S.nm[I];
        for (int a = 0; a < 3; ++a) {
            if (p)
                p[3 * I + a] = (double)P[a * S.nn + I];
            if (f)
                f[3 * I + a] = (double)F[a * S.nn + I];
        }
    }
}

// ------------------------------------------------------- step control --

// Item offsets of the batch; mode 0: every scene with steps left counts with
// all its items (start of a call, used by the first clear); mode 1: end of
// the sort stage of a step: apply a pending reorder, decide which scenes
// take part in this step, decrement their remaining steps, offsets over the
// active scenes only.
__global__ void k_step_control(BatchDev B, int mode)
{
    __shared__ uint32_t part[1024];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) {
        carry = 0;
        B.ioffs[0] = 0;
    }
    __syncthreads();
    for (int base = 0; base < B.nscenes; base += blockDim.x) {
        const int s = base + threadIdx.x;
        uint32_t items = 0;
        if (s < B.nscenes) {
            const SceneDev &S = *B.scenes[s];
            uint32_t *ctl = S.ctl;
            if (mode == 0) {
                items = ctl[CTL_N_ITEMS];
            } else {
                const bool go = ctl[CTL_ERR] == 0u && ctl[CTL_REMAIN] > 0u;
                if (go && ctl[CTL_NEED_SORT]) {
                    ctl[CTL_CUR] ^= 1u;
                    ctl[CTL_NEED_SORT] = 0u;
                    ctl[CTL_N_SORTS] += 1u;
                }
                ctl[CTL_ACTIVE] = go ? 1u : 0u;
                if (go) {
                    ctl[CTL_REMAIN] -= 1u;
                    ctl[CTL_STEPS] += 1u;
                }
                items = go ? ctl[CTL_N_ITEMS] : 0u;
            }
        }
        part[threadIdx.x] = items;
        __syncthreads();
        // inclusive scan (Hillis-Steele) of this chunk
        for (int o = 1; o < (int)blockDim.x; o <<= 1) {
            uint32_t t = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0u;
            __syncthreads();
            part[threadIdx.x] += t;
            __syncthreads();
        }
        if (s < B.nscenes)
            B.ioffs[s + 1] = carry + part[threadIdx.x];
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1)
            carry += part[threadIdx.x];
        __syncthreads();
    }
}

// Steps left per scene for this call (written before the first step).
__global__ void k_set_remaining(BatchDev B, const int64_t *nsteps)
{
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < B.nscenes; s += gridDim.x * blockDim.x) {
        int64_t k = nsteps[s];
        B.scenes[s]->ctl[CTL_REMAIN] = (uint32_t)(k < 0 ? 0 : (k > 0x7fffffff ? 0x7fffffff : k));
    }
}

// ---------------------------------------------------------------- clear --

// Zero m, p, f over the node tiles of the previous step's items.
template <typename R>
__global__ void __launch_bounds__(kBlock) k_clear(BatchDev B)
{
    const int64_t total = B.ioffs[B.nscenes];
    for (int64_t g = blockIdx.x; g < total; g += gridDim.x) {
        const ItemRef r = item_ref(B, g);
        const SceneDev &S = *r.S;
        if (!scene_pending(S))
            continue;
        const Tile t = S.tiles[r.it];
        const int vol = t.dim[0] * t.dim[1] * t.dim[2];
        R *P = (R *)S.np_;
        R *F = (R *)S.nf;
        for (int q = threadIdx.x; q < vol; q += blockDim.x) {
            const int i = t.lo[0] + q % t.dim[0];
            const int j = t.lo[1] + (q / t.dim[0]) % t.dim[1];
            const int k = t.lo[2] + q / (t.dim[0] * t.dim[1]);
            const int64_t I = node_id(S, i, j, k);
            S.nm[I] = 0.0;
            for (int a = 0; a < 3; ++a) {
                P[a * S.nn + I] = (R)0;
                F[a * S.nn + I] = (R)0;
            }
        }
    }
}

// ----------------------------------------------------------------- sort --

// rank[p] = arrival order of p among the particles of its key.
__global__ void k_sort_count(BatchDev B)
{
    for (int64_t gp = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; gp < B.total_particles;
         gp += (int64_t)gridDim.x * blockDim.x) {
        const int s = find_scene(B.poffs, B.nscenes, gp);
        const SceneDev &S = *B.scenes[s];
        if (!scene_pending(S) || !S.ctl[CTL_NEED_SORT])
            continue;
        const int64_t p = gp - B.poffs[s];
        const int cur = (int)S.ctl[CTL_CUR];
        S.rank[p] = atomicAdd(&S.cnt[S.key[cur][p]], 1u);
    }
}

// One wavefront per brick: particles and work items of the brick.
__global__ void k_sort_bricks(BatchDev B)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t gb = wave; gb < B.total_bricks; gb += nwaves) {
        const int s = find_scene(B.boffs, B.nscenes, gb);
        const SceneDev &S = *B.scenes[s];
        if (!scene_pending(S) || !S.ctl[CTL_NEED_SORT])
            continue;
        const int64_t b = gb - B.boffs[s];
        const uint32_t c = S.cnt[b * 64 + lane];
        const uint32_t tot = wave_sum(c);
        if (lane == 0) {
            S.bcnt[b] = tot;
            S.bitem[b] = (tot + kChunk - 1) / kChunk;
        }
    }
}

// One workgroup per scene: exclusive scans of particles and items per brick.
__global__ void __launch_bounds__(1024) k_sort_scan(BatchDev B)
{
    __shared__ uint32_t sp[1024], si[1024];
    for (int s = blockIdx.x; s < B.nscenes; s += gridDim.x) {
        const SceneDev &S = *B.scenes[s];
        if (!scene_pending(S) || !S.ctl[CTL_NEED_SORT])
            continue;
        const int64_t nb = S.nbricks;
        const int64_t per = (nb + blockDim.x - 1) / blockDim.x;
        const int64_t b0 = threadIdx.x * per;
        const int64_t b1 = min(b0 + per, nb);
        uint32_t tp = 0, ti = 0;
        for (int64_t b = b0; b < b1; ++b) {
            tp += S.bcnt[b];
            ti += S.bitem[b];
        }
        sp[threadIdx.x] = tp;
        si[threadIdx.x] = ti;
        __syncthreads();
        for (int o = 1; o < (int)blockDim.x; o <<= 1) {
            uint32_t a = threadIdx.x >= (unsigned)o ? sp[threadIdx.x - o] : 0u;
            uint32_t c = threadIdx.x >= (unsigned)o ? si[threadIdx.x - o] : 0u;
            __syncthreads();
            sp[threadIdx.x] += a;
            si[threadIdx.x] += c;
            __syncthreads();
        }
        uint32_t rp = sp[threadIdx.x] - tp, ri = si[threadIdx.x] - ti;   // exclusive
        for (int64_t b = b0; b < b1; ++b) {
            S.bstart[b] = rp;
            S.istart[b] = ri;
            rp += S.bcnt[b];
            ri += S.bitem[b];
        }
        if (threadIdx.x == blockDim.x - 1) {
            S.bstart[nb] = sp[threadIdx.x];
            S.istart[nb] = si[threadIdx.x];
            S.ctl[CTL_N_ITEMS] = si[threadIdx.x];
        }
        __syncthreads();
    }
}

// One wavefront per brick: start of each cell's run, the brick's work items;
// resets the counts for the next sort.
__global__ void k_sort_cells(BatchDev B)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t gb = wave; gb < B.total_bricks; gb += nwaves) {
        const int s = find_scene(B.boffs, B.nscenes, gb);
        const SceneDev &S = *B.scenes[s];
        if (!scene_pending(S) || !S.ctl[CTL_NEED_SORT])
            continue;
        const int64_t b = gb - B.boffs[s];
        const uint32_t c = S.cnt[b * 64 + lane];
        uint32_t inc = c;
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t t = __shfl_up(inc, o);
            if (lane >= o)
                inc += t;
        }
        const uint32_t bs = S.bstart[b];
        S.cstart[b * 64 + lane] = bs + inc - c;
        S.cnt[b * 64 + lane] = 0u;
        const uint32_t nit = S.bitem[b], tot = S.bcnt[b], i0 = S.istart[b];
        for (uint32_t i = lane; i < nit; i += 64) {
            Item it;
            it.start = bs + i * kChunk;
            it.count = min((uint32_t)kChunk, tot - i * kChunk);
            it.brick = (uint32_t)b;
            it.pad = 0;
            S.items[i0 + i] = it;
        }
    }
}

// Move every particle to its sorted slot in the other buffer.
template <typename R>
__global__ void k_sort_scatter(BatchDev B)
{
    for (int64_t gp = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; gp < B.total_particles;
         gp += (int64_t)gridDim.x * blockDim.x) {
        const int s = find_scene(B.poffs, B.nscenes, gp);
        const SceneDev &S = *B.scenes[s];
        if (!scene_pending(S) || !S.ctl[CTL_NEED_SORT])
            continue;
        const int64_t n = S.np;
        const int64_t p = gp - B.poffs[s];
        const int cur = (int)S.ctl[CTL_CUR], nxt = cur ^ 1;
        const uint32_t key = S.key[cur][p];
        const int64_t d = (int64_t)S.cstart[key] + S.rank[p];
        for (int a = 0; a < 3; ++a) {
            S.x[nxt][a * n + d] = S.x[cur][a * n + p];
            ((R *)S.v[nxt])[a * n + d] = ((const R *)S.v[cur])[a * n + p];
        }
        for (int k = 0; k < 6; ++k)
            ((R *)S.sig[nxt])[k * n + d] = ((const R *)S.sig[cur])[k * n + p];
        ((R *)S.vol[nxt])[d] = ((const R *)S.vol[cur])[p];
        ((R *)S.mass[nxt])[d] = ((const R *)S.mass[cur])[p];
        S.key[nxt][d] = key;
        S.pid[nxt][d] = S.pid[cur][p];
    }
}

// ---------------------------------------------------- per-item helpers --

// Node box of the item's particles (cell bbox extended by the support).
template <int SH>
__device__ inline Tile item_tile(const SceneDev &S, const Item &item, const uint32_t *key, int *red)
{
    int mn[3] = {1 << 30, 1 << 30, 1 << 30}, mx[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
    for (uint32_t q = threadIdx.x; q < item.count; q += blockDim.x) {
        int c[3];
        key_to_cell(S, key[item.start + q], c);
        for (int a = 0; a < 3; ++a) {
            mn[a] = min(mn[a], c[a]);
            mx[a] = max(mx[a], c[a]);
        }
    }
    for (int a = 0; a < 3; ++a) {
        mn[a] = wave_min(mn[a]);
        mx[a] = wave_max(mx[a]);
    }
    if (threadIdx.x == 0)
        for (int a = 0; a < 3; ++a) {
            red[a] = 1 << 30;
            red[3 + a] = -(1 << 30);
        }
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        for (int a = 0; a < 3; ++a) {
            atomicMin(&red[a], mn[a]);
            atomicMax(&red[3 + a], mx[a]);
        }
    __syncthreads();
    Tile t;
    for (int a = 0; a < 3; ++a) {
        t.lo[a] = red[a] - ShapeTraits<SH>::lo;
        t.dim[a] = red[3 + a] + ShapeTraits<SH>::hi - t.lo[a] + 1;
    }
    t.fits = (t.dim[0] * t.dim[1] * t.dim[2] <= kMaxTileNodes) ? 1 : 0;
    t.pad = 0;
    __syncthreads();
    return t;
}

template <int SH>
__device__ inline int tile_index(const Tile &t, const int base[3], int i, int j, int k)
{
    return (base[0] + i - t.lo[0]) + t.dim[0] * ((base[1] + j - t.lo[1]) + t.dim[1] * (base[2] + k - t.lo[2]));
}

// ------------------------------------------------------------------ p2g --

// Nodal mass and momentum (USF); with WITH_FORCE also the nodal force from
// the current stress and volume (USL).
template <typename R, int SH, bool WITH_FORCE>
__global__ void __launch_bounds__(kBlock) k_p2g(BatchDev B)
{
    constexpr int NS = ShapeTraits<SH>::NS;
    __shared__ double lm[kMaxTileNodes];
    __shared__ R lp[3][kMaxTileNodes];
    __shared__ R lf[WITH_FORCE ? 3 : 1][WITH_FORCE ? kMaxTileNodes : 1];
    __shared__ int red[6];
    const int64_t total = B.ioffs[B.nscenes];
    for (int64_t g = blockIdx.x; g < total; g += gridDim.x) {
        const ItemRef r = item_ref(B, g);
        const SceneDev &S = *r.S;
        if (!scene_active(S))
            continue;
        const Item item = S.items[r.it];
        const int cur = (int)S.ctl[CTL_CUR];
        const int64_t n = S.np;
        const Tile t = item_tile<SH>(S, item, S.key[cur], red);
        if (threadIdx.x == 0)
            S.tiles[r.it] = t;
        if (!t.fits) {
            if (threadIdx.x == 0)
                atomicOr(&S.ctl[CTL_ERR], ERR_TILE);
            continue;
        }
        const int tv = t.dim[0] * t.dim[1] * t.dim[2];
        for (int q = threadIdx.x; q < tv; q += blockDim.x) {
            lm[q] = 0.0;
            for (int a = 0; a < 3; ++a) {
                lp[a][q] = (R)0;
                if constexpr (WITH_FORCE)
                    lf[a][q] = (R)0;
            }
        }
        __syncthreads();
        const double *X = S.x[cur];
        const R *V = (const R *)S.v[cur];
        const R *M = (const R *)S.mass[cur];
        const R *SG = (const R *)S.sig[cur];
        const R *VO = (const R *)S.vol[cur];
        const R gx = (R)S.g[0], gy = (R)S.g[1], gz = (R)S.g[2];
        for (uint32_t q = threadIdx.x; q < item.count; q += blockDim.x) {
            const int64_t p = item.start + q;
            const double xp[3] = {X[p], X[n + p], X[2 * n + p]};
            int c[3];
            key_to_cell(S, S.key[cur][p], c);
            Support<R, SH> sp;
            make_support<R, SH>(S, xp, c, sp);
            const R mp = M[p];
            const R mv[3] = {mp * V[p], mp * V[n + p], mp * V[2 * n + p]};
            R sg[6], vol = (R)0;
            if constexpr (WITH_FORCE) {
                for (int k = 0; k < 6; ++k)
                    sg[k] = SG[k * n + p];
                vol = VO[p];
            }
            for (int k = 0; k < NS; ++k)
                for (int j = 0; j < NS; ++j)
                    for (int i = 0; i < NS; ++i) {
                        const R wyz = sp.w[1][j] * sp.w[2][k];
                        const R N = sp.w[0][i] * wyz;
                        const int li = tile_index<SH>(t, sp.base, i, j, k);
                        atomicAdd(&lm[li], (double)(N * mp));
                        atomicAdd(&lp[0][li], N * mv[0]);
                        atomicAdd(&lp[1][li], N * mv[1]);
                        atomicAdd(&lp[2][li], N * mv[2]);
                        if constexpr (WITH_FORCE) {
                            const R gxN = sp.dw[0][i] * wyz;
                            const R gyN = sp.w[0][i] * sp.dw[1][j] * sp.w[2][k];
                            const R gzN = sp.w[0][i] * sp.w[1][j] * sp.dw[2][k];
                            const R fx = -vol * (sg[0] * gxN + sg[3] * gyN + sg[5] * gzN) + N * mp * gx;
                            const R fy = -vol * (sg[3] * gxN + sg[1] * gyN + sg[4] * gzN) + N * mp * gy;
                            const R fz = -vol * (sg[5] * gxN + sg[4] * gyN + sg[2] * gzN) + N * mp * gz;
                            atomicAdd(&lf[0][li], fx);
                            atomicAdd(&lf[1][li], fy);
                            atomicAdd(&lf[2][li], fz);
                        }
                    }
        }
        __syncthreads();
        R *P = (R *)S.np_;
        R *F = (R *)S.nf;
        for (int q = threadIdx.x; q < tv; q += blockDim.x) {
            const double m = lm[q];
            if (m == 0.0)
                continue;
            const int i = t.lo[0] + q % t.dim[0];
            const int j = t.lo[1] + (q / t.dim[0]) % t.dim[1];
            const int k = t.lo[2] + q / (t.dim[0] * t.dim[1]);
            const int64_t I = node_id(S, i, j, k);
            atomicAdd(&S.nm[I], m);
            for (int a = 0; a < 3; ++a)
                atomicAdd(&P[a * S.nn + I], lp[a][q]);
            if constexpr (WITH_FORCE)
                for (int a = 0; a < 3; ++a)
                    atomicAdd(&F[a * S.nn + I], lf[a][q]);
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------- stress --

// USF: nodal velocity, strain increment, volume and stress update, nodal
// internal + external force.
template <typename R, int SH>
__global__ void __launch_bounds__(kBlock) k_stress(BatchDev B)
{
    constexpr int NS = ShapeTraits<SH>::NS;
    __shared__ R4<R> lv[kMaxTileNodes];
    __shared__ R lf[3][kMaxTileNodes];
    const int64_t total = B.ioffs[B.nscenes];
    for (int64_t g = blockIdx.x; g < total; g += gridDim.x) {
        const ItemRef r = item_ref(B, g);
        const SceneDev &S = *r.S;
        if (!scene_active(S))
            continue;
        const Item item = S.items[r.it];
        const Tile t = S.tiles[r.it];
        if (!t.fits)
            continue;
        const int cur = (int)S.ctl[CTL_CUR];
        const int64_t n = S.np;
        const int tv = t.dim[0] * t.dim[1] * t.dim[2];
        for (int q = threadIdx.x; q < tv; q += blockDim.x) {
            const int i = t.lo[0] + q % t.dim[0];
            const int j = t.lo[1] + (q / t.dim[0]) % t.dim[1];
            const int k = t.lo[2] + q / (t.dim[0] * t.dim[1]);
            R v[3];
            node_velocity<R>(S, i, j, k, v);
            lv[q] = R4<R>{v[0], v[1], v[2], (R)0};
            lf[0][q] = lf[1][q] = lf[2][q] = (R)0;
        }
        __syncthreads();
        const double *X = S.x[cur];
        const R *M = (const R *)S.mass[cur];
        R *SG = (R *)S.sig[cur];
        R *VO = (R *)S.vol[cur];
        const R dt = (R)S.dt;
        const R gx = (R)S.g[0], gy = (R)S.g[1], gz = (R)S.g[2];
        uint32_t bad = 0;
        for (uint32_t q = threadIdx.x; q < item.count; q += blockDim.x) {
            const int64_t p = item.start + q;
            const double xp[3] = {X[p], X[n + p], X[2 * n + p]};
            int c[3];
            key_to_cell(S, S.key[cur][p], c);
            Support<R, SH> sp;
            make_support<R, SH>(S, xp, c, sp);
            R L[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
            for (int k = 0; k < NS; ++k)
                for (int j = 0; j < NS; ++j)
                    for (int i = 0; i < NS; ++i) {
                        const R gxN = sp.dw[0][i] * sp.w[1][j] * sp.w[2][k];
                        const R gyN = sp.w[0][i] * sp.dw[1][j] * sp.w[2][k];
                        const R gzN = sp.w[0][i] * sp.w[1][j] * sp.dw[2][k];
                        const R4<R> v = lv[tile_index<SH>(t, sp.base, i, j, k)];
                        L[0][0] += v.x * gxN;
                        L[0][1] += v.x * gyN;
                        L[0][2] += v.x * gzN;
                        L[1][0] += v.y * gxN;
                        L[1][1] += v.y * gyN;
                        L[1][2] += v.y * gzN;
                        L[2][0] += v.z * gxN;
                        L[2][1] += v.z * gyN;
                        L[2][2] += v.z * gzN;
                    }
            const R de[6] = {dt * L[0][0], dt * L[1][1], dt * L[2][2], dt * (L[0][1] + L[1][0]),
                             dt * (L[1][2] + L[2][1]), dt * (L[0][2] + L[2][0])};
            R vol = VO[p] * ((R)1 + de[0] + de[1] + de[2]);
            R sg[6];
            for (int k = 0; k < 6; ++k)
                sg[k] = SG[k * n + p];
            constitutive<R>(S, de, sg);
            for (int k = 0; k < 6; ++k) {
                SG[k * n + p] = sg[k];
                if (!isfinite(sg[k]))
                    bad = ERR_NONFINITE;
            }
            VO[p] = vol;
            const R mp = M[p];
            for (int k = 0; k < NS; ++k)
                for (int j = 0; j < NS; ++j)
                    for (int i = 0; i < NS; ++i) {
                        const R wyz = sp.w[1][j] * sp.w[2][k];
                        const R N = sp.w[0][i] * wyz;
                        const R gxN = sp.dw[0][i] * wyz;
                        const R gyN = sp.w[0][i] * sp.dw[1][j] * sp.w[2][k];
                        const R gzN = sp.w[0][i] * sp.w[1][j] * sp.dw[2][k];
                        const int li = tile_index<SH>(t, sp.base, i, j, k);
                        atomicAdd(&lf[0][li], -vol * (sg[0] * gxN + sg[3] * gyN + sg[5] * gzN) + N * mp * gx);
                        atomicAdd(&lf[1][li], -vol * (sg[3] * gxN + sg[1] * gyN + sg[4] * gzN) + N * mp * gy);
                        atomicAdd(&lf[2][li], -vol * (sg[5] * gxN + sg[4] * gyN + sg[2] * gzN) + N * mp * gz);
                    }
        }
        if (bad)
            atomicOr(&S.ctl[CTL_ERR], bad);
        __syncthreads();
        R *F = (R *)S.nf;
        for (int q = threadIdx.x; q < tv; q += blockDim.x) {
            const R f0 = lf[0][q], f1 = lf[1][q], f2 = lf[2][q];
            if (f0 == (R)0 && f1 == (R)0 && f2 == (R)0)
                continue;
            const int i = t.lo[0] + q % t.dim[0];
            const int j = t.lo[1] + (q / t.dim[0]) % t.dim[1];
            const int k = t.lo[2] + q / (t.dim[0] * t.dim[1]);
            const int64_t I = node_id(S, i, j, k);
            atomicAdd(&F[I], f0);
            atomicAdd(&F[S.nn + I], f1);
            atomicAdd(&F[2 * S.nn + I], f2);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ g2p --

// Particle velocity and position from the nodal acceleration and updated
// velocity; new cell key; reorder and error flags.  WITH_STRESS (USL): then
// the strain increment from the updated nodal velocity and the stress update.
template <typename R, int SH, bool WITH_STRESS>
__global__ void __launch_bounds__(kBlock) k_g2p(BatchDev B)
{
    constexpr int NS = ShapeTraits<SH>::NS;
    __shared__ R4<R> la[kMaxTileNodes];
    __shared__ R4<R> lvn[kMaxTileNodes];
    const int64_t total = B.ioffs[B.nscenes];
    for (int64_t g = blockIdx.x; g < total; g += gridDim.x) {
        const ItemRef r = item_ref(B, g);
        const SceneDev &S = *r.S;
        if (!scene_active(S))
            continue;
        const Item item = S.items[r.it];
        const Tile t = S.tiles[r.it];
        if (!t.fits)
            continue;
        const int cur = (int)S.ctl[CTL_CUR];
        const int64_t n = S.np;
        const int tv = t.dim[0] * t.dim[1] * t.dim[2];
        for (int q = threadIdx.x; q < tv; q += blockDim.x) {
            const int i = t.lo[0] + q % t.dim[0];
            const int j = t.lo[1] + (q / t.dim[0]) % t.dim[1];
            const int k = t.lo[2] + q / (t.dim[0] * t.dim[1]);
            R a[3], vn[3];
            node_update<R>(S, i, j, k, a, vn);
            la[q] = R4<R>{a[0], a[1], a[2], (R)0};
            lvn[q] = R4<R>{vn[0], vn[1], vn[2], (R)0};
        }
        __syncthreads();
        double *X = S.x[cur];
        R *V = (R *)S.v[cur];
        R *SG = (R *)S.sig[cur];
        R *VO = (R *)S.vol[cur];
        uint32_t *KEY = S.key[cur];
        const R dt = (R)S.dt;
        const int pic = S.vel_update == 1;
        // home region: the item's brick widened by one cell
        const uint32_t bb = item.brick;
        const int hb[3] = {(int)(bb % (uint32_t)S.nb[0]) * 4, (int)((bb / (uint32_t)S.nb[0]) % (uint32_t)S.nb[1]) * 4,
                           (int)(bb / ((uint32_t)S.nb[0] * (uint32_t)S.nb[1])) * 4};
        uint32_t err = 0, drift = 0;
        for (uint32_t q = threadIdx.x; q < item.count; q += blockDim.x) {
            const int64_t p = item.start + q;
            double xp[3] = {X[p], X[n + p], X[2 * n + p]};
            int c[3];
            key_to_cell(S, KEY[p], c);
            Support<R, SH> sp;
            make_support<R, SH>(S, xp, c, sp);
            R dv[3] = {0, 0, 0}, vp[3] = {0, 0, 0};
            R L[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
            for (int k = 0; k < NS; ++k)
                for (int j = 0; j < NS; ++j)
                    for (int i = 0; i < NS; ++i) {
                        const R wyz = sp.w[1][j] * sp.w[2][k];
                        const R N = sp.w[0][i] * wyz;
                        const int li = tile_index<SH>(t, sp.base, i, j, k);
                        const R4<R> a = la[li];
                        const R4<R> w = lvn[li];
                        dv[0] += N * a.x;
                        dv[1] += N * a.y;
                        dv[2] += N * a.z;
                        vp[0] += N * w.x;
                        vp[1] += N * w.y;
                        vp[2] += N * w.z;
                        if constexpr (WITH_STRESS) {
                            const R gxN = sp.dw[0][i] * wyz;
                            const R gyN = sp.w[0][i] * sp.dw[1][j] * sp.w[2][k];
                            const R gzN = sp.w[0][i] * sp.w[1][j] * sp.dw[2][k];
                            L[0][0] += w.x * gxN;
                            L[0][1] += w.x * gyN;
                            L[0][2] += w.x * gzN;
                            L[1][0] += w.y * gxN;
                            L[1][1] += w.y * gyN;
                            L[1][2] += w.y * gzN;
                            L[2][0] += w.z * gxN;
                            L[2][1] += w.z * gyN;
                            L[2][2] += w.z * gzN;
                        }
                    }
            for (int a = 0; a < 3; ++a) {
                const R nv = pic ? vp[a] : V[a * n + p] + dt * dv[a];
                V[a * n + p] = nv;
                xp[a] += S.dt * (double)vp[a];
                X[a * n + p] = xp[a];
                if (!isfinite(nv))
                    err |= ERR_NONFINITE;
            }
            if constexpr (WITH_STRESS) {
                const R de[6] = {dt * L[0][0], dt * L[1][1], dt * L[2][2], dt * (L[0][1] + L[1][0]),
                                 dt * (L[1][2] + L[2][1]), dt * (L[0][2] + L[2][0])};
                VO[p] = VO[p] * ((R)1 + de[0] + de[1] + de[2]);
                R sg[6];
                for (int k = 0; k < 6; ++k)
                    sg[k] = SG[k * n + p];
                constitutive<R>(S, de, sg);
                for (int k = 0; k < 6; ++k) {
                    SG[k * n + p] = sg[k];
                    if (!isfinite(sg[k]))
                        err |= ERR_NONFINITE;
                }
            }
            int nc[3];
            const uint32_t e = locate(S, xp, nc);
            if (e) {
                err |= e;
                continue;   // keep the old key; the scene stops
            }
            KEY[p] = cell_to_key(S, nc);
            for (int a = 0; a < 3; ++a)
                if (nc[a] < hb[a] - 1 || nc[a] > hb[a] + kBrick)
                    drift = 1;
        }
        if (err)
            atomicOr(&S.ctl[CTL_ERR], err);
        if (drift || (S.sort_always && threadIdx.x == 0))
            S.ctl[CTL_NEED_SORT] = 1u;
        __syncthreads();
    }
}

// ------------------------------------------------------ instantiations --

template __global__ void k_load<float>(SceneDev *, const double *, const double *, const double *, const double *,
                                       const double *);
template __global__ void k_load<double>(SceneDev *, const double *, const double *, const double *, const double *,
                                        const double *);

}  // namespace mpmx

// --------------------------------------------------- host launch table --

#include "mpmx_launch.h"

namespace mpmx {

template <typename R, int SH>
static KernelSet make_set()
{
    KernelSet k;
    k.load = (const void *)&k_load<R>;
    k.read_out = (const void *)&k_read_out<R>;
    k.nodes_out = (const void *)&k_nodes_out<R>;
    k.clear = (const void *)&k_clear<R>;
    k.scatter = (const void *)&k_sort_scatter<R>;
    k.p2g = (const void *)&k_p2g<R, SH, false>;
    k.stress = (const void *)&k_stress<R, SH>;
    k.g2p = (const void *)&k_g2p<R, SH, false>;
    k.p2g_usl = (const void *)&k_p2g<R, SH, true>;
    k.g2p_usl = (const void *)&k_g2p<R, SH, true>;
    return k;
}

const KernelSet &kernel_set(int prec, int shape)
{
    static const KernelSet sets[2][2] = {{make_set<float, 0>(), make_set<float, 1>()},
                                         {make_set<double, 0>(), make_set<double, 1>()}};
    return sets[prec ? 1 : 0][shape ? 1 : 0];
}

const CommonKernels &common_kernels()
{
    static const CommonKernels c = {(const void *)&k_step_control, (const void *)&k_set_remaining,
                                    (const void *)&k_sort_count,   (const void *)&k_sort_bricks,
                                    (const void *)&k_sort_scan,    (const void *)&k_sort_cells,
                                    (const void *)&k_cell_counts};
    return c;
}

}  // namespace mpmx
