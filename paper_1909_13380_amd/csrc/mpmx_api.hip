// mpmx_api.hip -- host runtime of libmpmx: contexts, scenes, batches and the
// C ABI declared in include/mpmx.h.
//
// A scene owns its device buffers (layout in mpmx_dev.h).  Every step
// is a fixed sequence of launches over a BatchDev (one scene, or many):
//   reorder (its last workgroup runs the step control) -> stress -> g2p_p2g   (USF)
//   reorder -> p2g_usl -> g2p_usl                                              (USL)
//   reorder -> p2g_musl -> musl_g2p -> musl_stress                             (MUSL)
// plus one p2g at the start of a USF call for scenes whose node buffer is
// not yet filled.  The reorder kernel goes straight to the step control
// unless a scene flagged a reorder; all counts the kernels need live in
// device memory, so the host never waits on the GPU between steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "mpmx.h"
#include "mpmx_dev.h"
#include "mpmx_launch.h"

using namespace mpmx;

namespace {

constexpr int kParticleBlock = 256;

struct ProfEvent {
    const char *name;
    hipEvent_t a, b;
};

struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> pool;
    std::vector<ProfEvent> pending;
    std::map<std::string, std::pair<int64_t, double>> totals;
};

// An event recorded on the context stream after a batch's queued steps;
// shared by the batch and its scenes, destroyed with its last holder.
struct StepEvent {
    hipEvent_t e = nullptr;
    ~StepEvent()
    {
        if (e)
            (void)hipEventDestroy(e);
    }
};

// Launch shape of the item kernels: workgroup size (index into
// kItemThreadChoices) and workgroups per compute unit of the persistent
// grid, of the stress-side and of the G2P-side kernels.
struct LaunchCfg {
    int t_stress = 1, t_g2p = 1;
    int bpc_stress = 16, bpc_g2p = 16;
    bool operator==(const LaunchCfg &o) const
    {
        return t_stress == o.t_stress && t_g2p == o.t_g2p && bpc_stress == o.bpc_stress && bpc_g2p == o.bpc_g2p;
    }
};

struct Batch {
    std::vector<uint64_t> ids;
    void *dmem = nullptr;   // one block holding the arrays below
    size_t dcap = 0;
    SceneDev **d_scenes = nullptr;
    int64_t *d_poffs = nullptr, *d_boffs = nullptr, *d_nsteps = nullptr;
    uint32_t *d_ioffs = nullptr, *d_coffs = nullptr, *d_flags = nullptr;
    BatchDev bd{};
    int prec = 0, shape = 0, algo = 0;
    // the last queued steps of this batch (its image is free to rewrite
    // once they are done)
    std::shared_ptr<StepEvent> last_use;
    uint64_t used_at = 0;   // call counter of its last use (the older of two cached batches is rebuilt)
    // executable graph of `gsteps` steps recorded with launch shape gcfg
    hipGraphExec_t gexec = nullptr;
    int gsteps = 0;
    LaunchCfg gcfg;
    void drop_graph()
    {
        if (gexec)
            (void)hipGraphExecDestroy(gexec);
        gexec = nullptr;
        gsteps = 0;
    }
    // the image goes back to the context's device pool (no hipFree, which
    // would wait for the whole device)
    template <typename Pool>
    void release(Pool &pool)
    {
        drop_graph();
        if (dmem)
            pool.release(dmem);
        dmem = nullptr;
        dcap = 0;
        d_scenes = nullptr;
        d_poffs = d_boffs = d_nsteps = nullptr;
        d_ioffs = d_coffs = d_flags = nullptr;
        ids.clear();
        last_use.reset();
    }
};

// Caching pool of device blocks: a freed block is kept and handed out again
// for a request of at most 1.25x its size (+1 MiB), so scenes that come and
// go (the request loop) do not call hipMalloc / hipFree each time.
struct DevicePool {
    std::multimap<uint64_t, void *> idle;
    std::map<void *, uint64_t> size_of;
    void *alloc(uint64_t bytes)
    {
        auto it = idle.lower_bound(bytes);
        if (it != idle.end() && it->first <= bytes + bytes / 4 + (1u << 20)) {
            void *p = it->second;
            idle.erase(it);
            return p;
        }
        void *p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) {
            trim();
            if (hipMalloc(&p, bytes) != hipSuccess)
                return nullptr;
        }
        size_of[p] = bytes;
        return p;
    }
    void release(void *p)
    {
        if (p)
            idle.emplace(size_of[p], p);
    }
    void trim()
    {
        for (auto &kv : idle) {
            (void)hipFree(kv.second);
            size_of.erase(kv.second);
        }
        idle.clear();
    }
    void clear()
    {
        trim();
        for (auto &kv : size_of)
            (void)hipFree(kv.first);
        size_of.clear();
    }
};

struct Scene {
    uint64_t id = 0;
    uint64_t stamp = 0;      // last allocation-free batch call that listed the scene
    SceneDev h{};
    SceneDev *d = nullptr;
    void *block = nullptr;   // every device array of the scene, from the pool
    uint64_t bytes = 0;
    int prec = 0, shape = 0, algo = 0;
    Batch single;
    // the last queued steps of the scene; main_sync: it was last stepped
    // without an event (the allocation-free call), so waiting for it means
    // waiting for the whole context stream
    std::shared_ptr<StepEvent> last;
    bool main_sync = false;
};

}  // namespace

struct mpmx_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int num_cu = 256;
    int reorder_per_cu[2] = {0, 0};   // by precision; 0 until first queried
    std::string err;
    uint64_t next_id = 1;
    std::map<uint64_t, std::unique_ptr<Scene>> scenes;
    Batch cached_batch[2];                 // the two most recent batches of mpmx_batch_step
    uint64_t batch_calls = 0;
    // second stream of the context: scene uploads and read-backs, which then
    // overlap the steps queued on the context stream (default priority)
    hipStream_t aux = nullptr;
    Profiler prof;
    // launch options
    int graph_steps = 8;
    bool autotune = true;
    LaunchCfg fixed;                       // used when autotune is off
    LaunchCfg last;                        // shape of the last stepped batch
    std::map<uint64_t, LaunchCfg> tuned;   // per batch layout
    int64_t graph_launches = 0, tune_runs = 0;
    hipStream_t capture = nullptr;         // private stream for graph capture
    hipStream_t launch_stream = nullptr;   // stream of the launches being issued
    DevicePool pool;
    void *staging = nullptr;               // device staging of host inputs/outputs
    uint64_t staging_cap = 0;
    // mpmx_batch_step_noalloc: this device's address of the file-scope
    // scratch array, the host image of its per-call part (sized at creation)
    // and the call counter that marks the scenes of a call
    void *scratch = nullptr;
    std::vector<uint8_t> scratch_img;
    uint64_t scratch_calls = 0;
    // fences (mpmx_fence_*): events on the context stream, by id
    std::map<uint64_t, hipEvent_t> fences;
    uint64_t next_fence = 1;
};

// ---------------------------------------------- allocation-free batches --
// mpmx_batch_step_noalloc keeps the per-call arrays of a batch (scene list,
// offsets, step counts, reorder flags, brick-scan partial sums, brick list)
// in this array instead of a block the library allocates.  Each GPU holds
// its own copy for the life of the process; host code reaches it only
// through the address hipGetSymbolAddress returns (mpmx_ctx::scratch).
constexpr size_t kScratchBytes = 4u << 20;
constexpr int kNoAllocMaxScenes = 4096;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {

int fail(mpmx_ctx *ctx, int code, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return code;
}

#define HIPCHK(ctx, call)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail((ctx), MPMX_E_HIP, "%s: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                               \
    } while (0)

int flush_profile(mpmx_ctx *ctx)
{
    if (ctx->prof.pending.empty())
        return MPMX_OK;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (auto &pe : ctx->prof.pending) {
        float ms = 0.f;
        HIPCHK(ctx, hipEventElapsedTime(&ms, pe.a, pe.b));
        auto &t = ctx->prof.totals[pe.name];
        t.first += 1;
        t.second += ms;
        ctx->prof.pool.push_back(pe.a);
        ctx->prof.pool.push_back(pe.b);
    }
    ctx->prof.pending.clear();
    return MPMX_OK;
}

hipEvent_t pool_event(mpmx_ctx *ctx)
{
    if (ctx->prof.pool.empty()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess)
            return nullptr;
        return e;
    }
    hipEvent_t e = ctx->prof.pool.back();
    ctx->prof.pool.pop_back();
    return e;
}

int launch(mpmx_ctx *ctx, const char *name, const void *fn, dim3 grid, dim3 block, void **args)
{
    const hipStream_t st = ctx->launch_stream ? ctx->launch_stream : ctx->stream;
    if (st != ctx->stream) {
        HIPCHK(ctx, hipLaunchKernel(fn, grid, block, args, 0, st));
        return MPMX_OK;
    }
    hipEvent_t a = nullptr, b = nullptr;
    if (ctx->prof.on) {
        if (ctx->prof.pending.size() > 8192) {
            int rc = flush_profile(ctx);
            if (rc)
                return rc;
        }
        a = pool_event(ctx);
        b = pool_event(ctx);
        if (a)
            HIPCHK(ctx, hipEventRecord(a, ctx->stream));
    }
    HIPCHK(ctx, hipLaunchKernel(fn, grid, block, args, 0, ctx->stream));
    if (ctx->prof.on && a && b) {
        HIPCHK(ctx, hipEventRecord(b, ctx->stream));
        ctx->prof.pending.push_back({name, a, b});
    }
    return MPMX_OK;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

dim3 particle_grid(int64_t n, int cap = 8192)
{
    int64_t g = ceil_div(std::max<int64_t>(n, 1), kParticleBlock);
    return dim3((unsigned)std::min<int64_t>(g, cap));
}

// --- sizes -------------------------------------------------------------

struct Sizes {
    int64_t nb[3], nbricks, nkeys, nn, N[3], max_items, ncells;
    int ghost;
    size_t real;
};

Sizes sizes_of(const mpmx_mesh *m, int shape, int prec, int64_t np)
{
    Sizes s{};
    s.ghost = shape == MPMX_SHAPE_GIMP ? 1 : 0;
    s.real = prec == MPMX_FP64 ? 8 : 4;
    s.ncells = 1;
    for (int a = 0; a < 3; ++a) {
        s.nb[a] = ceil_div(m->n[a] + kBrick - 1, kBrick);   // any brick shift 0..3
        s.N[a] = m->n[a] + 1 + 2 * s.ghost;
        s.ncells *= m->n[a];
    }
    s.nbricks = s.nb[0] * s.nb[1] * s.nb[2];
    s.nkeys = s.nbricks * kBrickCells;
    s.nn = s.N[0] * s.N[1] * s.N[2];
    s.max_items = ceil_div(np, kChunk) + std::min<int64_t>(np, s.nbricks) + 1;
    return s;
}

uint64_t align_up(uint64_t b) { return (b + 255) & ~uint64_t(255); }

// Device bytes of a scene; the allocation below follows the same list.
uint64_t scene_bytes(const Sizes &s, int64_t np, bool extra_bc, bool force = false, bool iso = false,
                     bool remap = false)
{
    uint64_t b = 0;
    const uint64_t R = s.real;
    for (int buf = 0; buf < 2; ++buf) {
        b += align_up(3 * 8 * (uint64_t)np) + align_up(3 * R * np) + align_up(6 * R * np) + align_up(R * np) +
             align_up(R * np) + align_up(4 * (uint64_t)np) + align_up(4 * (uint64_t)np);
    }
    b += 2 * (align_up(8 * (uint64_t)s.nn) + 2 * align_up(3 * R * s.nn));
    b += 2 * align_up(4 * (uint64_t)s.nkeys) + 2 * align_up(4 * (uint64_t)np);
    b += 2 * align_up(4 * (uint64_t)s.nbricks) + 2 * align_up(4 * (uint64_t)(s.nbricks + 1));
    b += align_up(sizeof(Item) * (uint64_t)s.max_items) + 3 * align_up(sizeof(Tile) * (uint64_t)s.max_items);
    b += align_up(4 * CTL_WORDS) + align_up(sizeof(SceneDev));
    if (extra_bc || force)
        b += align_up((uint64_t)s.nn) + align_up(24 * (uint64_t)s.nn);
    if (force)
        b += align_up(24 * (uint64_t)s.nn);
    if (iso)
        b += align_up(24 * (uint64_t)s.nn);
    if (remap)
        b += align_up(3 * R * s.nn);
    return b;
}

int validate(mpmx_ctx *ctx, const mpmx_mesh *mesh, const mpmx_material *mat, const mpmx_bc *bc,
             const mpmx_scheme *sch)
{
    if (!mesh || mesh->size < sizeof(mpmx_mesh))
        return fail(ctx, MPMX_E_INVALID_ARG, "mesh descriptor missing or too small");
    for (int a = 0; a < 3; ++a)
        if (mesh->n[a] < 1 || mesh->n[a] > kMaxCells[a] || !std::isfinite(mesh->origin[a]))
            return fail(ctx, MPMX_E_INVALID_ARG, "mesh: n[%d]=%d outside 1..%d or origin not finite", a, mesh->n[a],
                        kMaxCells[a]);
    if (!(mesh->h > 0.0) || !std::isfinite(mesh->h))
        return fail(ctx, MPMX_E_INVALID_ARG, "mesh: h must be positive and finite");
    if (mesh->node_x) {
        if (sch && sch->size >= sizeof(mpmx_scheme) && sch->shape != MPMX_SHAPE_LINEAR)
            return fail(ctx, MPMX_E_INVALID_ARG, "mesh: an isoparametric mesh takes linear shape functions only");
        const int64_t N0 = mesh->n[0] + 1, N1 = mesh->n[1] + 1, N2 = mesh->n[2] + 1, nn = N0 * N1 * N2;
        if (24 * nn >= ((int64_t)1 << 32))
            return fail(ctx, MPMX_E_INVALID_ARG, "mesh: too many isoparametric nodes for 32-bit offsets");
        const double *X = mesh->node_x;
        for (int64_t i = 0; i < 3 * nn; ++i)
            if (!std::isfinite(X[i]))
                return fail(ctx, MPMX_E_INVALID_ARG, "mesh: node_x[%lld] not finite", (long long)i);
        // every cell: positive Jacobian det(dx/dxi) at its eight corners
        for (int64_t k = 0; k < mesh->n[2]; ++k)
            for (int64_t j = 0; j < mesh->n[1]; ++j)
                for (int64_t i = 0; i < mesh->n[0]; ++i)
                    for (int q = 0; q < 8; ++q) {
                        const int64_t ci = i + (q & 1), cj = j + ((q >> 1) & 1), ck = k + (q >> 2);
                        double e[3][3];   // edges from the corner towards its three neighbours in the cell
                        for (int a = 0; a < 3; ++a) {
                            const int64_t di = a == 0 ? ((q & 1) ? -1 : 1) : 0;
                            const int64_t dj = a == 1 ? (((q >> 1) & 1) ? -1 : 1) : 0;
                            const int64_t dk = a == 2 ? ((q >> 2) ? -1 : 1) : 0;
                            const double sgn = (di + dj + dk) > 0 ? 1.0 : -1.0;
                            const int64_t I0 = ci + N0 * (cj + N1 * ck);
                            const int64_t I1 = (ci + di) + N0 * ((cj + dj) + N1 * (ck + dk));
                            for (int b = 0; b < 3; ++b)
                                e[a][b] = sgn * (X[3 * I1 + b] - X[3 * I0 + b]);
                        }
                        const double det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                                           e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                                           e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
                        if (!(det > 0.0))
                            return fail(ctx, MPMX_E_INVALID_ARG,
                                        "mesh: cell (%lld,%lld,%lld) is inverted or degenerate at corner %d",
                                        (long long)i, (long long)j, (long long)k, q);
                    }
    }
    if (mat) {
        if (mat->size < sizeof(mpmx_material))
            return fail(ctx, MPMX_E_INVALID_ARG, "material descriptor too small");
        if (mat->model != MPMX_LINEAR_ELASTIC && mat->model != MPMX_DRUCKER_PRAGER)
            return fail(ctx, MPMX_E_INVALID_ARG, "material: unknown model %d", mat->model);
        if (!(mat->E > 0.0) || !(mat->nu > -1.0 && mat->nu < 0.5) || !(mat->rho > 0.0))
            return fail(ctx, MPMX_E_INVALID_ARG, "material: need E > 0, -1 < nu < 0.5, rho > 0");
        if (mat->model == MPMX_DRUCKER_PRAGER) {
            if (mat->dp_cone < 0 || mat->dp_cone > 2)
                return fail(ctx, MPMX_E_INVALID_ARG, "material: unknown cone %d", mat->dp_cone);
            if (!(mat->phi >= 0.0 && mat->phi < M_PI / 2) || !(mat->psi >= 0.0 && mat->psi <= mat->phi) ||
                !(mat->c >= 0.0))
                return fail(ctx, MPMX_E_INVALID_ARG, "material: need 0 <= psi <= phi < pi/2, c >= 0");
        }
    }
    if (bc) {
        if (bc->size < sizeof(mpmx_bc))
            return fail(ctx, MPMX_E_INVALID_ARG, "bc descriptor too small");
        for (int f = 0; f < 6; ++f)
            if (bc->face[f] < 0 || bc->face[f] > 2)
                return fail(ctx, MPMX_E_INVALID_ARG, "bc: face %d rule %d unknown", f, bc->face[f]);
        if (bc->n_extra < 0 || (bc->n_extra > 0 && (!bc->node || !bc->axis || !bc->value)))
            return fail(ctx, MPMX_E_INVALID_ARG, "bc: bad per-node constraint list");
        if (bc->n_force < 0 || (bc->n_force > 0 && (!bc->force_node || !bc->force_value)) ||
            bc->force_ramp_steps < 0)
            return fail(ctx, MPMX_E_INVALID_ARG, "bc: bad nodal force list or ramp");
    }
    if (!sch || sch->size < sizeof(mpmx_scheme))
        return fail(ctx, MPMX_E_INVALID_ARG, "scheme descriptor missing or too small");
    if ((sch->algo != MPMX_USF && sch->algo != MPMX_USL && sch->algo != MPMX_MUSL) ||
        (sch->shape != MPMX_SHAPE_LINEAR && sch->shape != MPMX_SHAPE_GIMP) ||
        (sch->velocity_update != MPMX_FLIP && sch->velocity_update != MPMX_PIC) ||
        (sch->precision != MPMX_FP32 && sch->precision != MPMX_FP64) ||
        (sch->sort_policy != MPMX_SORT_ON_DEMAND && sch->sort_policy != MPMX_SORT_ALWAYS))
        return fail(ctx, MPMX_E_INVALID_ARG, "scheme: unknown algo/shape/velocity_update/precision/sort_policy");
    if (!(sch->dt > 0.0) || !std::isfinite(sch->dt) || !(sch->mass_eps_rel >= 0.0))
        return fail(ctx, MPMX_E_INVALID_ARG, "scheme: need dt > 0 and mass_eps_rel >= 0");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(sch->gravity[a]))
            return fail(ctx, MPMX_E_INVALID_ARG, "scheme: gravity not finite");
    return MPMX_OK;
}

void dp_constants(const mpmx_material *m, double &eta, double &xi, double &etab)
{
    // Mohr-Coulomb matched cones (outer: compression meridian; inner:
    // extension meridian; plane strain).
    auto coef = [&](double ang, double &e, double &x) {
        const double s = std::sin(ang), c = std::cos(ang), t = std::tan(ang), r3 = std::sqrt(3.0);
        if (m->dp_cone == MPMX_DP_INNER) {
            e = 6.0 * s / (r3 * (3.0 + s));
            x = 6.0 * c / (r3 * (3.0 + s));
        } else if (m->dp_cone == MPMX_DP_PLANE_STRAIN) {
            const double d = std::sqrt(9.0 + 12.0 * t * t);
            e = 3.0 * t / d;
            x = 3.0 / d;
        } else {
            e = 6.0 * s / (r3 * (3.0 - s));
            x = 6.0 * c / (r3 * (3.0 - s));
        }
    };
    double xb;
    coef(m->phi, eta, xi);
    coef(m->psi, etab, xb);
}

Scene *find(mpmx_ctx *ctx, uint64_t id)
{
    auto it = ctx->scenes.find(id);
    return it == ctx->scenes.end() ? nullptr : it->second.get();
}

void free_scene(mpmx_ctx *ctx, Scene *s)
{
    s->single.release(ctx->pool);
    ctx->pool.release(s->block);
    s->block = nullptr;
}

// Device staging area of at least `bytes` (contents not preserved); every
// user synchronises the stream before returning.
void *staging(mpmx_ctx *ctx, uint64_t bytes)
{
    if (bytes > ctx->staging_cap) {
        if (ctx->staging)
            (void)hipFree(ctx->staging);
        ctx->staging = nullptr;
        ctx->staging_cap = 0;
        const uint64_t cap = std::max<uint64_t>(bytes, ctx->staging_cap * 2);
        if (hipMalloc(&ctx->staging, cap) != hipSuccess) {
            ctx->pool.trim();
            if (hipMalloc(&ctx->staging, cap) != hipSuccess) {
                ctx->staging = nullptr;
                return nullptr;
            }
        }
        ctx->staging_cap = cap;
    }
    return ctx->staging;
}

int build_batch(mpmx_ctx *ctx, Batch &b, const std::vector<Scene *> &list)
{
    // the previous image may still be read by this batch's queued steps
    if (b.last_use)
        HIPCHK(ctx, hipEventSynchronize(b.last_use->e));
    b.last_use.reset();
    b.drop_graph();
    const int n = (int)list.size();
    const size_t n1 = (size_t)n + 1;
    // layout: scenes[n] | poffs[n+1] | boffs[n+1] | nsteps[n] | ctls[n] | ioffs[n+1] | coffs[n+1] |
    // flags (128-byte aligned) | scan[4 per brick chunk] | bricks[total bricks]
    const size_t n8 = 8 * (size_t)std::max(n, 1);
    int64_t nbr = 0;
    for (auto *sc : list)
        nbr += sc->h.nbricks;
    const size_t o_po = n8, o_bo = o_po + 8 * n1, o_ns = o_bo + 8 * n1, o_ct = o_ns + n8, o_io = o_ct + n8,
                 o_co = o_io + 4 * n1, o_fl = (o_co + 4 * n1 + 127) & ~(size_t)127, o_sc = o_fl + 4 * BF_WORDS,
                 o_br = o_sc + 16 * (size_t)kScanChunks, total = o_br + 4 * (size_t)std::max<int64_t>(nbr, 1);
    std::vector<uint8_t> img(total, 0);
    int64_t maxit = 0, *po = (int64_t *)(img.data() + o_po), *bo = (int64_t *)(img.data() + o_bo);
    SceneDev **sp = (SceneDev **)img.data();
    uint32_t **cp = (uint32_t **)(img.data() + o_ct);
    for (int i = 0; i < n; ++i) {
        sp[i] = list[i]->d;
        cp[i] = list[i]->h.ctl;
        po[i + 1] = po[i] + list[i]->h.np;
        bo[i + 1] = bo[i] + list[i]->h.nbricks;
        maxit += list[i]->h.max_items;
    }
    if (total > b.dcap) {
        if (b.dmem)
            ctx->pool.release(b.dmem);
        b.dmem = ctx->pool.alloc(2 * total);
        b.dcap = 0;
        if (!b.dmem)
            return fail(ctx, MPMX_E_OOM, "batch image of %zu bytes", 2 * total);
        b.dcap = 2 * total;
    }
    uint8_t *base = (uint8_t *)b.dmem;
    HIPCHK(ctx, hipMemcpy(base, img.data(), total, hipMemcpyHostToDevice));
    b.d_scenes = (SceneDev **)base;
    b.d_poffs = (int64_t *)(base + o_po);
    b.d_boffs = (int64_t *)(base + o_bo);
    b.d_nsteps = (int64_t *)(base + o_ns);
    b.d_ioffs = (uint32_t *)(base + o_io);
    b.d_coffs = (uint32_t *)(base + o_co);
    b.d_flags = (uint32_t *)(base + o_fl);
    po = (int64_t *)(img.data() + o_po);
    bo = (int64_t *)(img.data() + o_bo);
    b.bd.scenes = b.d_scenes;
    b.bd.ctls = (uint32_t *const *)(base + o_ct);
    b.bd.poffs = b.d_poffs;
    b.bd.boffs = b.d_boffs;
    b.bd.ioffs = b.d_ioffs;
    b.bd.coffs = b.d_coffs;

    b.bd.flags = b.d_flags;
    b.bd.scan = (uint32_t *)(base + o_sc);
    b.bd.bricks = (uint32_t *)(base + o_br);
    b.bd.nscenes = n;
    b.bd.total_particles = po[n];
    b.bd.total_bricks = bo[n];
    b.bd.max_items = maxit;
    b.ids.clear();
    for (auto *s : list)
        b.ids.push_back(s->id);
    if (n) {
        b.prec = list[0]->prec;
        b.shape = list[0]->shape;
        b.algo = list[0]->algo;
    }
    return MPMX_OK;
}

// Reorder workgroups per CU: kReorderPerCu, or fewer if the kernel's
// resources allow fewer resident at once.
int reorder_per_cu(mpmx_ctx *ctx, int prec, const void *fn)
{
    int &n = ctx->reorder_per_cu[prec ? 1 : 0];
    if (n == 0) {
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, kBlock, 0) != hipSuccess || occ < 1)
            occ = 1;
        n = std::min(occ, kReorderPerCu);
    }
    return n;
}

// Launches of one step of every scene of b (the first step of a call also
// fills the node buffer of USF scenes that need it).  `ev`, when given,
// receives events around the item kernels: [0] before, [1] between, [2]
// after.
int enqueue_step(mpmx_ctx *ctx, Batch &b, const LaunchCfg &cfg, bool first, hipEvent_t *ev)
{
    const KernelSet &K = kernel_set(b.prec, b.shape);
    BatchDev bd = b.bd;
    void *a_bd[] = {&bd};
    const hipStream_t st = ctx->launch_stream ? ctx->launch_stream : ctx->stream;
    // the reorder kernel: enough workgroups for one pass over the particles
    // and one brick per wavefront, at most kReorderPerCu per CU; it returns
    // at once on steps that need no reorder
    const int64_t rwork = std::max({ceil_div(bd.total_particles, (int64_t)kBlock * kSortU),
                                    ceil_div(bd.total_bricks, kBlock / 64), (int64_t)bd.nscenes, (int64_t)1});
    const dim3 rg((unsigned)std::min<int64_t>(rwork, (int64_t)reorder_per_cu(ctx, b.prec, K.reorder) * ctx->num_cu));
    // item grids: a multiple of the XCD count unless there are fewer items
    auto item_grid = [&](int per_cu) {
        int64_t n = std::min<int64_t>(bd.max_items, (int64_t)per_cu * ctx->num_cu);
        if (n >= kXcds)
            n -= n % kXcds;
        return dim3((unsigned)std::max<int64_t>(1, n));
    };
    const dim3 igs = item_grid(cfg.bpc_stress), igg = item_grid(cfg.bpc_g2p);
    const dim3 ts(kItemThreadChoices[cfg.t_stress]), tg(kItemThreadChoices[cfg.t_g2p]);
    int rc;
    if ((rc = launch(ctx, "reorder", K.reorder, rg, dim3(kBlock), a_bd)))
        return rc;
    if (b.algo == MPMX_USF && first && (rc = launch(ctx, "p2g", K.p2g[cfg.t_g2p], igg, tg, a_bd)))
        return rc;
    if (ev)
        HIPCHK(ctx, hipEventRecord(ev[0], st));
    if (b.algo == MPMX_USF)
        rc = launch(ctx, "stress", K.stress[cfg.t_stress], igs, ts, a_bd);
    else if (b.algo == MPMX_USL)
        rc = launch(ctx, "p2g_usl", K.p2g_usl[cfg.t_stress], igs, ts, a_bd);
    else
        rc = launch(ctx, "p2g_musl", K.p2g_musl[cfg.t_stress], igs, ts, a_bd);
    if (rc)
        return rc;
    if (ev)
        HIPCHK(ctx, hipEventRecord(ev[1], st));
    if (b.algo == MPMX_USF)
        rc = launch(ctx, "g2p_p2g", K.g2p_p2g[cfg.t_g2p], igg, tg, a_bd);
    else if (b.algo == MPMX_USL)
        rc = launch(ctx, "g2p_usl", K.g2p_usl[cfg.t_g2p], igg, tg, a_bd);
    else if (!(rc = launch(ctx, "musl_g2p", K.musl_g2p[cfg.t_g2p], igg, tg, a_bd)))
        rc = launch(ctx, "musl_stress", K.musl_stress[cfg.t_g2p], igg, tg, a_bd);
    if (rc)
        return rc;
    if (ev)
        HIPCHK(ctx, hipEventRecord(ev[2], st));
    return MPMX_OK;
}

uint64_t layout_key(const Batch &b)
{
    int bucket = 0;
    while (bucket < 62 && ((int64_t)1 << (bucket + 1)) <= b.bd.total_particles)
        ++bucket;
    return (uint64_t)b.prec | (uint64_t)b.shape << 2 | (uint64_t)b.algo << 4 | (uint64_t)bucket << 8;
}

// Online tuning of the item kernels' launch shape on real steps of the call:
// every (grid density, workgroup size) pair, kTuneReps steps each, timing
// the stress-side and the G2P-side kernels separately (each keeps its
// fastest repeat), and each kernel keeps its own fastest pair.  Pairs within
// kTuneBand plus kTuneSlackMs of the fastest count as ties (the slack covers
// the timing jitter of short kernels), and ties go to the first pair in a
// fixed preference order (16 workgroups per CU, then 32, 8 and 64; larger
// workgroups first), so that timing noise between nearly equal shapes does
// not change the choice from one run to the next.
constexpr int kTuneReps = 3;
constexpr int kTuneDensity[] = {8, 16, 32, 64};
constexpr int kNumTuneDensity = 4;
constexpr int kTuneSteps = kTuneReps * kNumItemThreadChoices * kNumTuneDensity;
constexpr float kTuneBand = 0.01f;
constexpr float kTuneSlackMs = 0.002f;
static_assert(kTuneSteps + 1 <= MPMX_TUNE_MIN_STEPS, "tuning must fit in the calls it runs on");

int tune(mpmx_ctx *ctx, Batch &b, LaunchCfg &best)
{
    std::vector<hipEvent_t> ev(3 * kTuneSteps, nullptr);
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            for (auto &x : ev)
                if (x)
                    (void)hipEventDestroy(x);
            return fail(ctx, MPMX_E_HIP, "tuning: event creation failed");
        }
    int rc = MPMX_OK;
    int k = 0;
    LaunchCfg cfg = best;
    // repeats in the outer loop: a drift over the tuning steps (clocks, the
    // scene's own evolution) then weighs on every shape alike
    constexpr int kShapes = kNumTuneDensity * kNumItemThreadChoices;
    for (int r = 0; r < kTuneReps && !rc; ++r)
        for (int d = 0; d < kNumTuneDensity && !rc; ++d)
            for (int t = 0; t < kNumItemThreadChoices && !rc; ++t, ++k) {
                cfg.bpc_stress = cfg.bpc_g2p = kTuneDensity[d];
                cfg.t_stress = cfg.t_g2p = t;
                rc = enqueue_step(ctx, b, cfg, false, &ev[3 * k]);
            }
    if (!rc && hipEventSynchronize(ev[3 * k - 1]) != hipSuccess)
        rc = fail(ctx, MPMX_E_HIP, "tuning: event wait failed");
    // ts[d][t], tg[d][t]: fastest repeat of each kernel at density d, size t
    float ts[kNumTuneDensity][kNumItemThreadChoices], tg[kNumTuneDensity][kNumItemThreadChoices];
    for (int d = 0; d < kNumTuneDensity && !rc; ++d)
        for (int t = 0; t < kNumItemThreadChoices && !rc; ++t) {
            ts[d][t] = tg[d][t] = 1e30f;
            for (int r = 0; r < kTuneReps; ++r) {
                const int q = r * kShapes + d * kNumItemThreadChoices + t;
                float m1 = 0.f, m2 = 0.f;
                if (hipEventElapsedTime(&m1, ev[3 * q], ev[3 * q + 1]) != hipSuccess ||
                    hipEventElapsedTime(&m2, ev[3 * q + 1], ev[3 * q + 2]) != hipSuccess) {
                    rc = fail(ctx, MPMX_E_HIP, "tuning: event timing failed");
                    break;
                }
                ts[d][t] = std::min(ts[d][t], m1);
                tg[d][t] = std::min(tg[d][t], m2);
            }
        }
    if (!rc) {
        // preference order: 16 workgroups per CU, then 32, 8, 64; sizes
        // largest first
        const int dorder[kNumTuneDensity] = {1, 2, 0, 3};
        auto choose = [&](const float (&tm)[kNumTuneDensity][kNumItemThreadChoices], int &bpc, int &t_out) {
            float fastest = 1e30f;
            for (int d = 0; d < kNumTuneDensity; ++d)
                for (int t = 0; t < kNumItemThreadChoices; ++t)
                    fastest = std::min(fastest, tm[d][t]);
            for (int i = 0; i < kNumTuneDensity; ++i)
                for (int t = kNumItemThreadChoices - 1; t >= 0; --t)
                    if (tm[dorder[i]][t] <= fastest * (1.f + kTuneBand) + kTuneSlackMs) {
                        bpc = kTuneDensity[dorder[i]];
                        t_out = t;
                        return;
                    }
        };
        choose(ts, best.bpc_stress, best.t_stress);
        choose(tg, best.bpc_g2p, best.t_g2p);
    }
    for (auto &e : ev)
        (void)hipEventDestroy(e);
    ctx->tune_runs += rc ? 0 : 1;
    return rc;
}

// Record `steps` non-first steps of b into an executable graph.
int record_graph(mpmx_ctx *ctx, Batch &b, const LaunchCfg &cfg, int steps)
{
    b.drop_graph();
    if (!ctx->capture)
        HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
    HIPCHK(ctx, hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal));
    ctx->launch_stream = ctx->capture;
    int rc = MPMX_OK;
    for (int i = 0; i < steps && !rc; ++i)
        rc = enqueue_step(ctx, b, cfg, false, nullptr);
    ctx->launch_stream = nullptr;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(ctx->capture, &g);
    if (rc) {
        if (g)
            (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess)
        return fail(ctx, MPMX_E_HIP, "graph capture: %s", hipGetErrorString(e));
    const hipError_t ei = hipGraphInstantiate(&b.gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
        b.gexec = nullptr;
        return fail(ctx, MPMX_E_HIP, "graph instantiate: %s", hipGetErrorString(ei));
    }
    b.gsteps = steps;
    b.gcfg = cfg;
    return MPMX_OK;
}

// Record an event after the steps just queued for b; the batch and each of
// its scenes keep it, so that reading or freeing a scene waits for its own
// steps only.
int mark_queued(mpmx_ctx *ctx, Batch &b)
{
    auto ev = std::make_shared<StepEvent>();
    HIPCHK(ctx, hipEventCreateWithFlags(&ev->e, hipEventDisableTiming));
    HIPCHK(ctx, hipEventRecord(ev->e, ctx->stream));
    b.last_use = ev;
    for (uint64_t id : b.ids) {
        auto it = ctx->scenes.find(id);
        if (it != ctx->scenes.end()) {
            it->second->last = ev;
            it->second->main_sync = false;
        }
    }
    return MPMX_OK;
}

// Make stream st wait for the queued steps of scene s.
int wait_for_scene(mpmx_ctx *ctx, Scene *s, hipStream_t st)
{
    if (s->main_sync) {
        hipEvent_t e = nullptr;
        HIPCHK(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
        hipError_t r = hipEventRecord(e, ctx->stream);
        if (r == hipSuccess)
            r = hipStreamWaitEvent(st, e, 0);
        (void)hipEventDestroy(e);
        if (r != hipSuccess)
            return fail(ctx, MPMX_E_HIP, "stream wait: %s", hipGetErrorString(r));
    } else if (s->last) {
        HIPCHK(ctx, hipStreamWaitEvent(st, s->last->e, 0));
    }
    return MPMX_OK;
}

// Block the host until the queued steps of scene s are done.
int host_wait_for_scene(mpmx_ctx *ctx, Scene *s)
{
    if (s->main_sync)
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    else if (s->last)
        HIPCHK(ctx, hipEventSynchronize(s->last->e));
    return MPMX_OK;
}

// Queue `steps` steps of every scene of b (scene i: nsteps[i], or `uniform`
// for all when nsteps is null).  The host never waits on the GPU, except
// once per batch layout while tuning.
int run_steps(mpmx_ctx *ctx, Batch &b, const int64_t *nsteps, int64_t uniform)
{
    const int n = b.bd.nscenes;
    if (n == 0)
        return MPMX_OK;
    std::vector<int64_t> ns(n);
    int64_t smax = 0;
    for (int i = 0; i < n; ++i) {
        ns[i] = nsteps ? nsteps[i] : uniform;
        smax = std::max(smax, ns[i]);
    }
    if (smax <= 0)
        return MPMX_OK;
    ctx->launch_stream = nullptr;
    HIPCHK(ctx, hipMemcpyAsync(b.d_nsteps, ns.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, ctx->stream));
    const CommonKernels &C = common_kernels();
    BatchDev bd = b.bd;
    const int64_t *dns = b.d_nsteps;
    void *a_begin[] = {&bd, &dns};
    int rc;
    if ((rc = launch(ctx, "begin", C.begin, dim3(1), dim3(1024), a_begin)))
        return rc;
    LaunchCfg cfg = ctx->fixed;
    const uint64_t key = layout_key(b);
    bool tuned = !ctx->autotune;
    if (ctx->autotune) {
        auto it = ctx->tuned.find(key);
        if (it != ctx->tuned.end()) {
            cfg = it->second;
            tuned = true;
        }
    }
    if ((rc = enqueue_step(ctx, b, cfg, true, nullptr)))
        return rc;
    int64_t left = smax - 1;
    if (!tuned && !ctx->prof.on && smax >= MPMX_TUNE_MIN_STEPS) {
        if ((rc = tune(ctx, b, cfg)))
            return rc;
        ctx->tuned[key] = cfg;
        left -= kTuneSteps;
    }
    ctx->last = cfg;
    const int K = ctx->graph_steps;
    // the K-step graph is recorded by the first call of more than one step
    // with this launch shape (recording runs nothing), so that later calls
    // only replay it, however few steps this one has left
    if (K > 0 && !ctx->prof.on && smax > 1 && (!b.gexec || b.gsteps != K || !(b.gcfg == cfg)))
        if ((rc = record_graph(ctx, b, cfg, K)))
            return rc;
    if (K > 0 && !ctx->prof.on && left >= K) {
        for (; left >= K; left -= K) {
            HIPCHK(ctx, hipGraphLaunch(b.gexec, ctx->stream));
            ++ctx->graph_launches;
        }
    }
    for (; left > 0; --left)
        if ((rc = enqueue_step(ctx, b, cfg, false, nullptr)))
            return rc;
    return mark_queued(ctx, b);
}

int read_ctl(mpmx_ctx *ctx, Scene *s, uint32_t *ctl)
{
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    HIPCHK(ctx, hipMemcpy(ctl, s->h.ctl, sizeof(uint32_t) * CTL_WORDS, hipMemcpyDeviceToHost));
    return MPMX_OK;
}

int err_code(uint32_t bits)
{
    if (bits & ERR_OUT_OF_MESH)
        return MPMX_E_OUT_OF_MESH;
    if (bits & ERR_NONFINITE)
        return MPMX_E_NONFINITE;
    if (bits)
        return MPMX_E_STATE;
    return MPMX_OK;
}

}  // namespace

// ================================================================ C ABI ==

extern "C" {

int mpmx_version(void) { return MPMX_VERSION; }

int mpmx_create(mpmx_ctx **out, int device, void *stream)
{
    if (!out)
        return MPMX_E_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return MPMX_E_HIP;
    if (hipSetDevice(device) != hipSuccess)
        return MPMX_E_HIP;
    auto *ctx = new (std::nothrow) mpmx_ctx();
    if (!ctx)
        return MPMX_E_OOM;
    ctx->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        ctx->num_cu = prop.multiProcessorCount;
    if (stream) {
        ctx->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            delete ctx;
            return MPMX_E_HIP;
        }
        ctx->own_stream = true;
    }
    if (hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking) != hipSuccess) {
        if (ctx->own_stream)
            (void)hipStreamDestroy(ctx->stream);
        delete ctx;
        return MPMX_E_HIP;
    }
    // this device's copy of the allocation-free scratch array (the device
    // is current); the host image of its per-call part is sized here, so the
    // allocation-free call allocates nothing
    void *sp = nullptr;
    if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) != hipSuccess || !sp) {
        (void)hipStreamDestroy(ctx->aux);
        if (ctx->own_stream)
            (void)hipStreamDestroy(ctx->stream);
        delete ctx;
        return MPMX_E_HIP;
    }
    ctx->scratch = sp;
    ctx->scratch_img.assign(40 * (size_t)kNoAllocMaxScenes + 16, 0);
    *out = ctx;
    return MPMX_OK;
}

void mpmx_destroy(mpmx_ctx *ctx)
{
    if (!ctx)
        return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipStreamSynchronize(ctx->aux);
    for (auto &kv : ctx->scenes)
        free_scene(ctx, kv.second.get());
    ctx->scenes.clear();
    for (auto &cb : ctx->cached_batch)
        cb.release(ctx->pool);
    for (auto &kv : ctx->fences)
        (void)hipEventDestroy(kv.second);
    ctx->fences.clear();
    if (ctx->staging)
        (void)hipFree(ctx->staging);
    ctx->pool.clear();
    for (auto &pe : ctx->prof.pending) {
        (void)hipEventDestroy(pe.a);
        (void)hipEventDestroy(pe.b);
    }
    for (auto e : ctx->prof.pool)
        (void)hipEventDestroy(e);
    if (ctx->capture)
        (void)hipStreamDestroy(ctx->capture);
    if (ctx->aux)
        (void)hipStreamDestroy(ctx->aux);
    if (ctx->own_stream)
        (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

const char *mpmx_last_error(const mpmx_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

int mpmx_set_option(mpmx_ctx *ctx, int option, int64_t value)
{
    if (!ctx)
        return MPMX_E_INVALID_ARG;
    auto tindex = [](int64_t v) {
        for (int i = 0; i < kNumItemThreadChoices; ++i)
            if (kItemThreadChoices[i] == v)
                return i;
        return -1;
    };
    switch (option) {
    case MPMX_OPT_GRAPH_STEPS:
        if (value < 0 || value > 1024)
            return fail(ctx, MPMX_E_INVALID_ARG, "graph steps must be 0..1024");
        ctx->graph_steps = (int)value;
        return MPMX_OK;
    case MPMX_OPT_AUTOTUNE:
        if (value != 0 && value != 1)
            return fail(ctx, MPMX_E_INVALID_ARG, "autotune must be 0 or 1");
        ctx->autotune = value != 0;
        return MPMX_OK;
    case MPMX_OPT_STRESS_THREADS:
    case MPMX_OPT_G2P_THREADS: {
        const int t = tindex(value);
        if (t < 0)
            return fail(ctx, MPMX_E_INVALID_ARG, "workgroup size must be 64, 128 or 256");
        (option == MPMX_OPT_STRESS_THREADS ? ctx->fixed.t_stress : ctx->fixed.t_g2p) = t;
        ctx->autotune = false;
        return MPMX_OK;
    }
    case MPMX_OPT_BLOCKS_PER_CU:
    case MPMX_OPT_STRESS_BLOCKS_PER_CU:
    case MPMX_OPT_G2P_BLOCKS_PER_CU:
        if (value < 1 || value > 64)
            return fail(ctx, MPMX_E_INVALID_ARG, "blocks per CU must be 1..64");
        if (option != MPMX_OPT_G2P_BLOCKS_PER_CU)
            ctx->fixed.bpc_stress = (int)value;
        if (option != MPMX_OPT_STRESS_BLOCKS_PER_CU)
            ctx->fixed.bpc_g2p = (int)value;
        ctx->autotune = false;
        return MPMX_OK;
    default:
        return fail(ctx, MPMX_E_INVALID_ARG, "unknown or read-only option %d", option);
    }
}

int mpmx_get_option(mpmx_ctx *ctx, int option, int64_t *value)
{
    if (!ctx || !value)
        return MPMX_E_INVALID_ARG;
    switch (option) {
    case MPMX_OPT_GRAPH_STEPS: *value = ctx->graph_steps; return MPMX_OK;
    case MPMX_OPT_AUTOTUNE: *value = ctx->autotune ? 1 : 0; return MPMX_OK;
    case MPMX_OPT_STRESS_THREADS: *value = kItemThreadChoices[ctx->last.t_stress]; return MPMX_OK;
    case MPMX_OPT_G2P_THREADS: *value = kItemThreadChoices[ctx->last.t_g2p]; return MPMX_OK;
    case MPMX_OPT_BLOCKS_PER_CU:
    case MPMX_OPT_STRESS_BLOCKS_PER_CU: *value = ctx->last.bpc_stress; return MPMX_OK;
    case MPMX_OPT_G2P_BLOCKS_PER_CU: *value = ctx->last.bpc_g2p; return MPMX_OK;
    case MPMX_OPT_GRAPH_LAUNCHES: *value = ctx->graph_launches; return MPMX_OK;
    case MPMX_OPT_TUNE_RUNS: *value = ctx->tune_runs; return MPMX_OK;
    default: return fail(ctx, MPMX_E_INVALID_ARG, "unknown option %d", option);
    }
}

int mpmx_profile_enable(mpmx_ctx *ctx, int enable)
{
    if (!ctx)
        return MPMX_E_INVALID_ARG;
    if (!enable) {
        int rc = flush_profile(ctx);
        if (rc)
            return rc;
    }
    ctx->prof.on = enable != 0;
    return MPMX_OK;
}

int mpmx_profile_reset(mpmx_ctx *ctx)
{
    if (!ctx)
        return MPMX_E_INVALID_ARG;
    int rc = flush_profile(ctx);
    if (rc)
        return rc;
    ctx->prof.totals.clear();
    return MPMX_OK;
}

int mpmx_profile_read(mpmx_ctx *ctx, int cap, const char **names, int64_t *launches, double *ms, int *n)
{
    if (!ctx || !n || cap < 0)
        return MPMX_E_INVALID_ARG;
    int rc = flush_profile(ctx);
    if (rc)
        return rc;
    int i = 0;
    for (auto &kv : ctx->prof.totals) {
        if (i < cap) {
            if (names)
                names[i] = kv.first.c_str();
            if (launches)
                launches[i] = kv.second.first;
            if (ms)
                ms[i] = kv.second.second;
        }
        ++i;
    }
    *n = i;
    return MPMX_OK;
}

int mpmx_scene_bytes(const mpmx_mesh *mesh, const mpmx_scheme *scheme, int64_t n_particles, uint64_t *bytes)
{
    if (!bytes || n_particles < 0)
        return MPMX_E_INVALID_ARG;
    int rc = validate(nullptr, mesh, nullptr, nullptr, scheme);
    if (rc)
        return rc;
    Sizes s = sizes_of(mesh, scheme->shape, scheme->precision, n_particles);
    *bytes = scene_bytes(s, n_particles, false, false, mesh->node_x != nullptr, scheme->algo == MPMX_MUSL);
    return MPMX_OK;
}

int mpmx_scene_create(mpmx_ctx *ctx, const mpmx_mesh *mesh, const mpmx_material *mat, const mpmx_bc *bc,
                      const mpmx_scheme *sch, const mpmx_particles *parts, uint64_t *scene_out)
{
    if (!ctx || !scene_out)
        return MPMX_E_INVALID_ARG;
    ctx->err.clear();
    *scene_out = 0;
    if (!mat || !bc)
        return fail(ctx, MPMX_E_INVALID_ARG, "material and bc descriptors are required");
    int rc = validate(ctx, mesh, mat, bc, sch);
    if (rc)
        return rc;
    if (!parts || parts->size < sizeof(mpmx_particles) || parts->n < 0 ||
        (parts->mem != MPMX_MEM_HOST && parts->mem != MPMX_MEM_DEVICE))
        return fail(ctx, MPMX_E_INVALID_ARG, "particles descriptor invalid");
    const int64_t np = parts->n;
    if (np > 0 && (!parts->x || !parts->v || !parts->vol || !parts->mass))
        return fail(ctx, MPMX_E_INVALID_ARG, "particles: x, v, vol and mass are required");
    const Sizes sz = sizes_of(mesh, sch->shape, sch->precision, np);
    // the kernels address one field (all its components) with 32-bit byte offsets
    const int64_t rb = (int64_t)sz.real;
    if (np * std::max<int64_t>(24, 6 * rb) >= (int64_t)1 << 32)
        return fail(ctx, MPMX_E_INVALID_ARG, "particles: at most %lld per scene at this precision",
                    (long long)((((int64_t)1 << 32) - 1) / std::max<int64_t>(24, 6 * rb)));
    if (sz.nkeys >= (int64_t)1 << 32 || sz.nn * std::max<int64_t>(8, 3 * rb) >= (int64_t)1 << 32)
        return fail(ctx, MPMX_E_INVALID_ARG, "mesh too large for 32-bit cell keys and node offsets");
    const bool force = bc->n_force > 0;
    const bool extra = bc->n_extra > 0 || force;
    for (int64_t e = 0; e < bc->n_extra; ++e)
        if (bc->node[e] < 0 || bc->node[e] >= sz.nn || bc->axis[e] < 0 || bc->axis[e] > 2 ||
            !std::isfinite(bc->value[e]))
            return fail(ctx, MPMX_E_INVALID_ARG, "bc: constraint %lld names node %lld axis %d", (long long)e,
                        (long long)bc->node[e], bc->axis[e]);
    for (int64_t e = 0; e < bc->n_force; ++e)
        if (bc->force_node[e] < 0 || bc->force_node[e] >= sz.nn || !std::isfinite(bc->force_value[3 * e]) ||
            !std::isfinite(bc->force_value[3 * e + 1]) || !std::isfinite(bc->force_value[3 * e + 2]))
            return fail(ctx, MPMX_E_INVALID_ARG, "bc: force %lld names node %lld or is not finite", (long long)e,
                        (long long)bc->force_node[e]);
    HIPCHK(ctx, hipSetDevice(ctx->device));

    const bool iso = mesh->node_x != nullptr;
    auto sc = std::make_unique<Scene>();
    Scene *s = sc.get();
    s->prec = sch->precision;
    s->shape = iso ? 2 : sch->shape;   // kernel shape: 2 is the isoparametric trilinear hexahedron
    s->algo = sch->algo;
    SceneDev &h = s->h;
    // one block of exactly scene_bytes(); the arrays are carved in the order
    // scene_bytes() counts them
    const uint64_t total = scene_bytes(sz, np, extra, force, iso, sch->algo == MPMX_MUSL);
    s->block = ctx->pool.alloc(total);
    if (!s->block)
        return fail(ctx, MPMX_E_OOM, "device allocation of %llu bytes failed", (unsigned long long)total);
    s->bytes = total;
    uint64_t used = 0;
    std::vector<std::pair<void *, uint64_t>> zero_ranges;
    auto dalloc = [&](uint64_t bytes, bool zero) -> void * {
        if (bytes == 0)
            return nullptr;
        if (used + align_up(bytes) > total)
            return nullptr;
        void *p = (uint8_t *)s->block + used;
        used += align_up(bytes);
        if (zero)
            zero_ranges.push_back({p, align_up(bytes)});
        return p;
    };
    bool ok = true;
    auto need = [&](void *p, uint64_t bytes) {
        if (bytes && !p)
            ok = false;
        return p;
    };
    const uint64_t R = sz.real;
    for (int b = 0; b < 2; ++b) {
        h.x[b] = (double *)need(dalloc(3 * 8 * (uint64_t)np, false), np);
        h.v[b] = need(dalloc(3 * R * np, false), np);
        h.sig[b] = need(dalloc(6 * R * np, false), np);
        h.vol[b] = need(dalloc(R * np, false), np);
        h.mass[b] = need(dalloc(R * np, false), np);
        h.cell[b] = (uint32_t *)need(dalloc(4 * (uint64_t)np, false), np);
        h.pid[b] = (uint32_t *)need(dalloc(4 * (uint64_t)np, false), np);
    }
    for (int b = 0; b < 2; ++b) {
        h.nm[b] = (double *)need(dalloc(8 * (uint64_t)sz.nn, true), 1);
        h.np_[b] = need(dalloc(3 * R * sz.nn, true), 1);
        h.nf[b] = need(dalloc(3 * R * sz.nn, true), 1);
    }
    h.cnt = (uint32_t *)need(dalloc(4 * (uint64_t)sz.nkeys, true), 1);
    h.cstart = (uint32_t *)need(dalloc(4 * (uint64_t)sz.nkeys, false), 1);
    h.rank = (uint32_t *)need(dalloc(4 * (uint64_t)np, false), np);
    h.perm = (uint32_t *)need(dalloc(4 * (uint64_t)np, false), np);
    h.bcnt = (uint32_t *)need(dalloc(4 * (uint64_t)sz.nbricks, true), 1);
    h.bitem = (uint32_t *)need(dalloc(4 * (uint64_t)sz.nbricks, true), 1);
    h.bstart = (uint32_t *)need(dalloc(4 * (uint64_t)(sz.nbricks + 1), true), 1);
    h.istart = (uint32_t *)need(dalloc(4 * (uint64_t)(sz.nbricks + 1), true), 1);
    h.items = (Item *)need(dalloc(sizeof(Item) * (uint64_t)sz.max_items, true), 1);
    h.tiles[0] = (Tile *)need(dalloc(sizeof(Tile) * (uint64_t)sz.max_items, true), 1);
    h.tiles[1] = (Tile *)need(dalloc(sizeof(Tile) * (uint64_t)sz.max_items, true), 1);
    h.tstep = (Tile *)need(dalloc(sizeof(Tile) * (uint64_t)sz.max_items, true), 1);
    h.ctl = (uint32_t *)need(dalloc(4 * CTL_WORDS, true), 1);
    s->d = (SceneDev *)need(dalloc(sizeof(SceneDev), false), 1);
    if (sch->algo == MPMX_MUSL)   // zero at creation; each step clears what the previous one wrote
        h.nr = need(dalloc(3 * R * sz.nn, true), 1);
    if (extra) {
        std::vector<uint8_t> mask(sz.nn, 0);
        std::vector<double> val(3 * sz.nn, 0.0), fv(force ? 3 * sz.nn : 0, 0.0);
        for (int64_t e = 0; e < bc->n_extra; ++e) {
            mask[bc->node[e]] |= (uint8_t)(1u << bc->axis[e]);
            val[3 * bc->node[e] + bc->axis[e]] = bc->value[e];
        }
        for (int64_t e = 0; e < bc->n_force; ++e) {
            mask[bc->force_node[e]] |= (uint8_t)8u;
            for (int a = 0; a < 3; ++a)
                fv[3 * bc->force_node[e] + a] += bc->force_value[3 * e + a];
        }
        void *dm = need(dalloc(sz.nn, false), 1);
        void *dv = need(dalloc(24 * (uint64_t)sz.nn, false), 1);
        void *df = force ? need(dalloc(24 * (uint64_t)sz.nn, false), 1) : nullptr;
        if (ok) {
            HIPCHK(ctx, hipMemcpy(dm, mask.data(), sz.nn, hipMemcpyHostToDevice));
            HIPCHK(ctx, hipMemcpy(dv, val.data(), 24 * sz.nn, hipMemcpyHostToDevice));
            if (df)
                HIPCHK(ctx, hipMemcpy(df, fv.data(), 24 * sz.nn, hipMemcpyHostToDevice));
        }
        h.bc_mask = (const uint8_t *)dm;
        h.bc_val = (const double *)dv;
        h.bc_force = (const double *)df;
        h.force_ramp = bc->force_ramp_steps;
    }
    if (iso) {
        // node positions, structure of arrays x[3][nn]
        std::vector<double> X(3 * sz.nn);
        for (int64_t I = 0; I < sz.nn; ++I)
            for (int a = 0; a < 3; ++a)
                X[a * sz.nn + I] = mesh->node_x[3 * I + a];
        void *dX = need(dalloc(24 * (uint64_t)sz.nn, false), 1);
        if (ok)
            HIPCHK(ctx, hipMemcpy(dX, X.data(), 24 * sz.nn, hipMemcpyHostToDevice));
        h.X = (const double *)dX;
    }
    // uploads go through the second stream, so that they overlap steps
    // already queued on the context stream
    for (auto &z : zero_ranges)
        if (ok && hipMemsetAsync(z.first, 0, z.second, ctx->aux) != hipSuccess)
            ok = false;
    // the control words below are written with blocking copies: the zeroing
    // must be complete first
    if (ok && hipStreamSynchronize(ctx->aux) != hipSuccess)
        ok = false;
    if (!ok) {
        free_scene(ctx, s);
        return fail(ctx, MPMX_E_OOM, "device arrays of %llu bytes do not fit the scene's block",
                    (unsigned long long)total);
    }

    for (int a = 0; a < 3; ++a) {
        h.origin[a] = mesh->origin[a];
        h.n[a] = mesh->n[a];
        h.nb[a] = (int)sz.nb[a];
        h.cmin[a] = std::numeric_limits<int>::max();   // k_load takes the particles' minimum
        h.N[a] = (int)sz.N[a];
        h.g[a] = sch->gravity[a];
    }
    h.h = mesh->h;
    h.inv_h = 1.0 / mesh->h;
    h.ghost = sz.ghost;
    h.nn = sz.nn;
    h.nkeys = sz.nkeys;
    h.nbricks = sz.nbricks;
    h.np = np;
    h.max_items = sz.max_items;
    h.model = mat->model;
    h.sort_always = sch->sort_policy == MPMX_SORT_ALWAYS;
    const double E = mat->E, nu = mat->nu;
    h.G = E / (2.0 * (1.0 + nu));
    h.K = E / (3.0 * (1.0 - 2.0 * nu));
    h.lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    if (mat->model == MPMX_DRUCKER_PRAGER) {
        double eta, xi, etab;
        dp_constants(mat, eta, xi, etab);
        h.eta = eta;
        h.xic = xi * mat->c;
        h.etab = etab;
        h.has_apex = eta > 0.0;
        h.inv_hard = 1.0 / (h.G + h.K * eta * etab);
        h.apex_p = eta > 0.0 ? xi * mat->c / eta : 0.0;
    }
    h.algo = sch->algo;
    h.shape = sch->shape;
    h.vel_update = sch->velocity_update;
    h.prec = sch->precision;
    h.dt = sch->dt;
    uint32_t fb = 0;
    for (int f = 0; f < 6; ++f)
        fb |= (uint32_t)bc->face[f] << (2 * f);
    h.face_bits = fb;

    // particles: host inputs are staged through device memory
    const double *dx = parts->x, *dv = parts->v, *dsig = parts->stress, *dvol = parts->vol, *dmass = parts->mass;
    if (np > 0 && parts->mem == MPMX_MEM_HOST) {
        double mean = 0.0;
        for (int64_t p = 0; p < np; ++p)
            mean += parts->mass[p];
        h.eps_m = sch->mass_eps_rel * (mean / (double)np);
        uint8_t *stage = (uint8_t *)staging(ctx, align_up(24 * np) * 2 + align_up(48 * np) + 2 * align_up(8 * np));
        if (!stage)
            ok = false;
        uint64_t soff = 0;
        auto up = [&](const double *src, size_t count) -> const double * {
            if (!src || !ok)
                return nullptr;
            void *p = stage + soff;
            soff += align_up(count * 8);
            if (hipMemcpy(p, src, count * 8, hipMemcpyHostToDevice) != hipSuccess)
                ok = false;
            return (const double *)p;
        };
        dx = up(parts->x, 3 * np);
        dv = up(parts->v, 3 * np);
        dsig = up(parts->stress, 6 * np);
        dvol = up(parts->vol, np);
        dmass = up(parts->mass, np);
    } else if (np > 0) {
        std::vector<double> m(np);
        if (hipMemcpy(m.data(), parts->mass, 8 * np, hipMemcpyDeviceToHost) != hipSuccess)
            ok = false;
        double mean = 0.0;
        for (int64_t p = 0; p < np; ++p)
            mean += m[p];
        h.eps_m = sch->mass_eps_rel * (mean / (double)np);
    }
    h.f_dt = (float)h.dt;
    h.f_inv_h = (float)h.inv_h;
    for (int e = 0; e < 3; ++e)
        h.f_g[e] = (float)h.g[e];
    h.f_lam = (float)h.lam;
    h.f_G = (float)h.G;
    h.f_K = (float)h.K;
    h.f_eta = (float)h.eta;
    h.f_xic = (float)h.xic;
    h.f_etab = (float)h.etab;
    h.f_apex = (float)h.apex_p;
    h.f_inv_hard = (float)h.inv_hard;
    uint32_t ctl[CTL_WORDS] = {0};
    ctl[CTL_NEED_SORT] = 1;
    ctl[CTL_ALGO] = (uint32_t)h.algo;
    if (ok && hipMemcpy(h.ctl, ctl, sizeof ctl, hipMemcpyHostToDevice) != hipSuccess)
        ok = false;
    if (ok && hipMemcpy(s->d, &h, sizeof(SceneDev), hipMemcpyHostToDevice) != hipSuccess)
        ok = false;
    if (ok && np > 0) {
        const KernelSet &K = kernel_set(s->prec, s->shape);
        SceneDev *d = s->d;
        void *args[] = {&d, &dx, &dv, &dsig, &dvol, &dmass};
        if (hipLaunchKernel(K.load, particle_grid(np), dim3(kParticleBlock), args, 0, ctx->aux) != hipSuccess)
            ok = false;
    }
    if (ok && hipStreamSynchronize(ctx->aux) != hipSuccess)
        ok = false;
    if (!ok) {
        free_scene(ctx, s);
        return fail(ctx, MPMX_E_HIP, "scene upload failed");
    }
    if (hipMemcpy(ctl, h.ctl, sizeof ctl, hipMemcpyDeviceToHost) != hipSuccess) {
        free_scene(ctx, s);
        return fail(ctx, MPMX_E_HIP, "scene status read failed");
    }
    if (ctl[CTL_ERR]) {
        free_scene(ctx, s);
        return fail(ctx, err_code(ctl[CTL_ERR]), "input particle outside the mesh or not finite (bits %u)",
                    ctl[CTL_ERR]);
    }
    std::vector<Scene *> one{s};
    rc = build_batch(ctx, s->single, one);
    if (rc) {
        free_scene(ctx, s);
        return rc;
    }
    s->id = ctx->next_id++;
    s->single.ids.assign(1, s->id);
    *scene_out = s->id;
    ctx->scenes[s->id] = std::move(sc);
    return MPMX_OK;
}

int mpmx_scene_step(mpmx_ctx *ctx, uint64_t scene, int64_t nsteps)
{
    if (!ctx)
        return MPMX_E_INVALID_ARG;
    Scene *s = find(ctx, scene);
    if (!s)
        return fail(ctx, MPMX_E_NOT_FOUND, "unknown scene %llu", (unsigned long long)scene);
    if (nsteps < 0)
        return fail(ctx, MPMX_E_INVALID_ARG, "nsteps must be >= 0");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    return run_steps(ctx, s->single, nullptr, nsteps);
}

int mpmx_batch_step(mpmx_ctx *ctx, const uint64_t *scenes, const int64_t *nsteps, int n)
{
    if (!ctx || n < 0 || (n > 0 && (!scenes || !nsteps)))
        return MPMX_E_INVALID_ARG;
    if (n == 0)
        return MPMX_OK;
    std::vector<Scene *> list;
    std::vector<uint64_t> ids(scenes, scenes + n);
    for (int i = 0; i < n; ++i) {
        Scene *s = find(ctx, scenes[i]);
        if (!s)
            return fail(ctx, MPMX_E_NOT_FOUND, "unknown scene %llu", (unsigned long long)scenes[i]);
        if (nsteps[i] < 0)
            return fail(ctx, MPMX_E_INVALID_ARG, "nsteps[%d] < 0", i);
        if (std::find(list.begin(), list.end(), s) != list.end())
            return fail(ctx, MPMX_E_INVALID_ARG, "scene %llu listed twice", (unsigned long long)scenes[i]);
        if (!list.empty() && (s->prec != list[0]->prec || s->shape != list[0]->shape || s->algo != list[0]->algo))
            return fail(ctx, MPMX_E_INVALID_ARG, "batched scenes must share precision, shape and algorithm");
        list.push_back(s);
    }
    HIPCHK(ctx, hipSetDevice(ctx->device));
    // the two most recent batches stay built: a caller alternating between
    // batch compositions (the request loop) rebuilds the older one, whose
    // image its queued steps have most likely finished reading
    const uint64_t call = ++ctx->batch_calls;
    int slot = ctx->cached_batch[0].ids == ids ? 0 : (ctx->cached_batch[1].ids == ids ? 1 : -1);
    if (slot < 0) {
        slot = ctx->cached_batch[0].used_at <= ctx->cached_batch[1].used_at ? 0 : 1;
        int rc = build_batch(ctx, ctx->cached_batch[slot], list);
        if (rc)
            return rc;
    }
    ctx->cached_batch[slot].used_at = call;
    return run_steps(ctx, ctx->cached_batch[slot], nsteps, 0);
}

int mpmx_batch_step_noalloc(mpmx_ctx *ctx, const uint64_t *scenes, const int64_t *nsteps, int n)
{
    if (!ctx || n < 0 || (n > 0 && (!scenes || !nsteps)))
        return MPMX_E_INVALID_ARG;
    if (n == 0)
        return MPMX_OK;
    if (n > kNoAllocMaxScenes)
        return fail(ctx, MPMX_E_INVALID_ARG, "allocation-free batch: %d scenes, at most %d", n, kNoAllocMaxScenes);
    const uint64_t stamp = ++ctx->scratch_calls;
    Scene *first = nullptr;
    int64_t nbr = 0, np = 0, smax = 0;
    for (int i = 0; i < n; ++i) {
        auto it = ctx->scenes.find(scenes[i]);
        if (it == ctx->scenes.end())
            return fail(ctx, MPMX_E_NOT_FOUND, "unknown scene %llu", (unsigned long long)scenes[i]);
        Scene *s = it->second.get();
        if (nsteps[i] < 0)
            return fail(ctx, MPMX_E_INVALID_ARG, "nsteps[%d] < 0", i);
        if (s->stamp == stamp)
            return fail(ctx, MPMX_E_INVALID_ARG, "scene %llu listed twice", (unsigned long long)scenes[i]);
        s->stamp = stamp;
        if (first && (s->prec != first->prec || s->shape != first->shape || s->algo != first->algo))
            return fail(ctx, MPMX_E_INVALID_ARG, "batched scenes must share precision, shape and algorithm");
        if (!first)
            first = s;
        nbr += s->h.nbricks;
        np += s->h.np;
        smax = std::max(smax, nsteps[i]);
    }
    // the layout of mpmx_batch_step's block, inside the scratch array
    const size_t n1 = (size_t)n + 1, n8 = 8 * (size_t)n;
    const size_t o_po = n8, o_bo = o_po + 8 * n1, o_ns = o_bo + 8 * n1, o_ct = o_ns + n8, o_io = o_ct + n8,
                 o_co = o_io + 4 * n1, o_fl = (o_co + 4 * n1 + 127) & ~(size_t)127, o_sc = o_fl + 4 * BF_WORDS,
                 o_br = o_sc + 16 * (size_t)kScanChunks, total = o_br + 4 * (size_t)std::max<int64_t>(nbr, 1);
    if (total > kScratchBytes)
        return fail(ctx, MPMX_E_INVALID_ARG,
                    "allocation-free batch: %lld bricks need %zu bytes of scratch, at most %zu (about %zu bricks)",
                    (long long)nbr, total, kScratchBytes, (kScratchBytes - o_br) / 4);
    if (smax == 0)
        return MPMX_OK;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    // the part the host writes: scene descriptors, particle and brick
    // offsets, step counts, control blocks (the flags are cleared by the
    // first kernel, the rest is written by the kernels)
    uint8_t *img = ctx->scratch_img.data();
    SceneDev **sp = (SceneDev **)img;
    int64_t *po = (int64_t *)(img + o_po), *bo = (int64_t *)(img + o_bo), *ns = (int64_t *)(img + o_ns);
    uint32_t **cp = (uint32_t **)(img + o_ct);
    po[0] = bo[0] = 0;
    for (int i = 0; i < n; ++i) {
        Scene *s = ctx->scenes.find(scenes[i])->second.get();
        sp[i] = s->d;
        cp[i] = s->h.ctl;
        ns[i] = nsteps[i];
        po[i + 1] = po[i] + s->h.np;
        bo[i + 1] = bo[i] + s->h.nbricks;
    }
    uint8_t *base = (uint8_t *)ctx->scratch;
    HIPCHK(ctx, hipMemcpyAsync(base, img, o_io, hipMemcpyHostToDevice, ctx->stream));
    Batch b;
    b.bd.scenes = (SceneDev **)base;
    b.bd.ctls = (uint32_t *const *)(base + o_ct);
    b.bd.poffs = (const int64_t *)(base + o_po);
    b.bd.boffs = (const int64_t *)(base + o_bo);
    b.bd.ioffs = (uint32_t *)(base + o_io);
    b.bd.coffs = (uint32_t *)(base + o_co);
    b.bd.flags = (uint32_t *)(base + o_fl);
    b.bd.scan = (uint32_t *)(base + o_sc);
    b.bd.bricks = (uint32_t *)(base + o_br);
    b.bd.nscenes = n;
    b.bd.total_particles = np;
    b.bd.total_bricks = nbr;
    int64_t maxit = 0;
    for (int i = 0; i < n; ++i)
        maxit += ctx->scenes.find(scenes[i])->second->h.max_items;
    b.bd.max_items = maxit;
    b.prec = first->prec;
    b.shape = first->shape;
    b.algo = first->algo;
    // a launch shape the context already tuned for this layout, else the
    // fixed one; no tuning, no graphs, no per-launch events
    LaunchCfg cfg = ctx->fixed;
    if (ctx->autotune) {
        auto it = ctx->tuned.find(layout_key(b));
        if (it != ctx->tuned.end())
            cfg = it->second;
    }
    const bool prof = ctx->prof.on;
    ctx->prof.on = false;
    ctx->launch_stream = nullptr;
    BatchDev bd = b.bd;
    const int64_t *dns = (const int64_t *)(base + o_ns);
    void *a_begin[] = {&bd, &dns};
    int rc = launch(ctx, "begin", common_kernels().begin, dim3(1), dim3(1024), a_begin);
    for (int64_t k = 0; k < smax && !rc; ++k)
        rc = enqueue_step(ctx, b, cfg, k == 0, nullptr);
    ctx->prof.on = prof;
    // no event (that would allocate): reading or freeing these scenes waits
    // for the whole context stream
    for (int i = 0; i < n; ++i)
        ctx->scenes.find(scenes[i])->second->main_sync = true;
    if (!rc)
        ctx->last = cfg;
    return rc;
}

int mpmx_scene_read(mpmx_ctx *ctx, uint64_t scene, const mpmx_particles_out *out)
{
    if (!ctx || !out || out->size < sizeof(mpmx_particles_out) ||
        (out->mem != MPMX_MEM_HOST && out->mem != MPMX_MEM_DEVICE))
        return MPMX_E_INVALID_ARG;
    Scene *s = find(ctx, scene);
    if (!s)
        return fail(ctx, MPMX_E_NOT_FOUND, "unknown scene %llu", (unsigned long long)scene);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    // the read runs on the second stream once the scene's own queued steps
    // are done; later steps of other scenes keep running meanwhile
    int rc = wait_for_scene(ctx, s, ctx->aux);
    if (rc)
        return rc;
    const int64_t np = s->h.np;
    if (np > 0) {
        double *x = out->x, *v = out->v, *sg = out->stress, *vol = out->vol;
        int32_t *cell = out->cell;
        uint8_t *stage = nullptr;
        if (out->mem == MPMX_MEM_HOST)
            stage = (uint8_t *)staging(ctx, 2 * align_up(24 * np) + align_up(48 * np) + align_up(8 * np) +
                                                align_up(4 * np));
        uint64_t soff = 0;
        auto dev = [&](void *host, size_t bytes) -> void * {
            if (!host || out->mem == MPMX_MEM_DEVICE)
                return host;
            if (!stage)
                return nullptr;
            void *p = stage + soff;
            soff += align_up(bytes);
            return p;
        };
        double *dx = (double *)dev(x, 24 * np), *dv = (double *)dev(v, 24 * np);
        double *ds = (double *)dev(sg, 48 * np), *dvo = (double *)dev(vol, 8 * np);
        int32_t *dc = (int32_t *)dev(cell, 4 * np);
        bool ok = (!x || dx) && (!v || dv) && (!sg || ds) && (!vol || dvo) && (!cell || dc);
        const KernelSet &K = kernel_set(s->prec, s->shape);
        SceneDev *d = s->d;
        void *args[] = {&d, &dx, &dv, &ds, &dvo, &dc};
        if (ok && hipLaunchKernel(K.read_out, particle_grid(np), dim3(kParticleBlock), args, 0, ctx->aux) !=
                      hipSuccess)
            ok = false;
        if (ok && hipStreamSynchronize(ctx->aux) != hipSuccess)
            ok = false;
        if (ok && out->mem == MPMX_MEM_HOST) {
            if (x && hipMemcpy(x, dx, 24 * np, hipMemcpyDeviceToHost) != hipSuccess) ok = false;
            if (v && hipMemcpy(v, dv, 24 * np, hipMemcpyDeviceToHost) != hipSuccess) ok = false;
            if (sg && hipMemcpy(sg, ds, 48 * np, hipMemcpyDeviceToHost) != hipSuccess) ok = false;
            if (vol && hipMemcpy(vol, dvo, 8 * np, hipMemcpyDeviceToHost) != hipSuccess) ok = false;
            if (cell && hipMemcpy(cell, dc, 4 * np, hipMemcpyDeviceToHost) != hipSuccess) ok = false;
        }
        if (!ok)
            return fail(ctx, MPMX_E_HIP, "particle read failed");
    }
    HIPCHK(ctx, hipStreamSynchronize(ctx->aux));
    uint32_t ctl[CTL_WORDS];
    HIPCHK(ctx, hipMemcpy(ctl, s->h.ctl, sizeof(uint32_t) * CTL_WORDS, hipMemcpyDeviceToHost));
    if (ctl[CTL_ERR])
        return fail(ctx, err_code(ctl[CTL_ERR]), "scene stopped on error bits %u", ctl[CTL_ERR]);
    return MPMX_OK;
}

int mpmx_scene_cell_counts(mpmx_ctx *ctx, uint64_t scene, uint32_t *counts, int32_t mem)
{
    if (!ctx || !counts || (mem != MPMX_MEM_HOST && mem != MPMX_MEM_DEVICE))
        return MPMX_E_INVALID_ARG;
    Scene *s = find(ctx, scene);
    if (!s)
        return fail(ctx, MPMX_E_NOT_FOUND, "unknown scene %llu", (unsigned long long)scene);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const int64_t nc = (int64_t)s->h.n[0] * s->h.n[1] * s->h.n[2];
    uint32_t *d = counts;
    if (mem == MPMX_MEM_HOST)
        HIPCHK(ctx, hipMalloc(&d, 4 * nc));
    HIPCHK(ctx, hipMemsetAsync(d, 0, 4 * nc, ctx->stream));
    SceneDev *sd = s->d;
    void *args[] = {&sd, &d};
    hipError_t e = hipSuccess;
    if (s->h.np > 0)
        e = hipLaunchKernel(common_kernels().cell_counts, particle_grid(s->h.np), dim3(kParticleBlock), args, 0,
                            ctx->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess && mem == MPMX_MEM_HOST)
        e = hipMemcpy(counts, d, 4 * nc, hipMemcpyDeviceToHost);
    if (mem == MPMX_MEM_HOST)
        (void)hipFree(d);
    if (e != hipSuccess)
        return fail(ctx, MPMX_E_HIP, "cell counts: %s", hipGetErrorString(e));
    return MPMX_OK;
}

int mpmx_scene_nodes(mpmx_ctx *ctx, uint64_t scene, double *mass, double *momentum, double *force)
{
    if (!ctx)
        return MPMX_E_INVALID_ARG;
    Scene *s = find(ctx, scene);
    if (!s)
        return fail(ctx, MPMX_E_NOT_FOUND, "unknown scene %llu", (unsigned long long)scene);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const int64_t nn = s->h.nn;
    double *dm = nullptr, *dp = nullptr, *df = nullptr;
    if (mass)
        HIPCHK(ctx, hipMalloc(&dm, 8 * nn));
    if (momentum)
        HIPCHK(ctx, hipMalloc(&dp, 24 * nn));
    if (force)
        HIPCHK(ctx, hipMalloc(&df, 24 * nn));
    SceneDev *sd = s->d;
    void *args[] = {&sd, &dm, &dp, &df};
    hipError_t e = hipLaunchKernel(kernel_set(s->prec, s->shape).nodes_out, particle_grid(nn), dim3(kParticleBlock),
                                   args, 0, ctx->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess && mass)
        e = hipMemcpy(mass, dm, 8 * nn, hipMemcpyDeviceToHost);
    if (e == hipSuccess && momentum)
        e = hipMemcpy(momentum, dp, 24 * nn, hipMemcpyDeviceToHost);
    if (e == hipSuccess && force)
        e = hipMemcpy(force, df, 24 * nn, hipMemcpyDeviceToHost);
    if (dm) (void)hipFree(dm);
    if (dp) (void)hipFree(dp);
    if (df) (void)hipFree(df);
    if (e != hipSuccess)
        return fail(ctx, MPMX_E_HIP, "node read: %s", hipGetErrorString(e));
    return MPMX_OK;
}

int mpmx_scene_stats(mpmx_ctx *ctx, uint64_t scene, mpmx_stats *out)
{
    if (!ctx || !out || out->size < sizeof(mpmx_stats))
        return MPMX_E_INVALID_ARG;
    Scene *s = find(ctx, scene);
    if (!s)
        return fail(ctx, MPMX_E_NOT_FOUND, "unknown scene %llu", (unsigned long long)scene);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    uint32_t ctl[CTL_WORDS];
    int rc = read_ctl(ctx, s, ctl);
    if (rc)
        return rc;
    const int64_t nc = (int64_t)s->h.n[0] * s->h.n[1] * s->h.n[2];
    std::vector<uint32_t> counts(nc);
    rc = mpmx_scene_cell_counts(ctx, scene, counts.data(), MPMX_MEM_HOST);
    if (rc)
        return rc;
    int64_t active = 0;
    uint64_t hash = 14695981039346656037ull;   // FNV-1a over (cell, count) of the occupied cells
    for (int64_t c = 0; c < nc; ++c)
        if (counts[c] > 0) {
            ++active;
            hash = (hash ^ (uint64_t)c) * 1099511628211ull;
            hash = (hash ^ (uint64_t)counts[c]) * 1099511628211ull;
        }
    out->n_particles = s->h.np;
    out->pic_hash = hash;
    out->lost_particles = ctl[CTL_LOST];
    out->steps_done = ctl[CTL_STEPS];
    out->n_sorts = ctl[CTL_N_SORTS];
    out->n_items = ctl[CTL_N_ITEMS];
    out->active_cells = active;
    out->error_bits = ctl[CTL_ERR];
    out->device_bytes = s->bytes;
    return MPMX_OK;
}

int mpmx_fence_record(mpmx_ctx *ctx, uint64_t *fence)
{
    if (!ctx || !fence)
        return MPMX_E_INVALID_ARG;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipEvent_t e = nullptr;
    HIPCHK(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    const hipError_t r = hipEventRecord(e, ctx->stream);
    if (r != hipSuccess) {
        (void)hipEventDestroy(e);
        return fail(ctx, MPMX_E_HIP, "fence record: %s", hipGetErrorString(r));
    }
    *fence = ctx->next_fence++;
    ctx->fences[*fence] = e;
    return MPMX_OK;
}

int mpmx_fence_wait(mpmx_ctx *ctx, uint64_t fence, int block, int *done)
{
    if (!ctx || !done)
        return MPMX_E_INVALID_ARG;
    auto it = ctx->fences.find(fence);
    if (it == ctx->fences.end())
        return fail(ctx, MPMX_E_NOT_FOUND, "unknown fence %llu", (unsigned long long)fence);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    if (block) {
        HIPCHK(ctx, hipEventSynchronize(it->second));
    } else {
        const hipError_t r = hipEventQuery(it->second);
        if (r == hipErrorNotReady) {
            *done = 0;
            return MPMX_OK;
        }
        if (r != hipSuccess)
            return fail(ctx, MPMX_E_HIP, "fence query: %s", hipGetErrorString(r));
    }
    (void)hipEventDestroy(it->second);
    ctx->fences.erase(it);
    *done = 1;
    return MPMX_OK;
}

int mpmx_fence_release(mpmx_ctx *ctx, uint64_t fence)
{
    if (!ctx)
        return MPMX_E_INVALID_ARG;
    auto it = ctx->fences.find(fence);
    if (it == ctx->fences.end())
        return fail(ctx, MPMX_E_NOT_FOUND, "unknown fence %llu", (unsigned long long)fence);
    (void)hipEventDestroy(it->second);
    ctx->fences.erase(it);
    return MPMX_OK;
}

int mpmx_scene_destroy(mpmx_ctx *ctx, uint64_t scene)
{
    if (!ctx)
        return MPMX_E_INVALID_ARG;
    auto it = ctx->scenes.find(scene);
    if (it == ctx->scenes.end())
        return fail(ctx, MPMX_E_NOT_FOUND, "unknown scene %llu", (unsigned long long)scene);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    // its own queued steps, and reads of its buffers on the second stream
    int rc = host_wait_for_scene(ctx, it->second.get());
    if (rc)
        return rc;
    HIPCHK(ctx, hipStreamSynchronize(ctx->aux));
    for (auto &cb : ctx->cached_batch)
        if (std::find(cb.ids.begin(), cb.ids.end(), scene) != cb.ids.end()) {
            // keep the image until its queued steps are done (a rebuild waits)
            cb.drop_graph();
            cb.ids.clear();
        }
    free_scene(ctx, it->second.get());
    ctx->scenes.erase(it);
    return MPMX_OK;
}

}  // extern "C"
