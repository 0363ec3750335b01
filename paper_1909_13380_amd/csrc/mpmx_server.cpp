// mpmx_server.cpp -- request loop of libmpmx (mpmx_server_* in include/mpmx.h).
//
// Built only on the public C ABI: a request becomes a scene when it is
// admitted, resident scenes advance together through mpmx_batch_step (one
// launch per stage for each precision / shape / algorithm group), and a
// finished scene is read back to host memory and freed.  Admission is in
// arrival order against a device-memory budget, so a large request at the
// head of the queue is never overtaken by later small ones.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <tuple>
#include <vector>

#include "mpmx.h"

namespace {

struct Pending {
    uint64_t id = 0, tag = 0;
    int64_t nsteps = 0, n = 0;
    double t_submit = 0.0;
    uint64_t bytes = 0;
    mpmx_mesh mesh{};
    mpmx_material mat{};
    mpmx_bc bc{};
    mpmx_scheme sch{};
    std::vector<int64_t> bc_node;
    std::vector<int32_t> bc_axis;
    std::vector<double> bc_value;
    std::vector<int64_t> force_node;
    std::vector<double> force_value;
    std::vector<double> node_x;   // isoparametric mesh nodes (empty: uniform)
    std::vector<double> x, v, stress, vol, mass;
    mpmx_particles borrowed{};    // MPMX_REQ_BORROW: the caller's arrays
    bool borrow = false;
    mpmx_particles_out out{};     // caller's output buffers (out.size == 0: none)
};

struct Resident {
    uint64_t id = 0, tag = 0, scene = 0, bytes = 0;
    int64_t n = 0, nsteps = 0, remaining = 0;
    double t_submit = 0.0, t_admit = 0.0;
    std::tuple<int, int, int> group;
    mpmx_particles_out out{};     // caller's output buffers (out.size == 0: none)
};

struct Done {
    mpmx_completion c{};
    std::unique_ptr<double[]> x, v, stress, vol;   // unless the request gave output buffers
};

// Device bytes a request occupies once admitted.
int request_bytes(const mpmx_mesh *mesh, const mpmx_scheme *sch, const mpmx_bc *bc, int64_t n, uint64_t *out)
{
    int rc = mpmx_scene_bytes(mesh, sch, n, out);
    if (rc)
        return rc;
    if (bc->n_extra > 0 || bc->n_force > 0) {
        const int g = sch->shape == MPMX_SHAPE_GIMP ? 1 : 0;
        uint64_t nn = 1;
        for (int a = 0; a < 3; ++a)
            nn *= (uint64_t)(mesh->n[a] + 1 + 2 * g);
        *out += ((nn + 255) & ~uint64_t(255)) + ((24 * nn + 255) & ~uint64_t(255));
        if (bc->n_force > 0)
            *out += (24 * nn + 255) & ~uint64_t(255);
    }
    return MPMX_OK;
}

}  // namespace

struct mpmx_server {
    mpmx_ctx *ctx = nullptr;
    uint64_t budget = 0, used = 0;
    int64_t max_tick = 0;
    int64_t fill = 0;                    // admission stops at this many active particles (0: off)
    uint64_t next_id = 1;
    std::chrono::steady_clock::time_point t0;
    std::deque<Pending> queue;
    std::vector<Resident> resident;      // scenes with steps still to queue
    struct Round {
        uint64_t fence = 0;              // after the round's steps
        std::vector<Resident> last;      // scenes whose last steps the round queued
    };
    std::deque<Round> rounds;            // queued rounds not yet known finished, oldest first
    std::deque<uint64_t> ready;          // completed, not yet polled
    std::map<uint64_t, Done> done;       // completed, not yet released
    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

// Shortest tick: finishing scenes wait for at most this many steps of the
// others, which keeps ticks (each of which synchronises) from shrinking to
// single steps when completions are close together.
constexpr int64_t kMinTickSteps = 16;

// Rounds the host may keep queued ahead of the GPU: enough that the GPU
// never waits for the host between rounds, few enough that a request
// arriving now joins the batch within a couple of rounds.
constexpr size_t kMaxAhead = 2;

int finish(mpmx_server *srv, Resident &r)
{
    Done d;
    const size_t n = (size_t)r.n;
    mpmx_particles_out out = r.out;
    if (!out.size) {   // the server's own arrays (never zero-filled: the read writes every element)
        d.x.reset(new (std::nothrow) double[3 * n]);
        d.v.reset(new (std::nothrow) double[3 * n]);
        d.stress.reset(new (std::nothrow) double[6 * n]);
        d.vol.reset(new (std::nothrow) double[n]);
        if (n && (!d.x || !d.v || !d.stress || !d.vol)) {
            // no host memory for the result: free the scene and report it
            if (int rc = mpmx_scene_destroy(srv->ctx, r.scene))
                return rc;
            srv->used -= r.bytes;
            Done f;
            f.c.size = sizeof(mpmx_completion);
            f.c.status = MPMX_E_OOM;
            f.c.request = r.id;
            f.c.tag = r.tag;
            f.c.n = r.n;
            f.c.t_submit = r.t_submit;
            f.c.t_admit = r.t_admit;
            f.c.t_done = srv->now();
            srv->ready.push_back(r.id);
            srv->done[r.id] = std::move(f);
            return MPMX_OK;
        }
        out.size = sizeof out;
        out.mem = MPMX_MEM_HOST;
        out.x = d.x.get();
        out.v = d.v.get();
        out.stress = d.stress.get();
        out.vol = d.vol.get();
    }
    const int status = mpmx_scene_read(srv->ctx, r.scene, &out);
    if (status == MPMX_E_HIP || status == MPMX_E_INVALID_ARG || status == MPMX_E_NOT_FOUND)
        return status;
    mpmx_stats st{};
    st.size = sizeof st;
    int64_t steps = r.nsteps;
    if (status != MPMX_OK && mpmx_scene_stats(srv->ctx, r.scene, &st) == MPMX_OK)
        steps = st.steps_done;
    int rc = mpmx_scene_destroy(srv->ctx, r.scene);
    if (rc)
        return rc;
    srv->used -= r.bytes;
    d.c.size = sizeof(mpmx_completion);
    d.c.status = status;
    d.c.request = r.id;
    d.c.tag = r.tag;
    d.c.n = r.n;
    d.c.steps_done = steps;
    d.c.t_submit = r.t_submit;
    d.c.t_admit = r.t_admit;
    d.c.t_done = srv->now();
    d.c.x = out.x;
    d.c.v = out.v;
    d.c.stress = out.stress;
    d.c.vol = out.vol;
    srv->ready.push_back(r.id);
    srv->done[r.id] = std::move(d);
    return MPMX_OK;
}

// Admit from the head of the queue while the next request fits the budget
// and the scenes still stepping hold fewer particles than the fill limit.
int admit(mpmx_server *srv)
{
    int64_t active = 0;
    for (const auto &r : srv->resident)
        active += r.n;
    while (!srv->queue.empty()) {
        Pending &p = srv->queue.front();
        if (srv->used + p.bytes > srv->budget)
            break;
        if (srv->fill > 0 && !srv->resident.empty() && active >= srv->fill)
            break;
        mpmx_particles parts{};
        if (p.borrow) {
            parts = p.borrowed;
        } else {
            parts.size = sizeof parts;
            parts.mem = MPMX_MEM_HOST;
            parts.n = p.n;
            parts.x = p.x.data();
            parts.v = p.v.data();
            parts.stress = p.stress.empty() ? nullptr : p.stress.data();
            parts.vol = p.vol.data();
            parts.mass = p.mass.data();
        }
        p.bc.node = p.bc_node.data();
        p.bc.axis = p.bc_axis.data();
        p.bc.value = p.bc_value.data();
        p.bc.force_node = p.force_node.data();
        p.bc.force_value = p.force_value.data();
        p.mesh.node_x = p.node_x.empty() ? nullptr : p.node_x.data();
        uint64_t scene = 0;
        const int rc = mpmx_scene_create(srv->ctx, &p.mesh, &p.mat, &p.bc, &p.sch, &parts, &scene);
        if (rc == MPMX_E_OOM || rc == MPMX_E_HIP)
            return rc;   // stays queued; the caller sees the failure
        if (rc != MPMX_OK) {
            // inputs rejected by the library (e.g. a particle outside the
            // mesh): complete at once with that status
            Done d;
            d.c.size = sizeof(mpmx_completion);
            d.c.status = rc;
            d.c.request = p.id;
            d.c.tag = p.tag;
            d.c.n = p.n;
            d.c.t_submit = p.t_submit;
            d.c.t_admit = d.c.t_done = srv->now();
            srv->ready.push_back(p.id);
            srv->done[p.id] = std::move(d);
            srv->queue.pop_front();
            continue;
        }
        Resident r;
        r.id = p.id;
        r.tag = p.tag;
        r.scene = scene;
        r.bytes = p.bytes;
        r.n = p.n;
        r.nsteps = r.remaining = p.nsteps;
        r.t_submit = p.t_submit;
        r.t_admit = srv->now();
        r.group = std::make_tuple(p.sch.precision, p.sch.shape, p.sch.algo);
        r.out = p.out;
        srv->used += p.bytes;
        active += p.n;
        srv->resident.push_back(r);
        srv->queue.pop_front();
    }
    return MPMX_OK;
}

}  // namespace

extern "C" {

int mpmx_server_create(mpmx_ctx *ctx, uint64_t budget_bytes, int64_t max_tick_steps, mpmx_server **out)
{
    if (!ctx || !out || budget_bytes == 0 || max_tick_steps < 1)
        return MPMX_E_INVALID_ARG;
    auto *s = new (std::nothrow) mpmx_server();
    if (!s)
        return MPMX_E_OOM;
    s->ctx = ctx;
    s->budget = budget_bytes;
    s->max_tick = max_tick_steps;
    s->t0 = std::chrono::steady_clock::now();
    *out = s;
    return MPMX_OK;
}

int mpmx_server_set_fill(mpmx_server *srv, int64_t particles)
{
    if (!srv || particles < 0)
        return MPMX_E_INVALID_ARG;
    srv->fill = particles;
    return MPMX_OK;
}

double mpmx_server_clock(const mpmx_server *srv) { return srv ? srv->now() : 0.0; }

int mpmx_server_submit(mpmx_server *srv, const mpmx_request *req, uint64_t *id)
{
    if (!srv || !req || !id || req->size < sizeof(mpmx_request) || !req->mesh || !req->material || !req->bc ||
        !req->scheme || !req->particles || req->nsteps < 0)
        return MPMX_E_INVALID_ARG;
    const mpmx_particles *pp = req->particles;
    if (pp->size < sizeof(mpmx_particles) || pp->mem != MPMX_MEM_HOST || pp->n < 0 ||
        (pp->n > 0 && (!pp->x || !pp->v || !pp->vol || !pp->mass)))
        return MPMX_E_INVALID_ARG;
    if (req->mesh->size < sizeof(mpmx_mesh) || req->material->size < sizeof(mpmx_material) ||
        req->bc->size < sizeof(mpmx_bc) || req->scheme->size < sizeof(mpmx_scheme))
        return MPMX_E_INVALID_ARG;
    if (req->bc->n_extra < 0 || (req->bc->n_extra > 0 && (!req->bc->node || !req->bc->axis || !req->bc->value)))
        return MPMX_E_INVALID_ARG;
    if (req->bc->n_force < 0 || (req->bc->n_force > 0 && (!req->bc->force_node || !req->bc->force_value)))
        return MPMX_E_INVALID_ARG;
    if ((req->flags & ~(uint32_t)MPMX_REQ_BORROW) != 0)
        return MPMX_E_INVALID_ARG;
    const mpmx_particles_out *o = req->out;
    if (o && (o->size < sizeof(mpmx_particles_out) || o->mem != MPMX_MEM_HOST ||
              (pp->n > 0 && (!o->x || !o->v || !o->stress || !o->vol))))
        return MPMX_E_INVALID_ARG;
    uint64_t bytes = 0;
    int rc = request_bytes(req->mesh, req->scheme, req->bc, pp->n, &bytes);
    if (rc)
        return rc;
    if (bytes > srv->budget)
        return MPMX_E_BUDGET;
    Pending p;
    p.id = srv->next_id++;
    p.tag = req->tag;
    p.nsteps = req->nsteps;
    p.n = pp->n;
    p.bytes = bytes;
    p.t_submit = srv->now();
    p.mesh = *req->mesh;
    if (req->mesh->node_x) {
        const size_t nn = (size_t)(req->mesh->n[0] + 1) * (req->mesh->n[1] + 1) * (req->mesh->n[2] + 1);
        p.node_x.assign(req->mesh->node_x, req->mesh->node_x + 3 * nn);
    }
    p.mat = *req->material;
    p.bc = *req->bc;
    p.sch = *req->scheme;
    const size_t ne = (size_t)req->bc->n_extra;
    p.bc_node.assign(req->bc->node, req->bc->node + ne);
    p.bc_axis.assign(req->bc->axis, req->bc->axis + ne);
    p.bc_value.assign(req->bc->value, req->bc->value + ne);
    const size_t nf = (size_t)req->bc->n_force;
    p.force_node.assign(req->bc->force_node, req->bc->force_node + nf);
    p.force_value.assign(req->bc->force_value, req->bc->force_value + 3 * nf);
    const size_t n = (size_t)pp->n;
    if (req->flags & MPMX_REQ_BORROW) {
        p.borrow = true;
        p.borrowed = *pp;
        p.borrowed.size = sizeof(mpmx_particles);
    } else {
        p.x.assign(pp->x, pp->x + 3 * n);
        p.v.assign(pp->v, pp->v + 3 * n);
        if (pp->stress)
            p.stress.assign(pp->stress, pp->stress + 6 * n);
        p.vol.assign(pp->vol, pp->vol + n);
        p.mass.assign(pp->mass, pp->mass + n);
    }
    if (o)
        p.out = *o;
    srv->queue.push_back(std::move(p));
    *id = srv->queue.back().id;
    return MPMX_OK;
}

int mpmx_server_tick(mpmx_server *srv, int *n_resident, int *n_queued)
{
    if (!srv)
        return MPMX_E_INVALID_ARG;
    // admission uploads on the context's second stream, overlapping the
    // steps already queued
    int rc = admit(srv);
    if (rc)
        return rc;
    // queue this round's steps: every resident scene, as a batch per group,
    // by the steps until the first of them completes (at least
    // kMinTickSteps, at most max_tick)
    int64_t k = srv->max_tick;
    for (auto &r : srv->resident)
        if (r.remaining > 0)
            k = std::min(k, r.remaining);
    k = std::min(std::max(k, kMinTickSteps), srv->max_tick);
    std::map<std::tuple<int, int, int>, std::pair<std::vector<uint64_t>, std::vector<int64_t>>> groups;
    for (auto &r : srv->resident)
        if (r.remaining > 0) {
            auto &g = groups[r.group];
            g.first.push_back(r.scene);
            g.second.push_back(std::min(r.remaining, k));
        }
    // the groups whose steps were queued: a failure part-way leaves the
    // bookkeeping of the queued groups right, then reports the error
    std::vector<std::tuple<int, int, int>> queued;
    int launch_rc = MPMX_OK;
    for (auto &kv : groups) {
        launch_rc = mpmx_batch_step(srv->ctx, kv.second.first.data(), kv.second.second.data(),
                                    (int)kv.second.first.size());
        if (launch_rc)
            break;
        queued.push_back(kv.first);
    }
    {
        mpmx_server::Round round;
        std::vector<Resident> keep;
        for (auto &r : srv->resident) {
            if (r.remaining > 0 && std::find(queued.begin(), queued.end(), r.group) != queued.end())
                r.remaining -= std::min(r.remaining, k);
            (r.remaining == 0 ? round.last : keep).push_back(r);   // (requests of 0 steps too)
        }
        srv->resident.swap(keep);
        // without a fence (0) the round counts as finished: each read below
        // still waits for its own scene's steps
        if (!queued.empty() && mpmx_fence_record(srv->ctx, &round.fence) != MPMX_OK)
            round.fence = 0;
        if (!queued.empty() || !round.last.empty())
            srv->rounds.push_back(std::move(round));
    }
    if (launch_rc)
        return launch_rc;
    // finish rounds oldest first: those already finished, after waiting for
    // the oldest while more than kMaxAhead are queued or when this round
    // queued nothing
    bool wait = queued.empty();
    while (!srv->rounds.empty()) {
        const bool block = wait || srv->rounds.size() > kMaxAhead;
        int done = 1;
        if (srv->rounds.front().fence &&
            (rc = mpmx_fence_wait(srv->ctx, srv->rounds.front().fence, block ? 1 : 0, &done)))
            return rc;
        if (!done)
            break;
        wait = false;
        mpmx_server::Round round = std::move(srv->rounds.front());
        srv->rounds.pop_front();
        for (auto &r : round.last)
            if ((rc = finish(srv, r)))
                return rc;
    }
    if (n_resident) {
        size_t waiting = 0;
        for (auto &rd : srv->rounds)
            waiting += rd.last.size();
        *n_resident = (int)(srv->resident.size() + waiting);
    }
    if (n_queued)
        *n_queued = (int)srv->queue.size();
    return MPMX_OK;
}

int mpmx_server_poll(mpmx_server *srv, mpmx_completion *out, int max, int *n)
{
    if (!srv || !n || max < 0 || (max > 0 && !out))
        return MPMX_E_INVALID_ARG;
    int k = 0;
    while (k < max && !srv->ready.empty()) {
        out[k++] = srv->done[srv->ready.front()].c;
        srv->ready.pop_front();
    }
    *n = k;
    return MPMX_OK;
}

int mpmx_server_release(mpmx_server *srv, uint64_t id)
{
    if (!srv)
        return MPMX_E_INVALID_ARG;
    auto it = srv->done.find(id);
    if (it == srv->done.end() ||
        std::find(srv->ready.begin(), srv->ready.end(), id) != srv->ready.end())
        return MPMX_E_NOT_FOUND;
    srv->done.erase(it);
    return MPMX_OK;
}

void mpmx_server_destroy(mpmx_server *srv)
{
    if (!srv)
        return;
    for (auto &r : srv->resident)
        (void)mpmx_scene_destroy(srv->ctx, r.scene);
    for (auto &rd : srv->rounds) {
        for (auto &r : rd.last)
            (void)mpmx_scene_destroy(srv->ctx, r.scene);
        if (rd.fence)
            (void)mpmx_fence_release(srv->ctx, rd.fence);
    }
    delete srv;
}

}  // extern "C"
