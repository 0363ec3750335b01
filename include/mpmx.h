/*
 * mpmx.h -- C ABI of the MI355X (gfx950) explicit material point method step.
 *
 * The calls follow the paper's statement of the problem (Kumar et al.,
 * "Scalable and modular material point method for large-scale simulations",
 * arXiv:1909.13380):
 *   - a background mesh of nodes and cells (code overview: Mesh, Node, Cell;
 *     here a uniform grid of 8-node hexahedra),
 *   - material points carrying position, velocity, stress and volume
 *     (introduction: points carry the state; nodal values are reset every
 *     step),
 *   - a material that returns the stress for a strain increment (code
 *     overview: Material; linear elastic or Drucker-Prager),
 *   - velocity constraints held at nodes (code overview; isoparametric-mesh
 *     section: boundary conditions are applied at the nodes),
 *   - an explicit algorithm, update-stress-first or update-stress-last, and
 *     linear or GIMP shape functions (code overview); beyond the paper, the
 *     modified update-stress-last (MUSL: the strain increment comes from
 *     the updated particle momenta mapped back to the nodes; Sulsky, Zhou
 *     & Schreyer 1995),
 *   - a time step and a step count (benchmark section: 1000 explicit USF
 *     steps);
 * in, and the updated particle state out.
 *
 * Every entry point returns MPMX_OK (0) or a negative MPMX_E_* code; the
 * context keeps a message for the last failure (mpmx_last_error).  A context
 * is used by one host thread at a time.  Work is queued on the context's HIP
 * stream; calls that return data to the caller synchronise that stream.
 *
 * Ownership: every const input is copied before the call returns and stays
 * the caller's.  Scene state lives in device memory owned by the library
 * until mpmx_scene_destroy.  Outputs go to caller-allocated buffers; the
 * library never frees caller memory.  A pointer flagged MPMX_MEM_DEVICE must
 * be device memory of the context's GPU.
 *
 * Conventions: SI units; tension positive; Voigt stress order xx, yy, zz,
 * xy, yz, xz; particle arrays are row-major (n x 3, n x 6); cells are
 * half-open [o + h c, o + h (c + 1)) and numbered c_x + n_x (c_y + n_y c_z);
 * nodes (i, j, k) sit at o + h (i, j, k), numbered
 * (i + g) + N_x ((j + g) + N_y (k + g)) with g = 0 for linear and g = 1 for
 * GIMP shape functions (one ghost layer) and N_a = n_a + 1 + 2 g.
 */
#ifndef MPMX_H
#define MPMX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPMX_VERSION 4

/* ------------------------------------------------------------ codes ---- */
enum {
    MPMX_OK = 0,
    MPMX_E_INVALID_ARG = -1, /* bad pointer, size, enum or descriptor */
    MPMX_E_OOM = -2,         /* device or host allocation failed */
    MPMX_E_BUDGET = -3,      /* the scene can never fit the server budget */
    MPMX_E_OUT_OF_MESH = -4, /* a particle left the mesh; the scene stops */
    MPMX_E_NONFINITE = -5,   /* a non-finite position, velocity or stress */
    MPMX_E_HIP = -6,         /* a HIP runtime call failed */
    MPMX_E_AGAIN = -7,       /* request queued, or nothing to report yet */
    MPMX_E_NOT_FOUND = -8,   /* unknown scene, request or server id */
    MPMX_E_STATE = -9        /* call not valid in the object's state */
};

enum { MPMX_LINEAR_ELASTIC = 0, MPMX_DRUCKER_PRAGER = 1 };
/* Drucker-Prager cone matched to Mohr-Coulomb: through the triaxial
 * compression meridian (outer), the extension meridian (inner), or the
 * plane-strain match. */
enum { MPMX_DP_OUTER = 0, MPMX_DP_INNER = 1, MPMX_DP_PLANE_STRAIN = 2 };
enum { MPMX_BC_FREE = 0, MPMX_BC_FIXED = 1, MPMX_BC_SLIP = 2 };
enum { MPMX_USF = 0, MPMX_USL = 1, MPMX_MUSL = 2 };
enum { MPMX_SHAPE_LINEAR = 0, MPMX_SHAPE_GIMP = 1 };
enum { MPMX_FLIP = 0, MPMX_PIC = 1 };
enum { MPMX_FP32 = 0, MPMX_FP64 = 1 };
/* Particle reordering: keep particles grouped by 4x4x4-cell brick,
 * re-sorting when a particle has moved more than one cell outside the
 * brick of its work item (ON_DEMAND), or re-sort after every step (ALWAYS). */
enum { MPMX_SORT_ON_DEMAND = 0, MPMX_SORT_ALWAYS = 1 };
enum { MPMX_MEM_HOST = 0, MPMX_MEM_DEVICE = 1 };

/* Scene error bits reported by mpmx_scene_stats (sticky: the scene stops at
 * the step that raised one).  OUT_OF_MESH and NONFINITE come from the
 * particles; TILE (a work item's particles spread beyond its LDS node tile)
 * and SORT (a reorder gave up waiting for one of its phases) are failures of
 * the implementation that its own rules exclude, reported rather than
 * silently mishandled; mpmx_scene_read maps them to MPMX_E_STATE. */
enum {
    MPMX_ERRBIT_OUT_OF_MESH = 1u,
    MPMX_ERRBIT_NONFINITE = 2u,
    MPMX_ERRBIT_TILE = 4u,
    MPMX_ERRBIT_SORT = 8u
};

/* --------------------------------------------------------- descriptors -- */
/* Each descriptor starts with its own size in bytes (sizeof), so that later
 * versions can grow it; a size smaller than this version's is rejected. */

/* Background mesh of n[0] x n[1] x n[2] 8-node hexahedra (code overview:
 * Mesh, Node, Cell).  Uniform grid when node_x is NULL: node (i, j, k) at
 * origin + h (i, j, k).  Isoparametric mesh otherwise (isoparametric-mesh
 * section): the same logically structured cells, node numbering and face
 * rules, node I at node_x[3 I + a] (host memory, (n0+1)(n1+1)(n2+1) x 3,
 * copied at scene creation), each cell the trilinear image of the natural
 * cube [-1,1]^3 of its eight nodes.  A particle belongs to the cell whose
 * inverse map puts it at natural coordinates -1 <= xi_a < 1 (found by
 * Newton-Raphson from the cell's affine guess, by a walk across cell faces
 * from the particle's previous cell); origin and h then name the uniform
 * grid the mesh was made from, whose cells start the walk at scene
 * creation.  Isoparametric meshes take MPMX_SHAPE_LINEAR only, and every
 * cell must have a positive Jacobian at its eight corners
 * (MPMX_E_INVALID_ARG otherwise). */
typedef struct {
    uint32_t size;
    int32_t n[3];       /* cells per axis, each >= 1 */
    double origin[3];   /* position of node (0,0,0) */
    double h;           /* cell edge length, > 0 */
    const double *node_x;   /* NULL, or the isoparametric mesh's node positions */
} mpmx_mesh;

typedef struct {
    uint32_t size;
    int32_t model;      /* MPMX_LINEAR_ELASTIC or MPMX_DRUCKER_PRAGER */
    int32_t dp_cone;    /* MPMX_DP_* (Drucker-Prager only) */
    int32_t pad_;
    double rho, E, nu;  /* density, Young's modulus, Poisson ratio (-1 < nu < 0.5) */
    double phi, psi, c; /* friction and dilation angles (radians), cohesion */
} mpmx_material;

/* Velocity constraints: face rules for faces -x,+x,-y,+y,-z,+z (a node with
 * index i_b <= 0 lies on face -b, i_b >= n_b on face +b, ghost nodes
 * included; FIXED constrains all components to 0, SLIP the normal one), then
 * n_extra per-node constraints (node id, axis 0..2, prescribed velocity) that
 * take precedence.  Constrained components get the prescribed velocity and
 * zero acceleration (code overview: velocity constraints held at nodes;
 * isoparametric-mesh section: boundary conditions applied at the nodes).
 *
 * Nodal external forces (benchmark section: a traction applied at the ends
 * of the strip, here as the equivalent nodal forces): n_force entries of
 * node id and force vector (force_value[3 e + a], newtons), added to the
 * nodal force of every step before the acceleration a = f / m is formed (so
 * a void node, m <= eps_m, still gets a = 0).  Entries naming the same node
 * add up.  In the scene's n-th step (n = 1 for its first) the forces are
 * scaled by u^2 (3 - 2 u) with u = n / force_ramp_steps while n <
 * force_ramp_steps, and by 1 from then on: a smooth ramp to a hold, which
 * loads the body quasi-statically (its residual vibration falls with the
 * square of the ramp time); force_ramp_steps = 0 applies them in full from
 * the first step.  n_force = 0 (and NULL pointers) for none. */
typedef struct {
    uint32_t size;
    int32_t face[6];
    int64_t n_extra;
    const int64_t *node;
    const int32_t *axis;
    const double *value;
    int64_t n_force;
    const int64_t *force_node;
    const double *force_value;
    int64_t force_ramp_steps;   /* >= 0 */
} mpmx_bc;

typedef struct {
    uint32_t size;
    int32_t algo;            /* MPMX_USF, MPMX_USL or MPMX_MUSL */
    int32_t shape;           /* MPMX_SHAPE_LINEAR or MPMX_SHAPE_GIMP */
    int32_t velocity_update; /* MPMX_FLIP or MPMX_PIC */
    int32_t precision;       /* MPMX_FP32 (x and nodal mass FP64) or MPMX_FP64 */
    int32_t sort_policy;     /* MPMX_SORT_* */
    double gravity[3];
    double dt;               /* > 0 */
    double mass_eps_rel;     /* nodes with m <= mass_eps_rel * mean(m_p) are void */
} mpmx_scheme;

/* Particle input: n rows; x, v (n x 3), stress (n x 6, NULL = zero), vol and
 * mass (n).  All double; in FP32 scenes v, stress, vol and mass are rounded
 * to float.  mem says where the arrays live. */
typedef struct {
    uint32_t size;
    int32_t mem;
    int64_t n;
    const double *x, *v, *stress, *vol, *mass;
} mpmx_particles;

/* Particle output in the original input order: any pointer may be NULL to
 * skip that field; cell receives the linear cell id of each particle. */
typedef struct {
    uint32_t size;
    int32_t mem;
    double *x, *v, *stress, *vol;
    int32_t *cell;
} mpmx_particles_out;

/* Scene counters.  pic_hash identifies the particles-per-cell histogram of
 * the current positions (code overview: a cell is active when it holds a
 * material point): starting from h = 14695981039346656037, for every cell
 * c (linear cell id, ascending) holding k > 0 particles, h = (h ^ c) *
 * 1099511628211, then h = (h ^ k) * 1099511628211 (64-bit FNV-1a steps on
 * the two integers, modulo 2^64).  Equal histograms give equal hashes.
 * lost_particles counts the particles that left the mesh in the step that
 * stopped the scene (0 while it runs). */
typedef struct {
    uint32_t size;
    int64_t n_particles;
    int64_t steps_done;     /* steps completed (queued work included after a sync) */
    int64_t n_sorts;        /* particle reorders performed */
    int64_t n_items;        /* current work items (brick chunks) */
    int64_t active_cells;   /* cells holding at least one particle */
    uint32_t error_bits;    /* MPMX_ERRBIT_* */
    uint32_t pad_;
    uint64_t device_bytes;  /* device memory held by the scene */
    uint64_t pic_hash;      /* hash of the particles-per-cell histogram (above) */
    int64_t lost_particles; /* particles outside the mesh when the scene stopped */
} mpmx_stats;

typedef struct mpmx_ctx mpmx_ctx;

/* ------------------------------------------------------------ context -- */

/* Library version (MPMX_VERSION). */
int mpmx_version(void);

/* Create a context on HIP device `device`.  stream: a hipStream_t to queue
 * work on (e.g. torch.cuda.current_stream().cuda_stream), or NULL for a
 * stream the context creates and owns.  Fails with MPMX_E_HIP if the device
 * is not a usable GPU. */
int mpmx_create(mpmx_ctx **out, int device, void *stream);

/* Destroy a context, its scenes and servers; waits for queued work. */
void mpmx_destroy(mpmx_ctx *ctx);

/* Message of the last failed call on ctx (valid until the next call). */
const char *mpmx_last_error(const mpmx_ctx *ctx);

/* Launch options of a context (not of the method: results do not depend on
 * them beyond the order of floating-point sums).
 *   MPMX_OPT_GRAPH_STEPS   steps recorded into one HIP graph and replayed
 *                          with one launch; 0 launches every kernel
 *                          directly.  Default 8.  The graph of a batch is
 *                          recorded by its first call of more than one step
 *                          (after tuning, when that call tunes), so later
 *                          calls only replay it.  Graphs are not used while
 *                          per-kernel profiling is on.
 *   MPMX_OPT_AUTOTUNE      1 (default): on the first call that runs at least
 *                          MPMX_TUNE_MIN_STEPS steps on a batch layout
 *                          (precision, shape function, algorithm and the
 *                          power-of-two bucket of its particle count), time
 *                          the item kernels at every pair of workgroup size
 *                          and grid density (3 steps each), then keep, for
 *                          each of the two kernels, its fastest pair for
 *                          that layout; pairs at most 1 % plus 2 us
 *                          slower than the fastest count as ties, settled
 *                          by a fixed preference order (16 workgroups per
 *                          CU and 256 threads first), so that the choice is
 *                          stable between runs.  The timed steps are steps
 *                          of the call.
 *                          0: use the values below.
 *   MPMX_OPT_STRESS_THREADS  workgroup size of the stress kernel (USL and
 *                          MUSL: the P2G kernel): 64, 128 or 256.  Setting
 *                          it, or any launch shape below, turns autotuning
 *                          off.
 *   MPMX_OPT_G2P_THREADS   same for the G2P(+P2G) kernel (MUSL: both G2P
 *                          kernels).
 *   MPMX_OPT_BLOCKS_PER_CU workgroups per compute unit of both item
 *                          kernels' persistent grids, 1..64 (reads back
 *                          the stress kernel's).
 *   MPMX_OPT_STRESS_BLOCKS_PER_CU, MPMX_OPT_G2P_BLOCKS_PER_CU  the same for
 *                          one of the two kernels.
 *   MPMX_OPT_GRAPH_LAUNCHES  read-only: graph launches so far.
 *   MPMX_OPT_TUNE_RUNS     read-only: tuning passes so far.
 * mpmx_get_option of the launch shapes returns the values of the last call
 * that stepped a batch.  Errors: MPMX_E_INVALID_ARG for an unknown option
 * or a value out of range. */
#define MPMX_TUNE_MIN_STEPS 40
enum {
    MPMX_OPT_GRAPH_STEPS = 1,
    MPMX_OPT_AUTOTUNE = 2,
    MPMX_OPT_STRESS_THREADS = 3,
    MPMX_OPT_G2P_THREADS = 4,
    MPMX_OPT_BLOCKS_PER_CU = 5,
    MPMX_OPT_GRAPH_LAUNCHES = 6,
    MPMX_OPT_TUNE_RUNS = 7,
    MPMX_OPT_STRESS_BLOCKS_PER_CU = 8,
    MPMX_OPT_G2P_BLOCKS_PER_CU = 9
};
int mpmx_set_option(mpmx_ctx *ctx, int option, int64_t value);
int mpmx_get_option(mpmx_ctx *ctx, int option, int64_t *value);

/* Per-kernel timing with HIP events on the context stream.  enable != 0
 * records an event pair around every kernel launch from now on;
 * mpmx_profile_read synchronises and returns, for up to `cap` kernels, the
 * kernel name, launch count and summed milliseconds; *n gets the number of
 * kernels seen.  mpmx_profile_reset clears the totals. */
int mpmx_profile_enable(mpmx_ctx *ctx, int enable);
int mpmx_profile_reset(mpmx_ctx *ctx);
int mpmx_profile_read(mpmx_ctx *ctx, int cap, const char **names, int64_t *launches,
                      double *ms, int *n);

/* ------------------------------------------------------------- scenes -- */

/* Device bytes a scene of this mesh, scheme and particle count would hold
 * (used for admission).  Pure: touches no device. */
int mpmx_scene_bytes(const mpmx_mesh *mesh, const mpmx_scheme *scheme, int64_t n_particles,
                     uint64_t *bytes);

/* Create a scene: validate and copy the descriptors, upload the particles,
 * bin them into cells (on the context's second stream, so that the upload
 * overlaps steps already queued on the context stream; returns when it is
 * done).  *scene receives an id > 0.  A particle outside the
 * mesh or a non-finite input fails with MPMX_E_OUT_OF_MESH /
 * MPMX_E_NONFINITE and creates nothing.  The kernels address each particle
 * and node field with 32-bit byte offsets, so a scene holds fewer than
 * 2^32 / 24 particles at MPMX_FP32 (2^32 / 48 at MPMX_FP64) and fewer than
 * 2^32 / 12 nodes (2^32 / 24); larger ones fail with MPMX_E_INVALID_ARG. */
int mpmx_scene_create(mpmx_ctx *ctx, const mpmx_mesh *mesh, const mpmx_material *mat,
                      const mpmx_bc *bc, const mpmx_scheme *scheme,
                      const mpmx_particles *particles, uint64_t *scene);

/* Queue nsteps (>= 0) time steps.  Asynchronous; a particle leaving the
 * mesh or a non-finite value stops the scene at the step where it happened
 * and is reported by mpmx_scene_stats / mpmx_scene_read. */
int mpmx_scene_step(mpmx_ctx *ctx, uint64_t scene, int64_t nsteps);

/* Copy the particle state, in the original particle order, to the caller's
 * buffers.  Waits for this scene's queued steps only (steps queued for
 * other scenes keep running), and returns with the copies done.  Returns MPMX_E_OUT_OF_MESH / MPMX_E_NONFINITE
 * (after copying) if the scene has stopped on that error, and MPMX_E_STATE
 * if it stopped for a reason of the implementation: a work item's particles
 * spread beyond its node tile, or a reorder that gave up waiting (neither
 * is expected; the scene stops, and its state is what the failing step
 * left). */
int mpmx_scene_read(mpmx_ctx *ctx, uint64_t scene, const mpmx_particles_out *out);

/* Particles per cell (n_x n_y n_z uint32 in linear cell order) for the
 * current positions, to host or device memory (synchronises). */
int mpmx_scene_cell_counts(mpmx_ctx *ctx, uint64_t scene, uint32_t *counts, int32_t mem);

/* Nodal mass (nn), momentum and force (nn x 3) accumulated by the last step,
 * before constraints, to host buffers (synchronises); nn as in the header
 * comment.  Any pointer may be NULL. */
int mpmx_scene_nodes(mpmx_ctx *ctx, uint64_t scene, double *mass, double *momentum, double *force);

/* Counters and error bits of a scene (synchronises). */
int mpmx_scene_stats(mpmx_ctx *ctx, uint64_t scene, mpmx_stats *out);

/* Free a scene (waits for its own queued work only). */
int mpmx_scene_destroy(mpmx_ctx *ctx, uint64_t scene);

/* ------------------------------------------------------------- batches -- */

/* Advance n scenes together, scene i by nsteps[i] steps: every stage is one
 * launch over the flattened (scene, work item) list of all scenes still
 * stepping.  Scenes must share shape function and precision.  Asynchronous.
 * Results equal running each scene alone up to the order of floating-point
 * sums. */
int mpmx_batch_step(mpmx_ctx *ctx, const uint64_t *scenes, const int64_t *nsteps, int n);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * steps as mpmx_batch_step on scenes created beforehand, with every device
 * array of the call (scene list, offsets, step counts, reorder flags and
 * brick-scan partial sums, list of non-empty bricks) in a fixed 4 MiB
 * scratch array that each GPU holds for the life of the process.  It calls
 * no hipMalloc or hipFree and creates no graph or event: every step is
 * launched directly, with the launch shape the context has already tuned
 * for this batch layout, else the fixed one (mpmx_set_option).  Limits: at
 * most 4096 scenes, and about one million 4x4x4-cell bricks over all the
 * scenes' meshes (a brick is counted over the whole mesh, occupied or not);
 * larger batches fail with MPMX_E_INVALID_ARG and run nothing.  The array
 * is shared by every call on one GPU and keeps the last call's contents:
 * calls on the same context are ordered by its stream, but calls from
 * different contexts on one GPU whose work overlaps race on it.  Other
 * errors as mpmx_batch_step.  Asynchronous. */
int mpmx_batch_step_noalloc(mpmx_ctx *ctx, const uint64_t *scenes, const int64_t *nsteps, int n);

/* -------------------------------------------------------------- fences -- */

/* A fence marks the work queued so far on the context stream (the steps of
 * every batch and scene; uploads and read-backs run on the context's second
 * stream and are not covered).  Not a method of the paper: it lets a host
 * loop keep a bounded amount of work queued ahead of the GPU and learn,
 * without blocking, which of it has finished.
 * mpmx_fence_record: *fence gets the new fence's id.  Errors:
 * MPMX_E_INVALID_ARG, MPMX_E_HIP. */
int mpmx_fence_record(mpmx_ctx *ctx, uint64_t *fence);

/* Whether the fence's work has finished.  block = 0: *done = 1 or 0 at once;
 * block != 0: waits, then *done = 1.  A fence reported done is freed and its
 * id is no longer valid.  Errors: MPMX_E_INVALID_ARG, MPMX_E_NOT_FOUND
 * (unknown or already freed id), MPMX_E_HIP. */
int mpmx_fence_wait(mpmx_ctx *ctx, uint64_t fence, int block, int *done);

/* Free a fence without waiting.  Errors: MPMX_E_INVALID_ARG,
 * MPMX_E_NOT_FOUND. */
int mpmx_fence_release(mpmx_ctx *ctx, uint64_t fence);

/* ------------------------------------------------------------- serving -- */

/* A request loop over one context: independent scenes arrive at any time,
 * are admitted in arrival order while their device bytes (mpmx_scene_bytes,
 * plus per-node constraint arrays) fit the budget, stay resident on the
 * device while they step, and leave their final particle state in host
 * memory.  Not a method of the paper: it serves many of the paper's
 * problems (mesh, particles, material, constraints, scheme, step count) on
 * one GPU.  A server drives its context from one host thread; scenes the
 * caller creates on the same context are not touched by it. */
typedef struct mpmx_server mpmx_server;

/* mpmx_request.flags: MPMX_REQ_BORROW keeps the particle arrays (x, v,
 * stress, vol, mass) by pointer instead of copying them at submit; they must
 * stay valid and unchanged until the request's completion has been polled.
 * Descriptors, constraint and force lists and node positions are always
 * copied. */
enum { MPMX_REQ_BORROW = 1 };

typedef struct mpmx_request {
    uint32_t size;                       /* sizeof(mpmx_request) */
    uint32_t flags;                      /* MPMX_REQ_* */
    const mpmx_mesh *mesh;
    const mpmx_material *material;
    const mpmx_bc *bc;
    const mpmx_scheme *scheme;
    const mpmx_particles *particles;     /* MPMX_MEM_HOST */
    int64_t nsteps;                      /* >= 0 */
    uint64_t tag;                        /* returned in the completion */
    /* optional caller-owned host buffers (MPMX_MEM_HOST; x, v, stress, vol
     * required, cell optional) that receive the final state; they must stay
     * valid until the completion has been polled.  NULL: the server holds
     * the state until mpmx_server_release. */
    const mpmx_particles_out *out;
} mpmx_request;

typedef struct mpmx_completion {
    uint32_t size;                       /* sizeof(mpmx_completion) */
    int32_t status;                      /* MPMX_OK or the scene's error code */
    uint64_t request;                    /* id from mpmx_server_submit */
    uint64_t tag;
    int64_t n;                           /* particles */
    int64_t steps_done;
    /* final state in the original particle order: x, v (n x 3), stress
     * (n x 6), vol; the request's output buffers, or host memory owned by the
     * server until mpmx_server_release */
    const double *x, *v, *stress, *vol;
    double t_submit, t_admit, t_done;    /* seconds, mpmx_server_clock */
} mpmx_completion;

/* Create a server on ctx with a device-memory budget (bytes) and the most
 * steps one tick runs.  Errors: MPMX_E_INVALID_ARG. */
int mpmx_server_create(mpmx_ctx *ctx, uint64_t budget_bytes, int64_t max_tick_steps, mpmx_server **out);

/* Admission by occupancy: while the resident scenes that still have steps
 * to run hold at least `particles` particles, tick admits nothing more, so
 * requests wait in arrival order instead of sharing the GPU with scenes
 * that already fill it (sharing slows each of them and lengthens every
 * latency).  A request is admitted whatever its size when no such scene is
 * resident.  0 (the default) turns the limit off.  Errors:
 * MPMX_E_INVALID_ARG (srv NULL or particles < 0). */
int mpmx_server_set_fill(mpmx_server *srv, int64_t particles);

/* Queue a request; its inputs are copied before return (the particle
 * arrays are only kept by pointer with MPMX_REQ_BORROW).  *id identifies it.
 * MPMX_E_BUDGET if the scene alone exceeds the budget; descriptor errors as
 * mpmx_scene_create. */
int mpmx_server_submit(mpmx_server *srv, const mpmx_request *req, uint64_t *id);

/* One scheduling round, continuous batching: admit queued requests in
 * arrival order while they fit the budget and the fill limit (their uploads
 * overlap the steps already queued); queue the steps of every resident
 * scene, one batch per (precision, shape, algorithm) group, by the number of
 * steps until the first of them completes (at least 16, at most
 * max_tick_steps), and record a fence after them; then, oldest round first,
 * copy to host memory, free and record as complete the scenes whose last
 * steps a finished round queued.  The host stays at most two rounds ahead
 * of the GPU: a round that leaves three unfinished waits for the oldest, and
 * a round that queues nothing waits for the oldest unfinished one.
 * Optional outputs: requests resident (not yet complete) and queued after
 * the round. */
int mpmx_server_tick(mpmx_server *srv, int *n_resident, int *n_queued);

/* Move up to max completions (oldest first) into out[]; *n gets the count.
 * Their arrays stay valid until mpmx_server_release(id). */
int mpmx_server_poll(mpmx_server *srv, mpmx_completion *out, int max, int *n);

/* Free the host arrays of a polled completion. */
int mpmx_server_release(mpmx_server *srv, uint64_t id);

/* Seconds on the server's monotonic clock (the completion timestamps). */
double mpmx_server_clock(const mpmx_server *srv);

/* Free the server, its queued requests, resident scenes and completions. */
void mpmx_server_destroy(mpmx_server *srv);

#ifdef __cplusplus
}
#endif

#endif
