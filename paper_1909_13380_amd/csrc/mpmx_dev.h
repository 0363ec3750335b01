// mpmx_dev.h -- device-side scene description shared by the gfx950 kernels and
// the host runtime of libmpmx.
//
// Layout in HBM (per scene):
//   particles, structure of arrays, two buffers (a reorder moves between them):
//     x[3][n] f64 | v[3][n] R | sig[6][n] R | vol[n] R | mass[n] R | cell[n] u32 | pid[n] u32
//   nodes, dense over the (ghost-padded) node grid, two buffers (one step
//   fills one while the other still holds the previous step):
//     m[nn] f64 | p[3][nn] R | f[3][nn] R      (R = float or double)
//   sort scratch: cnt[nkeys] u32, cstart[nkeys] u32, rank[n] u32, perm[n] u32,
//     bcnt/bitem[nbricks] u32, bstart/istart[nbricks+1] u32
//   work list: items[max_items]; node boxes tiles[2][max_items], tstep[max_items]
// A particle's cell is stored packed: cx | cy << 11 | cz << 22.  Cells are
// grouped in bricks of 4x4x4; the sort key is brick_id * 64 + local cell
// index, brick_id = bx + nbx (by + nby bz).  A reorder groups each brick's
// particles together and, inside the brick, stores them level-major: the
// first particle of every occupied cell, then the second of every cell
// holding two or more, and so on.
#pragma once

#include <stdint.h>

namespace mpmx {

constexpr int kBrick = 4;                 // cells per brick edge
constexpr int kBrickCells = 64;           // cells per brick
constexpr int kChunk = 512;               // max particles per work item
constexpr int kXcds = 8;                  // accelerator dies (one L2 each) of the GPU
constexpr int kBlock = 1024;              // threads per workgroup of the reorder and control kernel
constexpr int kSortU = 4;                 // particles per lane in flight in the reorder's particle phases
constexpr int kReorderPerCu = 1;          // most reorder workgroups per compute unit
constexpr uint32_t kScanChunks = 4096;     // most chunks of the reorder's brick scan
// Linear shape functions: per-thread register cache of the gathered support
// nodes, and per-thread register sums of the scattered values, per kernel
// (chosen by measurement on the 2M-particle column: the stress kernel is
// faster with neither, G2P+P2G with the gather cache only).
constexpr bool kStressCacheGather = false;
constexpr bool kStressCacheScatter = false;
constexpr bool kG2PCacheGather = true;
constexpr bool kG2PCacheScatter = false;
constexpr int kMaxCells[3] = {2047, 2047, 1023};   // packed-cell limits

enum Ctl : int {
    CTL_CUR = 0,        // which particle buffer is current (0/1)
    CTL_NEED_SORT = 1,  // reorder before the next step
    CTL_N_ITEMS = 2,    // work items of the current order
    CTL_ERR = 3,        // error bits (sticky)
    CTL_N_SORTS = 4,    // reorders performed
    CTL_STEPS = 5,      // completed steps
    CTL_REMAIN = 6,     // steps still to run in the current call
    CTL_ACTIVE = 7,     // the scene takes part in the step being run
    CTL_NBUF = 8,       // node buffer of the current (or last completed) step
    CTL_READY = 9,      // the other node buffer already holds the next step's P2G
    CTL_HAVE_P2G = 10,  // node buffer CTL_NBUF holds this step's P2G
    CTL_ACC0 = 11,      // items whose tiles[b] cover node buffer b's data (b = 0, 1)
    CTL_ACC1 = 12,
    CTL_BOX_OK = 13,    // tiles[CTL_NBUF] holds this step's node box of every item
    CTL_ALGO = 14,      // the scene's algorithm (0 USF, 1 USL), set at creation
    CTL_LOST = 15,      // particles found outside the mesh (the scene stops on the first)
    CTL_WORDS = 16
};

// ERR_TILE: an item's particles spread beyond the LDS node tile, which the
// reorder rule makes impossible; reported rather than silently mishandled.
// ERR_SORT: the reorder kernel gave up waiting at a grid barrier (its
// workgroups are all resident, so this does not happen); the particles stay
// in their previous order.
enum ErrBit : uint32_t { ERR_OUT_OF_MESH = 1u, ERR_NONFINITE = 2u, ERR_TILE = 4u, ERR_SORT = 8u };

struct Item {
    uint32_t start;  // first particle (storage order)
    uint32_t count;  // particles in the item (<= kChunk)
    uint32_t brick;  // brick the item's particles were sorted into
    uint32_t pad;
};

// Box of nodes: lo per axis (ghost nodes have index -1) and extent.
struct Tile {
    int lo[3];
    int dim[3];
    int fits;   // extent fits the shape's LDS tile size
    int pad;
};

struct SceneDev {
    // mesh
    double origin[3];
    double h, inv_h;
    const double *X;   // isoparametric mesh: node positions x[3][nn] (FP64); null for the uniform grid
    int n[3];        // cells
    int nb[3];       // bricks per axis: room for every brick shift
    int cmin[3];     // smallest cell of the particles at creation (sets the brick shift)
    int N[3];        // nodes per axis incl. ghosts
    int ghost;       // 0 linear, 1 GIMP
    int64_t nn;      // nodes
    int64_t nkeys;   // nbricks * 64
    int64_t nbricks;
    int64_t np;      // particles
    int64_t max_items;
    // material (host-derived constants)
    int model;       // 0 LE, 1 DP
    int sort_always;
    double lam, G, K;
    double eta, xic, etab, apex_p;  // DP: eta, xi*c, eta_bar, apex pressure
    double inv_hard;                // DP: 1 / (G + K eta eta_bar)
    int has_apex;
    // scheme
    int algo, shape, vel_update, prec;
    double dt;
    double g[3];
    double eps_m;
    uint32_t face_bits;  // 2 bits per face: 0 free, 1 fixed, 2 slip
    // optional per-node constraints and external forces
    const uint8_t *bc_mask;   // bits 0..2: component constrained; bit 3: the node has an external force
    const double *bc_val;     // 3 per node (prescribed velocity)
    const double *bc_force;   // 3 per node (external force), or null
    int64_t force_ramp;       // the forces reach full size at this step (0: from the first)
    // particles (two buffers)
    double *x[2];
    void *v[2];
    void *sig[2];
    void *vol[2];
    void *mass[2];
    uint32_t *cell[2];
    uint32_t *pid[2];
    // nodes (two buffers)
    double *nm[2];
    void *np_[2];   // momentum p[3][nn]
    void *nf[2];    // force f[3][nn]
    void *nr;       // MUSL: the updated particle momenta mapped back, r[3][nn]; null otherwise
    // sort scratch
    uint32_t *cnt, *cstart, *rank, *perm;
    uint32_t *bcnt, *bitem, *bstart, *istart;
    Item *items;
    Tile *tiles[2];  // per node buffer: boxes its data was accumulated over
    Tile *tstep;     // per item: node box of its particles in the current step
    uint32_t *ctl;
    // FP32 copies of the constants above, rounded once on the host
    float f_dt, f_inv_h, f_g[3];
    float f_lam, f_G, f_K, f_eta, f_xic, f_etab, f_apex, f_inv_hard;
};

// Words of BatchDev::flags (the array is 128-byte aligned; the words that
// many workgroups update or poll at once sit on 128-byte lines of their
// own).  The reorder kernel uses them; the stage kernel after it clears them.
enum BatchFlag : int {
    BF_ANY_SORT = 0,      // some scene of the batch reorders this step
    BF_SORT_FAIL = 1,     // a reorder workgroup gave up waiting for a phase
    BF_EXIT = 32,         // reorder workgroups finished (the last runs the step control)
    BF_NBRICKS = 64,      // non-empty bricks listed by the reorder
    BF_CLAIM = 96,        // + 32 p: chunks of reorder phase p claimed
    BF_DONE = 96 + 32 * 5,          // + 32 p: chunks of reorder phase p done
    BF_RELEASE = 96 + 64 * 5,       // + 32 g: reorder phases complete, polled by group g
    BF_WORDS = 96 + 64 * 5 + 32 * kXcds
};

// A launch over several scenes: work is flattened over scenes in order.
struct BatchDev {
    const SceneDev *const *scenes;  // device array of device pointers
    uint32_t *const *ctls;          // each scene's control block (CTL_WORDS words)
    const int64_t *poffs;           // particle offsets [nscenes+1] (static)
    const int64_t *boffs;           // brick offsets [nscenes+1] (static)
    uint32_t *ioffs;                // this step's item offsets [nscenes+1]
    uint32_t *coffs;                // offsets of the boxes to clear [nscenes+1]
    uint32_t *flags;                // BF_*
    uint32_t *scan;                 // reorder: per brick chunk, 4 words of brick-scan partial sums [4 kScanChunks]
    uint32_t *bricks;               // reorder: the non-empty bricks (flattened index) [total_bricks]
    int nscenes;
    int pad;
    int64_t total_particles;
    int64_t total_bricks;
    int64_t max_items;              // upper bound of the flattened item count
};

}  // namespace mpmx
