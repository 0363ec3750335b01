// mpmx_dev.h -- device-side scene description shared by the gfx950 kernels and
// the host runtime of libmpmx.
//
// Layout in HBM (per scene):
//   particles, structure of arrays, double-buffered for reordering:
//     x[3][n] f64 | v[3][n] R | sig[6][n] R | vol[n] R | mass[n] R | key[n] u32 | pid[n] u32
//   nodes, dense over the (ghost-padded) node grid:
//     m[nn] f64 | p[3][nn] R | f[3][nn] R      (R = float or double)
//   sort scratch: cnt[nkeys] u32, cstart[nkeys] u32, rank[n] u32,
//     bcnt/bitem[nbricks] u32, bstart/istart[nbricks+1] u32
//   work list: items[max_items], tiles[max_items]
// Cells are grouped in bricks of 4x4x4; a particle's key is
//   brick_id * 64 + local cell index, brick_id = bx + nbx (by + nby bz),
// so sorting by key groups a brick's particles together and orders them by
// cell inside it.
#pragma once

#include <stdint.h>

namespace mpmx {

constexpr int kBrick = 4;                 // cells per brick edge
constexpr int kBrickCells = 64;           // cells per brick
constexpr int kChunk = 512;               // max particles per work item
constexpr int kBlock = 256;               // threads per work-item workgroup
constexpr int kMaxTileNodes = 729;        // 9^3: GIMP tile with one cell of drift

enum Ctl : int {
    CTL_CUR = 0,        // which particle buffer is current (0/1)
    CTL_NEED_SORT = 1,  // reorder before the next step
    CTL_N_ITEMS = 2,    // work items of the current order
    CTL_ERR = 3,        // error bits (sticky)
    CTL_N_SORTS = 4,    // reorders performed
    CTL_STEPS = 5,      // completed steps
    CTL_REMAIN = 6,     // steps still to run in the current call
    CTL_ACTIVE = 7,     // the scene takes part in the step being run
    CTL_WORDS = 16
};

// ERR_TILE: an item's particles spread beyond the LDS node tile, which the
// reorder rule makes impossible; reported rather than silently mishandled.
enum ErrBit : uint32_t { ERR_OUT_OF_MESH = 1u, ERR_NONFINITE = 2u, ERR_TILE = 4u };

struct Item {
    uint32_t start;  // first particle (storage order)
    uint32_t count;  // particles in the item (<= kChunk)
    uint32_t brick;  // brick the item's particles were sorted into
    uint32_t pad;
};

// Node box touched by an item: lo (node index per axis, ghost-relative
// indexing i.e. may be -1) and extent per axis.  Written by the first
// scatter of a step, read by the later stages and by the next step's clear.
struct Tile {
    int lo[3];
    int dim[3];
    int fits;   // extent fits the LDS tile
    int pad;
};

struct SceneDev {
    // mesh
    double origin[3];
    double h;
    int n[3];        // cells
    int nb[3];       // bricks
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
    int has_apex;
    // scheme
    int algo, shape, vel_update, prec;
    double dt;
    double g[3];
    double eps_m;
    uint32_t face_bits;  // 2 bits per face: 0 free, 1 fixed, 2 slip
    // optional per-node constraints
    const uint8_t *bc_mask;   // bits 0..2: component constrained
    const double *bc_val;     // 3 per node (prescribed velocity)
    // particles (two buffers)
    double *x[2];
    void *v[2];
    void *sig[2];
    void *vol[2];
    void *mass[2];
    uint32_t *key[2];
    uint32_t *pid[2];
    // nodes
    double *nm;
    void *np_;   // momentum p[3][nn]
    void *nf;    // force f[3][nn]
    // sort scratch
    uint32_t *cnt, *cstart, *rank;
    uint32_t *bcnt, *bitem, *bstart, *istart;
    Item *items;
    Tile *tiles;
    uint32_t *ctl;
};

// A launch over several scenes: work is flattened over scenes in order.
struct BatchDev {
    const SceneDev *const *scenes;  // device array of device pointers
    const int64_t *poffs;           // particle offsets [nscenes+1] (static)
    const int64_t *boffs;           // brick offsets [nscenes+1] (static)
    uint32_t *ioffs;                // item offsets [nscenes+1] (device-written)
    int nscenes;
    int pad;
    int64_t total_particles;
    int64_t total_bricks;
    int64_t max_items;              // upper bound of the flattened item count
};

}  // namespace mpmx
