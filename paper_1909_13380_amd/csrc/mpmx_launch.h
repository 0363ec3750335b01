// mpmx_launch.h -- kernel entry addresses handed from the kernel translation
// unit to the host runtime, which launches them with hipLaunchKernel.
#pragma once

namespace mpmx {

// Kernels instantiated per (precision, shape function).
struct KernelSet {
    const void *load;       // (SceneDev*, x, v, sig, vol, mass)
    const void *read_out;   // (const SceneDev*, x, v, sig, vol, cell)
    const void *nodes_out;  // (const SceneDev*, m, p, f)
    const void *clear;      // (BatchDev)
    const void *scatter;    // (BatchDev)
    const void *p2g;        // (BatchDev)
    const void *stress;     // (BatchDev)
    const void *g2p;        // (BatchDev)
    const void *p2g_usl;    // (BatchDev)
    const void *g2p_usl;    // (BatchDev)
};

struct CommonKernels {
    const void *step_control;   // (BatchDev, int mode)
    const void *set_remaining;  // (BatchDev, const int64_t*)
    const void *sort_count;     // (BatchDev)
    const void *sort_bricks;    // (BatchDev)
    const void *sort_scan;      // (BatchDev)
    const void *sort_cells;     // (BatchDev)
    const void *cell_counts;    // (const SceneDev*, uint32_t*)
};

const KernelSet &kernel_set(int prec, int shape);
const CommonKernels &common_kernels();

}  // namespace mpmx
