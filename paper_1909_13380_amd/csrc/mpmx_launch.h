// mpmx_launch.h -- kernel entry addresses handed from the kernel translation
// unit to the host runtime, which launches them with hipLaunchKernel.
#pragma once

namespace mpmx {

// Workgroup sizes the item kernels are built for (the autotuner picks one
// per kernel).
constexpr int kItemThreadChoices[3] = {64, 128, 256};
constexpr int kNumItemThreadChoices = 3;

// Kernels instantiated per (precision, shape function); the item kernels
// also per workgroup size (index into kItemThreadChoices).
struct KernelSet {
    const void *load;       // (SceneDev*, x, v, sig, vol, mass)
    const void *read_out;   // (const SceneDev*, x, v, sig, vol, cell)
    const void *nodes_out;  // (const SceneDev*, m, p, f)
    const void *reorder;    // (BatchDev): reorder, then the step control
    const void *p2g[kNumItemThreadChoices];      // (BatchDev)
    const void *stress[kNumItemThreadChoices];   // (BatchDev)
    const void *g2p_p2g[kNumItemThreadChoices];  // (BatchDev)
    const void *p2g_usl[kNumItemThreadChoices];  // (BatchDev)
    const void *g2p_usl[kNumItemThreadChoices];  // (BatchDev)
    const void *p2g_musl[kNumItemThreadChoices];     // (BatchDev)
    const void *musl_g2p[kNumItemThreadChoices];     // (BatchDev)
    const void *musl_stress[kNumItemThreadChoices];  // (BatchDev)
};

struct CommonKernels {
    const void *begin;        // (BatchDev, const int64_t*)
    const void *cell_counts;  // (const SceneDev*, uint32_t*)
};

const KernelSet &kernel_set(int prec, int shape);
const CommonKernels &common_kernels();

}  // namespace mpmx
