// Device descriptors of the batched KFBI steps (see batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace kfbi {

constexpr int kBatchNmax = 4096;    // largest grid a batch serves
// LDS of the batched fast solve holds this many doubles of mode solutions
// (and, after them, kMaxModesPerGroup x kMaxExtra sums of extra pieces):
// eight padded modes of the 2048^2 grid, four of the 4096^2 grid
constexpr int kBatchXs = 8 * (2048 + 64);

// Modes per workgroup of a batched problem with grid N: the largest power of two
// up to kMaxModesPerGroup whose padded solutions fit kBatchXs.
__host__ __device__ constexpr int batch_modes_per_group(int N) {
    int R = kMaxModesPerGroup;
    while (R > 1 && R * (N + 64) > kBatchXs) R /= 2;
    return R;
}

// One live problem of a batch, resident in device memory.
struct SlotDev {
    DevPlan p;
    GmresBufs b;
    double* corr_il;   // interleaved corrections (T x 64)
    double* partial;   // Gs x M partial sums, one row per mode block
    int Gs;            // mode blocks: ceil((n-1) / batch_modes_per_group(N))
    int pad;
};

// Work lists of the batched launches, rebuilt on the host when a slot is
// admitted or released.  counts = {correction items, mode items, sample items,
// live slots, GMRES chunk items}; items are (slot, first index) pairs.
struct BatchWork {
    const int* counts;
    const int2* corr_items;   // blocks of 256 irregular nodes
    const int2* mode_items;   // mode blocks of batch_modes_per_group(N) modes
    const int2* cp_items;     // blocks of 64 samples
    const int* live;          // live slot ids
    const int2* gm_items;     // (slot, chunk) of the GMRES vector launches
    int max_live;
};
constexpr int kBatchCounts = 5;

size_t modes_b_lds_bytes();
hipError_t launch_batch_step(const SlotDev* slots, BatchWork w, int n_cu, hipStream_t s);

}  // namespace kfbi
