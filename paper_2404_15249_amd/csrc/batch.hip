// Batched KFBI steps: many problems of uneven size advance through one launch
// per stage of a GMRES iteration.  Every launch is persistent: a fixed grid
// walks a device-resident work list of (slot, block) items, so the same
// captured graph serves any mix of live slots, and a slot that has converged
// turns its items into no-ops.  Each slot's arithmetic is split into the same
// blocks whatever else is in the batch (one workgroup partial per mode block,
// fixed reduction order), so its result does not depend on the mix.
#include <hip/hip_runtime.h>

#include "batch.h"
#include "device.h"
#include "gmres.h"
#include "graph.h"

namespace kfbi {

namespace {

__device__ __forceinline__ bool slot_done(const SlotDev& S) { return S.b.st->converged != 0; }

__global__ __launch_bounds__(256) void k_correct_b(const SlotDev* __restrict__ slots, BatchWork w) {
    const int n_items = w.counts[0];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 item = w.corr_items[it];
        const SlotDev& S = slots[item.x];
        if (slot_done(S)) continue;
        const int r = item.y + threadIdx.x;
        if (r >= S.p.I) continue;
        const JumpSrc js{S.b.xcur, S.b.s2cur, nullptr, nullptr, nullptr, nullptr};
        S.corr_il[S.p.il_pos[r]] = correction_at(S.p, js, r);
    }
}

template <int C>
__device__ __forceinline__ void modes_item(const DevPlan& p, const double* corr, int row, const ModesLds& L,
                                           double* part) {
    constexpr int R = batch_modes_per_group(64 * C);
    modes_round<C, R>(p, corr, row * R, L, [&](int cp, double s) { part[(size_t)row * p.M + cp] = s; });
}

__global__ __launch_bounds__(kModeWaves * 64) void k_modes_b(const SlotDev* __restrict__ slots, BatchWork w) {
    extern __shared__ double smem[];
    ModesLds L;
    L.sq = smem;
    L.xs = smem + (kBatchNmax / 2 + 2);
    L.ex = L.xs + kBatchXs;
    const int n_items = w.counts[1];
    int curN = -1;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 item = w.mode_items[it];
        const SlotDev& S = slots[item.x];
        if (slot_done(S)) continue;
        const DevPlan& p = S.p;
        if (p.N != curN) {
            __syncthreads();
            for (int k = threadIdx.x; k <= p.N / 2; k += kModeWaves * 64) L.sq[k] = p.sinq[k];
            curN = p.N;
        }
        switch (p.N) {
            case 64: modes_item<1>(p, S.corr_il, item.y, L, S.partial); break;
            case 128: modes_item<2>(p, S.corr_il, item.y, L, S.partial); break;
            case 256: modes_item<4>(p, S.corr_il, item.y, L, S.partial); break;
            case 512: modes_item<8>(p, S.corr_il, item.y, L, S.partial); break;
            case 1024: modes_item<16>(p, S.corr_il, item.y, L, S.partial); break;
            case 2048: modes_item<32>(p, S.corr_il, item.y, L, S.partial); break;
            default: modes_item<64>(p, S.corr_il, item.y, L, S.partial); break;
        }
    }
}

__global__ __launch_bounds__(1024) void k_reduce_b(const SlotDev* __restrict__ slots, BatchWork w) {
    __shared__ double red[16 * 64];
    const int n_items = w.counts[2];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 item = w.cp_items[it];
        const SlotDev& S = slots[item.x];
        if (slot_done(S)) continue;
        const JumpSrc js{S.b.xcur, S.b.s2cur, nullptr, nullptr, nullptr, nullptr};
        reduce_samples64(S.p, js, S.partial, S.Gs, item.y, S.b.w, red);
        gm_dots1_64(S.b, S.p.M, item.y / 64, red);
        __syncthreads();                                 // red is reused by the next item
    }
}

// GMRES (gmres.h): the update and emit launches walk (slot, chunk) items; the
// first pass's dots ride on k_reduce_b and the commit on the update.
template <int Kind>
__global__ __launch_bounds__(kGmChunk) void k_gm_vec_b(const SlotDev* __restrict__ slots, BatchWork w) {
    const int n_items = w.counts[4];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 item = w.gm_items[it];
        const SlotDev& S = slots[item.x];
        if (Kind == 1) gm_update1_commit(S.b, S.p.M, item.y);
        if (Kind == 3) gm_emit(S.p.taps, S.b, S.p.M, item.y);
        __syncthreads();                                 // the item's LDS is reused by the next item
    }
}


}  // namespace

size_t modes_b_lds_bytes() {
    return sizeof(double) * ((size_t)(kBatchNmax / 2 + 2) + (size_t)kBatchXs + (size_t)kMaxModesPerGroup * kMaxExtra);
}

hipError_t launch_batch_step(const SlotDev* slots, BatchWork w, int n_cu, hipStream_t s) {
    const size_t lds = modes_b_lds_bytes();
    if (hipError_t e = hipFuncSetAttribute((const void*)k_modes_b, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds))
        return e;
    const dim3 t(kGmChunk), gv(n_cu);
    if (hipError_t e = klaunch(&k_correct_b, dim3(n_cu * 2), dim3(256), 0, s, slots, w)) return e;
    if (hipError_t e = klaunch(&k_modes_b, dim3(n_cu), dim3(kModeWaves * 64), lds, s, slots, w)) return e;
    if (hipError_t e = klaunch(&k_reduce_b, dim3(n_cu), dim3(1024), 0, s, slots, w)) return e;
    if (hipError_t e = klaunch(&k_gm_vec_b<1>, gv, t, 0, s, slots, w)) return e;
    return klaunch(&k_gm_vec_b<3>, gv, t, 0, s, slots, w);
}

}  // namespace kfbi
