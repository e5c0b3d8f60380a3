// Batched ensemble kernel: many independent lattices advanced by one
// persistent launch, each work item one tile of one instance, stepped by the
// single-lattice tile body (Sec. II, the same step as axi_tile_kernel).
#pragma once

#include "step_kernel.hpp"

namespace lbm {

// Many independent lattices (each with its own size, parameters and
// buffers) advanced by one persistent launch.  Work item k is (instance,
// tile); each XCD's workgroups stride over its share of the work list, so
// one launch covers every instance whatever their sizes.  `parity` selects
// which of an instance's two buffers is read.
struct BatchInstance {
    StepArgs args[2];  // [parity]: fin/fout swapped
};

template <class P, int TZ, int TR, int NT, int kOpt = 0>
__global__ __launch_bounds__(NT) void axi_batch_kernel(const BatchInstance* __restrict__ insts,
                                                      const int2* __restrict__ items, int n_items, int parity) {
    // workgroups are dealt to the 8 XCDs in turn (XCD = block id mod 8), so
    // XCD x takes the contiguous eighth [x n / 8, (x + 1) n / 8) of the work
    // list: the tiles it runs together are neighbours in one instance and
    // read each other's halo rows from its own L2.  The grid is a multiple
    // of 8, so every XCD has at least one workgroup.
    const int x = blockIdx.x & 7;
    const int per = (int)(gridDim.x - x + 7) >> 3;
    const int hi = (int)(((long long)n_items * (x + 1)) >> 3);
    for (int k = (int)(((long long)n_items * x) >> 3) + (blockIdx.x >> 3); k < hi; k += per) {
        // the work item is uniform over the workgroup: keep it (and the
        // instance arguments it selects) in scalar registers
        const int2 w = items[k];
        const int inst = __builtin_amdgcn_readfirstlane(w.x);
        const int tile = __builtin_amdgcn_readfirstlane(w.y);
        const StepArgs a = insts[inst].args[parity];
        // the thread index passes through an empty asm on every item, so
        // the values the tile body derives from it (window coordinates, LDS
        // addresses) are formed per item instead of being hoisted out of the
        // loop and held in registers across it (FP32 64 x 16 / 512 threads:
        // 124 -> 76 VGPRs, 2 -> 3 workgroups per CU)
        int t = threadIdx.x;
        asm volatile("" : "+v"(t));
        // FP32 stores device scope, as on a single large lattice (41.4 ->
        // 42.1 GLUPS on a 256-instance ensemble)
        tile_body<P, TZ, TR, NT, false, kOpt, sizeof(typename P::S) == 4 ? 16 : 0>(a, tile, 0, t);
        __syncthreads();  // the next item reuses the LDS windows
    }
}

}  // namespace lbm
