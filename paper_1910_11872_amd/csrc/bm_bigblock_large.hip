// Block windows of 15 x 15 and 17 x 17 (the paper's experimental window and
// the top of its window-size table, Sec. 3 and 4), 128 lanes per block, one
// wave per SIMD: the largest instantiations, in a translation unit of their own.
#include "bm_rootmusic_kernels.h"

namespace bm {

hipError_t launch_big_block_window_15_17(int L, const RmBatch& b, int grid, hipStream_t s) {
    switch (L) {
        case 15: return launch_big_block<15>(b, grid, s);
        case 17: return launch_big_block<17>(b, grid, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bm
