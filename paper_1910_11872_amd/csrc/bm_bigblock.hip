// Block windows above 8 x 8 (the paper's (2L+1) x (2L+1) window, Sec. 3, with
// its window-size table reaching 17 x 17): odd sizes 9 .. 17, 128 lanes per
// block, one wave per SIMD.  Their own translation unit: these instantiations
// are large (fully unrolled L x L eigen-split, degree 2L-2 polynomial, FP64
// certificate) and compile alongside the rest; 15 x 15 and 17 x 17 in
// bm_bigblock_large.hip.
#include "bm_rootmusic_kernels.h"

namespace bm {

hipError_t launch_big_block_window(int L, const RmBatch& b, int grid, hipStream_t s) {
    if (b.total <= 0 || b.njobs <= 0) return hipSuccess;
    if (grid <= 0 || grid > b.total) grid = b.total;
    switch (L) {
        case 9: return launch_big_block<9>(b, grid, s);
        case 11: return launch_big_block<11>(b, grid, s);
        case 13: return launch_big_block<13>(b, grid, s);
        case 15:
        case 17: return launch_big_block_window_15_17(L, b, grid, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bm
