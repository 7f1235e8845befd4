// Launchers of the root-MUSIC kernels for line windows and for block windows
// up to 8 x 8; the larger block windows are instantiated in bm_bigblock.hip.
#include "bm_rootmusic_kernels.h"

namespace bm {

int rootmusic_windows_per_block(int L, int block, bool line_kernel) {
    return line_kernel ? line_windows_per_block(L, block) : block - (L - 1);
}

hipError_t launch_rootmusic(int L, const RmBatch& b, int block, int grid, hipStream_t s) {
    if (b.total <= 0 || b.njobs <= 0) return hipSuccess;
    if (block != 128 && block != 256) return hipErrorInvalidValue;
    if (grid <= 0 || grid > b.total) grid = b.total;
    if (L > kMaxL) return launch_big_block_window(L, b, grid, s);
    return b.jacobi ? launch_rootmusic_jacobi(L, b, block, grid, s) : launch_rootmusic_J<false>(L, b, block, grid, s);
}

// The training labels: L = 8 only.
hipError_t launch_rootmusic_gather(int L, const RmBatch& b, const int2* list, const unsigned long long* count, int grid,
                                   hipStream_t s) {
    if (grid <= 0) return hipSuccess;
    if (L != 8) return hipErrorInvalidValue;
    return b.jacobi ? launch_gather_LJ<8, true>(b, list, count, grid, s)
                    : launch_gather_LJ<8, false>(b, list, count, grid, s);
}

}  // namespace bm
