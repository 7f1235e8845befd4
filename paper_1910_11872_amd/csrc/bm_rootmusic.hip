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
    switch (L) {
        case 2: return launch_L<2>(b, block, grid, s);
        case 3: return launch_L<3>(b, block, grid, s);
        case 4: return launch_L<4>(b, block, grid, s);
        case 5: return launch_L<5>(b, block, grid, s);
        case 6: return launch_L<6>(b, block, grid, s);
        case 7: return launch_L<7>(b, block, grid, s);
        case 8: return launch_L<8>(b, block, grid, s);
        default: return launch_big_block_window(L, b, grid, s);
    }
}

hipError_t launch_rootmusic_gather(int L, const RmBatch& b, const int2* list, const unsigned long long* count, int grid,
                                   hipStream_t s) {
    if (grid <= 0) return hipSuccess;
    switch (L) {
        case 2: return launch_gather_L<2>(b, list, count, grid, s);
        case 3: return launch_gather_L<3>(b, list, count, grid, s);
        case 4: return launch_gather_L<4>(b, list, count, grid, s);
        case 5: return launch_gather_L<5>(b, list, count, grid, s);
        case 6: return launch_gather_L<6>(b, list, count, grid, s);
        case 7: return launch_gather_L<7>(b, list, count, grid, s);
        case 8: return launch_gather_L<8>(b, list, count, grid, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bm
