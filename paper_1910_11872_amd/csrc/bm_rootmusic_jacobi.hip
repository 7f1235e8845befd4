// Launchers of the root-MUSIC kernels with the cyclic Jacobi eigen-split
// (BM_OPT_JACOBI) for line windows and block windows up to 8 x 8: their own
// translation unit, so that they compile alongside the default ones.
#include "bm_rootmusic_kernels.h"

namespace bm {

hipError_t launch_rootmusic_jacobi(int L, const RmBatch& b, int block, int grid, hipStream_t s) {
    return launch_rootmusic_J<true>(L, b, block, grid, s);
}

}  // namespace bm
