// BF16X3 instantiations of the pipelined contraction kernel (bb_fast.h).
#include "bb_fast.h"

namespace bb {
hipError_t launch_fast_bf16(int nb, int b2, int b3, int c64, const GemmArgs &a, int grid, hipStream_t st)
{
    return fast::Launcher<BF16X3>::launch(nb, b2, b3, c64, a, grid, st);
}
hipError_t prepare_fast_bf16(int bytes) { return fast::Launcher<BF16X3>::prepare(bytes); }
}  // namespace bb
