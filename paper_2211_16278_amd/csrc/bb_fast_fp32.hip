// FP32 instantiations of the pipelined contraction kernel (bb_fast.h), the
// kidx phase-index table kernel, and the dispatch of the pipelined path.
#include "bb_fast.h"

namespace bb {
hipError_t launch_fast_bf16(int nb, int b2, int b3, int c64, const GemmArgs &a, int grid, hipStream_t st);
hipError_t prepare_fast_bf16(int bytes);

int fast_lds_bytes(int prec, int nb, int b2, int b3, int L)
{
    if (prec != FP32 && prec != BF16X3) return -1;
    return fast::lds_bytes(nb, b2, b3, L);
}

hipError_t launch_fast(int prec, int nb, int b2, int b3, int in_c64, const GemmArgs &a, int grid, hipStream_t st)
{
    if (prec == BF16X3) return launch_fast_bf16(nb, b2, b3, in_c64, a, grid, st);
    if (prec == FP32) return fast::Launcher<FP32>::launch(nb, b2, b3, in_c64, a, grid, st);
    return hipErrorInvalidValue;
}

hipError_t prepare_fast_kernels(int bytes)
{
    hipError_t e = fast::Launcher<FP32>::prepare(bytes);
    hipError_t f = prepare_fast_bf16(bytes);
    return e != hipSuccess ? e : f;
}

// kidx[p][x] = (n_p . x) mod L, x = ix + L (iy + L iz); momenta reduced to [0, L).
__global__ void bb_phase_index(const int *mom, int n_mom, int L, int kstride, unsigned char *kidx)
{
    const int V = L * L * L;
    const size_t total = (size_t)n_mom * kstride;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const int p = (int)(i / kstride), x = (int)(i - (size_t)p * kstride);
        const int ix = x % L, iy = (x / L) % L, iz = x / (L * L);
        kidx[i] = x < V ? (unsigned char)((mom[3 * p] * ix + mom[3 * p + 1] * iy + mom[3 * p + 2] * iz) % L) : 0;
    }
}

hipError_t launch_phase_index(const int *mom, int n_mom, int L, int kstride, unsigned char *kidx, hipStream_t st)
{
    const size_t total = (size_t)n_mom * kstride;
    const int grid = (int)std::min<size_t>(4096, (total + 255) / 256);
    hipLaunchKernelGGL(bb_phase_index, dim3(grid), dim3(256), 0, st, mom, n_mom, L, kstride, kidx);
    return hipGetLastError();
}
}  // namespace bb
