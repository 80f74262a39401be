// Internal types and device helpers shared by the host API (bb_api.hip) and
// the HIP kernels of libbblock.so: the block descriptor, launch arguments and
// the helpers every contraction kernel uses.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <type_traits>

namespace bb {

enum Prec : int { FP64 = 0, FP32 = 1, BF16X3 = 2 };

// Sites per generation chunk.  Each chunk contributes 3 * CHUNK_SITES values
// of the contraction index kappa = (colour, site) to the GEMM.
constexpr int CHUNK_SITES = 8;
constexpr int CHUNK_KAPPA = 3 * CHUNK_SITES;
constexpr int THREADS = 256;  // four wave64 per workgroup
constexpr int MAX_MOM = 128;
constexpr int MAX_MODES = 4096;  // eigenvectors or coefficient rows of the LapH-subspace entry points
constexpr int MAX_L = 256;

// A value every lane of the wave holds alike, moved to scalar registers
// (loads of the tile tables are vector loads; the compiler cannot tell on its
// own), so that buffer resources built from it need no waterfall loop.
template <class T>
__device__ __forceinline__ T wave_uniform(const T &v)
{
    static_assert(sizeof(T) % 4 == 0, "word-sized fields only");
    struct Words {
        uint32_t w[sizeof(T) / 4];
    };
    Words x = __builtin_bit_cast(Words, v);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) x.w[i] = __builtin_amdgcn_readfirstlane(x.w[i]);
    return __builtin_bit_cast(T, x);
}

// One baryon block as the kernels see it (device resident table).
struct BlockDesc {
    const void *q1, *q2, *q3;  // [V][3][n_i] complex (c128 or c64)
    double *out;               // [n_mom][n1][n2][n3] complex128
    void *ws;                  // split-K partials [S][2][M][N] (float or double), null if direct
    int n1, n2, n3;
    int M, N;                  // M = n1*n2 rows (d1,d2); N = n3*n_mom columns (p,d3)
    int S;                     // number of site splits
    int sps;                   // sites per split (multiple of CHUNK_SITES)
    // Rectangular tiles of the pipelined kernel: m-tile = (d1 block) x (d2
    // block), n-tile = (momentum block of bp momenta) x (d3 block).
    int n_mt2;                 // d2 blocks
    int n_nt3;                 // d3 blocks
    int bp;                    // momenta per n-tile
    int b3;                    // d3 per n-tile
    // W images of the precomputed-W kernel: [split - img_s0][n-tile][chunk],
    // one image per n-tile and chunk; null for the other kernels.  A block
    // whose images exceed the workspace runs in rounds of consecutive splits
    // (one descriptor per round, img_s0 = the round's first split).
    void *wimg;
    int cps;                   // chunks per split
    int n_nt;                  // n-tiles
    int img_s0;
    int direct;                // 1: one split, the kernel writes out itself; 0: partials in ws
    int walk;                  // 1: the workgroup of a tile runs all S splits in order and sums them into out
};

// One element of a tile's result: part 0 (real) or 1 (imaginary) of
// B[p][m][d3] (m = d1 n2 + d2, column nu = p n3 + d3) from site split s.
//   PUT_STORE (one split, or the first split of a walking tile): written to
//     out;
//   PUT_ADD (a later split of a walking tile, whose workgroup runs every
//     split in order): added to out in FP64 -- the same sums in the same
//     order as the split-K reduction of partials (Algorithm 1 sums the site
//     blocks into tmpBuf the same way), so the block is bitwise the one the
//     reduction would give;
//   PUT_PARTIAL: stored as split s's partial for the reduction kernel.
// The add is a returnless FP64 atomic: each element has one writer (one lane
// of one workgroup, splits in program order with a barrier between them), so
// the adds apply in split order with IEEE round-to-nearest, exactly as a
// load, add and store would -- but without a load whose latency would
// serialise the epilogue.
enum PutMode : int { PUT_PARTIAL = 0, PUT_STORE = 1, PUT_ADD = 2 };

template <int MODE, class PartT>
__device__ __forceinline__ void put_result(const BlockDesc &bd, int s, int m, int nu, int p, int d3, int part, double v)
{
    if constexpr (MODE == PUT_PARTIAL) {
        reinterpret_cast<PartT *>(bd.ws)[(((size_t)s * 2 + part) * bd.M + m) * bd.N + nu] = (PartT)v;
    } else {
        double *o = bd.out + (((size_t)p * bd.M + m) * bd.n3 + d3) * 2 + part;
        if constexpr (MODE == PUT_ADD)
            (void)unsafeAtomicAdd(o, v);
        else
            *o = v;
    }
}

// Runs the epilogue f with the tile's write mode as a compile-time constant
// (f(std::integral_constant<int, mode>)): one copy of the epilogue per mode,
// chosen by a wave-uniform branch, instead of a three-way branch per element
// inside divergent code, which keeps values of all three paths live and
// pushes the accumulators out of the register file.
template <class F>
__device__ __forceinline__ void with_put_mode(const BlockDesc &bd, int s, F &&f)
{
    if (bd.walk && s > 0)
        f(std::integral_constant<int, PUT_ADD>{});
    else if (bd.direct || bd.walk)
        f(std::integral_constant<int, PUT_STORE>{});
    else
        f(std::integral_constant<int, PUT_PARTIAL>{});
}

// Arguments of one grouped GEMM launch.
struct GemmArgs {
    const BlockDesc *blocks;
    const int4 *tiles;   // (block, m-tile, n-tile, split), cost-sorted
    int n_tiles;
    int *counter;        // [2] persistent work counter and exit counter; null = one tile per workgroup
    const int *mom;      // [n_mom][3]
    int n_mom;
    int L, V;
    int in_c64;
    const double *roots; // [L] complex128 exp(-2 pi i k / L)
    const unsigned char *kidx;  // [n_mom][kstride] phase index (n_p . x) mod L (pipelined, paper-order)
    int kstride;                // row stride of kidx: V rounded up to a multiple of 4 (padding reads 0)
    // Paper-order FP64/FP32 kernels: index of a zero momentum whose
    // projection (a plain sum over sites: its phase is 1) they form on the
    // vector unit, its column left out of the MFMA tiles; -1 for none.
    int p_skip;
};

// Arguments of the W-image launch of the precomputed-W kernel.
struct WImageArgs {
    const BlockDesc *blocks;
    const int4 *entries;  // (block, n-tile, split, 0)
    int n_entries;
    const int *mom;       // [n_mom][3], reduced mod L
    int n_mom;
    int L, V;
    const double *roots;  // [L] complex128 exp(-2 pi i k / L)
};

// Combination of blocks into outputs (spin projection): output group g sums
// c_i * B_i over the members i in [gstart[g], gstart[g+1]) of list, in that
// order; accumulate[g] = 1 adds to what an earlier launch wrote.
struct CombineArgs {
    const BlockDesc *blocks;
    const int *list;      // member block indices
    const double *coef;   // [n_list][2] complex coefficient per member
    const int *gstart;    // [n_groups + 1]
    const int *accumulate;  // [n_groups]
    int n_groups;
};

struct ReduceArgs {
    const BlockDesc *blocks;
    const int *list;     // indices of blocks with S > 1
    int n_list;
};

// Offset of batch entry b of one GEMM operand, in complex elements: two
// terms ((b / d) % m) * s, so that an operand can run with the whole batch
// index, with an outer part of it only, or stay fixed (s = 0).
struct BatchOff {
    long long s0 = 0, s1 = 0;
    int d0 = 1, m0 = 0x7fffffff, d1 = 1, m1 = 1;
};
inline BatchOff batch_uniform(long long s)
{
    BatchOff o;
    o.s0 = s;
    return o;
}

// Strided batched complex double GEMM on the FP64 matrix cores:
// C[b](m, n) = sum_k A[b](m, k) B[b](k, n).  Strides count complex elements;
// column n of C lives at (n / c_ng) * c_sg + (n % c_ng) * c_sn.
struct ZgemmArgs {
    const double *A;                 // complex128
    long long a_sm, a_sk;
    BatchOff a_b;
    const double *B;                 // complex128
    long long b_sk, b_sn;
    BatchOff b_b;
    void *C;                         // complex128, or complex64 when c_c64
    long long c_sm, c_sn, c_sg;
    BatchOff c_b;
    int c_ng, c_c64;
    int M, N, K, batch;
    int tiles_m, tiles_n;            // set by the launcher
};

}  // namespace bb

// Host-side launch and geometry entry points of the kernels.
#include "bb_launch.h"
