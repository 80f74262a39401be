// Host-side entry points of the kernels of libbblock.so: geometry queries
// and launch functions, each defined next to its kernel.  Not part of the
// public ABI.  Declarations only: nothing here changes the code of a kernel.
#pragma once

#include "bb_internal.h"

namespace bb {

// Geometry of one kernel instantiation.
struct KernelGeom {
    int m_tile;       // complex rows (d1,d2) per workgroup
    int frag_cols;    // columns per MFMA fragment
    int lds_bytes;    // dynamic LDS for (nb, n_mom, L)
};

// Column fragments per wave available for each precision.
int nb_options(int prec, const int **list);
KernelGeom kernel_geom(int prec, int nb, int n_mom, int L);

hipError_t launch_gemm(int prec, int nb, const GemmArgs &a, int grid, hipStream_t st);

// Pipelined kernel (FP32 and BF16X3; d2 and d3 blocks of 16 or 32).
// Returns the dynamic LDS bytes, or -1 when no instantiation exists.
int fast_lds_bytes(int prec, int nb, int b2, int b3, int L);
hipError_t launch_fast(int prec, int nb, int b2, int b3, int in_c64, const GemmArgs &a, int grid, hipStream_t st);
hipError_t prepare_fast_kernels(int lds_bytes);
// kidx[p][x] = (n_p . x) mod L for all sites of one timeslice (momenta already
// in [0, L)), rows of kstride >= V bytes, 0 past V.
hipError_t launch_phase_index(const int *mom, int n_mom, int L, int kstride, unsigned char *kidx, hipStream_t st);
// Precomputed-W kernel (BF16X3; d2 blocks of 8, 16 or 32, nb 4 to 7): static
// LDS bytes (-1 when no instantiation), bytes per W image, launches.  The
// contraction runs with 4 waves per workgroup (one per SIMD) or 8 (two per
// SIMD, the column fragments split between the two).
int w3_lds_bytes(int nb, int b2);
size_t w3_image_bytes(int nb);
hipError_t launch_w3_image(int nb, int c64, const WImageArgs &a, int cps_max, hipStream_t st);
hipError_t launch_w3(int nb, int b2, int waves, int c64, const GemmArgs &a, int grid, hipStream_t st);
// Paper-order kernel (BF16X3; singlet on the VALU, momentum GEMM on MFMA;
// nb column fragments of 32 momenta, d3 blocks of 16 or 32): (d1,d2) pairs
// per workgroup (-1 when no instantiation), launch.  Its tiles use
// BlockDesc.n_mt2 for the number of d3 blocks.
int pord_pairs(int nb, int b3);
hipError_t launch_pord(int nb, int b3, int c64, const GemmArgs &a, int grid, hipStream_t st);
// FP64 kernel (plan kernel 5): eight waves per workgroup, each running the
// three-product complex GEMM of 16 rows on the matrix cores and building its
// share of the next chunk's D and W tiles; 128 complex rows x 16 cf columns
// per tile (cf 2, 4 or 7).  Static LDS bytes (-1 when no instantiation),
// launch.
int f64_lds_bytes(int cf);
hipError_t launch_f64(int cf, int c64, const GemmArgs &a, int grid, hipStream_t st);
// FP64 paper-order kernels 6 and 8: the singlet on the vector unit in the
// MFMA operand layout, the momentum projection as a three-product complex
// GEMM on the matrix cores; tiles of 128 rows ((d1,d2) pairs x a d3 block of
// 16) per row set of 16 rows a wave holds, w cf momenta: kernel 6 w = 16 on
// v_mfma_f64_16x16x4_f64 (cf 1 to 3, f64p_row_sets(cf) row sets), kernel 8
// w = 4 on v_mfma_f64_4x4x4_f64 (cf 1 to 4, F64N_ROW_SETS row sets).  Static
// LDS bytes and pairs per tile (-1 when no instantiation), launches.  Their
// tiles use BlockDesc.n_mt2 for the number of d3 blocks.
constexpr int F64N_ROW_SETS = 2;
// Two row sets up to two fragments of 16 (at three they spill).
constexpr int f64p_row_sets(int cf) { return cf <= 2 ? 2 : 1; }
int f64p_lds_bytes(int cf, int b3, int w);
int f64p_pairs(int cf, int b3, int w);
hipError_t launch_f64p(int cf, int b3, int c64, const GemmArgs &a, int grid, hipStream_t st);
hipError_t launch_f64n(int cf, int b3, int c64, const GemmArgs &a, int grid, hipStream_t st);
// FP32 paper-order kernels (plan kernels 7 and 9): kernel 6's design in
// single precision, the momentum projection on v_mfma_f32_16x16x4_f32
// (kernel 7, 16 cf momenta per tile) or v_mfma_f32_4x4x1_16b_f32 (kernel 9,
// 4 cf), three real products up to cf 2, else four, chunks of 32 sites
// (cf 1 to 4).  Static LDS bytes and pairs per tile (-1 when no
// instantiation), launch.
int f32p_lds_bytes(int cf, int b3, int w);  // w: momenta per fragment, 16 (kernel 7) or 4 (kernel 9)
int f32p_pairs(int b3);
int f32p_wgs(int cf, int b3, int w);  // workgroups of kernels 7 and 9 per CU
hipError_t launch_f32p(int cf, int b3, int c64, const GemmArgs &a, int grid, hipStream_t st);
hipError_t launch_f32n(int cf, int c64, const GemmArgs &a, int grid, hipStream_t st);  // kernel 9: d3 blocks of 16
int zgemm_shape(int M, int N, int K, int batch);  // index of the wave layout a launch uses
hipError_t launch_zgemm(const ZgemmArgs &a, hipStream_t st);
hipError_t launch_reduce(int prec, const ReduceArgs &a, int max_mn, hipStream_t st);
hipError_t launch_combine(int prec, const CombineArgs &a, int max_mn, hipStream_t st);
hipError_t prepare_kernels(int lds_bytes);  // dynamic-LDS limit of every contraction kernel

}  // namespace bb
