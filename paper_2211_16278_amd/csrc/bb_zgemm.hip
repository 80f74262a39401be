// Complex double GEMM on the FP64 matrix cores (gfx950), strided and batched:
//
//     C[b](m, n) = sum_k A[b](m, k) B[b](k, n)
//
// It carries the two LapH-subspace steps around the baryon block (paper,
// Sec. 2): the quark-field reconstruction of eq. (2) (one GEMM over all sites
// and colours, M = 3V, N = coefficient rows, K = eigenvectors) and the
// contraction of quark-field coefficients onto the mode triplets of eq. (4)
// (three GEMMs, one per eigenvector index).  Operands are complex128 with
// arbitrary element strides; C is stored as complex128 or complex64, with an
// optional grouping of columns (column n goes to group n / c_ng at stride
// c_sg, position n % c_ng inside it) so that several coefficient sets can
// share one pass over the eigenvectors.
//
// Tiling: 256 threads = 4 waves, each wave owns 32 x 32 complex outputs
// (2 x 2 fragments of v_mfma_f64_16x16x4_f64); the waves sit WM x WN in the
// workgroup tile.  A and B chunks of KC complex k values are staged through
// LDS as separate Re/Im planes, [k][m] and [k][n], so a fragment read is 16
// consecutive doubles per k row; the next chunk's global loads are in flight
// while the current one is multiplied.  A complex product is four real MFMAs
// (Re += ar br - ai bi, Im += ar bi + ai br); the FP64 MFMA takes 64 cycles,
// so the staging work is far below the matrix time.
#include "bb_internal.h"

namespace bb {
namespace zg {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef double d2_t __attribute__((ext_vector_type(2)));

constexpr int KC = 8;  // complex k values per staged chunk (2 MFMA k-steps)

template <int WM, int WN>
struct Tile {
    static constexpr int TM = 32 * WM, TN = 32 * WN;
    static constexpr int AE = TM * KC / THREADS;  // A elements per thread per chunk
    static constexpr int BE = TN * KC / THREADS;
    static_assert(WM * WN == 4, "four waves");
    static_assert(AE >= 1 && BE >= 1, "tile too small for the thread count");
};

template <int WM, int WN>
__global__ void __launch_bounds__(THREADS, 2) zgemm(ZgemmArgs a)
{
    using T = Tile<WM, WN>;
    constexpr int TM = T::TM, TN = T::TN;
    __shared__ __align__(16) double As[2][2][KC][TM];  // [buffer][re/im][k][m]
    __shared__ __align__(16) double Bs[2][2][KC][TN];  // [buffer][re/im][k][n]

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;

    // Workgroup -> (batch, m-tile, n-tile).  Consecutive workgroups go to
    // different XCDs; the remap gives each XCD a contiguous range of tiles so
    // that the n-tiles sharing an A tile share an L2.
    const long long total = (long long)a.batch * a.tiles_m * a.tiles_n;
    long long bid = blockIdx.x;
    if (total % 8 == 0) bid = (bid % 8) * (total / 8) + bid / 8;
    const int per_b = a.tiles_m * a.tiles_n;
    const int b = (int)(bid / per_b);
    const int t = (int)(bid % per_b);
    const int m0 = (t % a.tiles_m) * TM, n0 = (t / a.tiles_m) * TN;

    const d2_t *A = reinterpret_cast<const d2_t *>(a.A) + (long long)b * a.a_sb;
    const d2_t *B = reinterpret_cast<const d2_t *>(a.B) + (long long)b * a.b_sb;

    // Element -> (row, k) of the loads: k fastest when k is the contiguous
    // axis of the operand, the row (column) fastest otherwise.
    const bool a_kfast = a.a_sk == 1, b_kfast = a.b_sk == 1 && a.b_sn != 1;
    d2_t ra[T::AE], rb[T::BE];
    auto load = [&](int k0) {
#pragma unroll
        for (int j = 0; j < T::AE; ++j) {
            const int e = tid + THREADS * j;
            const int m = a_kfast ? e / KC : e % TM, k = a_kfast ? e % KC : e / TM;
            const int gm = m0 + m, gk = k0 + k;
            ra[j] = gm < a.M && gk < a.K ? A[(long long)gm * a.a_sm + (long long)gk * a.a_sk] : d2_t{0.0, 0.0};
        }
#pragma unroll
        for (int j = 0; j < T::BE; ++j) {
            const int e = tid + THREADS * j;
            const int n = b_kfast ? e / KC : e % TN, k = b_kfast ? e % KC : e / TN;
            const int gn = n0 + n, gk = k0 + k;
            rb[j] = gn < a.N && gk < a.K ? B[(long long)gk * a.b_sk + (long long)gn * a.b_sn] : d2_t{0.0, 0.0};
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int j = 0; j < T::AE; ++j) {
            const int e = tid + THREADS * j;
            const int m = a_kfast ? e / KC : e % TM, k = a_kfast ? e % KC : e / TM;
            As[buf][0][k][m] = ra[j].x;
            As[buf][1][k][m] = ra[j].y;
        }
#pragma unroll
        for (int j = 0; j < T::BE; ++j) {
            const int e = tid + THREADS * j;
            const int n = b_kfast ? e / KC : e % TN, k = b_kfast ? e % KC : e / TN;
            Bs[buf][0][k][n] = rb[j].x;
            Bs[buf][1][k][n] = rb[j].y;
        }
    };

    d4_t cr[2][2], ci[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) cr[i][j] = ci[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

    // Fragment operands: A(row, k) from lane row + 16 k, B(k, col) from lane col + 16 k.
    const int fr = lane & 15, fk = lane >> 4;
    const int n_chunks = (a.K + KC - 1) / KC;
    load(0);
    store(0);
    __syncthreads();
    for (int c = 0; c < n_chunks; ++c) {
        const int buf = c & 1;
        if (c + 1 < n_chunks) load((c + 1) * KC);
#pragma unroll
        for (int ks = 0; ks < KC / 4; ++ks) {
            const int k = 4 * ks + fk;
            double ar[2], ai[2], nai[2], br[2], bi[2];
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                const int m = wm * 32 + f * 16 + fr, n = wn * 32 + f * 16 + fr;
                ar[f] = As[buf][0][k][m];
                ai[f] = As[buf][1][k][m];
                nai[f] = -ai[f];
                br[f] = Bs[buf][0][k][n];
                bi[f] = Bs[buf][1][k][n];
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], cr[i][j], 0, 0, 0);
                    cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(nai[i], bi[j], cr[i][j], 0, 0, 0);
                    ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi[j], ci[i][j], 0, 0, 0);
                    ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br[j], ci[i][j], 0, 0, 0);
                }
        }
        if (c + 1 < n_chunks) store(buf ^ 1);
        __syncthreads();
    }

    // Accumulator register r of a 16x16 f64 fragment holds (row 4 r + lane / 16, col lane % 16).
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm * 32 + i * 16 + 4 * r + fk;
                const int gn = n0 + wn * 32 + j * 16 + fr;
                if (gm >= a.M || gn >= a.N) continue;
                const long long off = (long long)b * a.c_sb + (long long)gm * a.c_sm +
                                      (long long)(gn / a.c_ng) * a.c_sg + (long long)(gn % a.c_ng) * a.c_sn;
                if (a.c_c64)
                    reinterpret_cast<float2 *>(a.C)[off] = make_float2((float)cr[i][j][r], (float)ci[i][j][r]);
                else
                    reinterpret_cast<d2_t *>(a.C)[off] = d2_t{cr[i][j][r], ci[i][j][r]};
            }
}

template <int WM, int WN>
hipError_t run(ZgemmArgs a, hipStream_t st)
{
    using T = Tile<WM, WN>;
    a.tiles_m = (a.M + T::TM - 1) / T::TM;
    a.tiles_n = (a.N + T::TN - 1) / T::TN;
    const long long grid = (long long)a.batch * a.tiles_m * a.tiles_n;
    if (grid <= 0 || grid > 0x7fffffffLL) return hipErrorInvalidValue;
    zgemm<WM, WN><<<dim3((unsigned)grid), dim3(THREADS), 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace zg

int zgemm_shape(int M, int N)
{
    if (M <= 32 && N > 32) return 0;  // 32 x 128 tiles
    if (N <= 32 && M > 32) return 2;  // 128 x 32 tiles
    return 1;                         // 64 x 64 tiles
}

hipError_t launch_zgemm(const ZgemmArgs &a, hipStream_t st)
{
    if (a.M < 1 || a.N < 1 || a.K < 1 || a.batch < 1 || a.c_ng < 1) return hipErrorInvalidValue;
    switch (zgemm_shape(a.M, a.N)) {
    case 0: return zg::run<1, 4>(a, st);
    case 2: return zg::run<4, 1>(a, st);
    default: return zg::run<2, 2>(a, st);
    }
}

}  // namespace bb
