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
// (2 x 2 fragments of v_mfma_f64_16x16x4_f64); the waves sit WM x WN x WK in
// the workgroup: WM x WN output blocks, and WK waves per block that take
// every WK-th k-step and are summed through LDS at the end (small GEMMs get
// more workgroups that way).  A and B chunks of KC complex k values are
// staged through LDS as separate Re/Im planes, [k][m] and [k][n], so a
// fragment read is 16 consecutive doubles per k row; the next chunk's global
// loads are in flight while the current one is multiplied.  A complex
// product is four real MFMAs (Re += ar br - ai bi, Im += ar bi + ai br); the
// FP64 MFMA takes 64 cycles, so the staging work is far below the matrix
// time.
#include <cmath>
#include <cstdlib>
#include <type_traits>

#include "bb_internal.h"

namespace bb {
namespace zg {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef double d2_t __attribute__((ext_vector_type(2)));

// Complex k values per staged chunk: 16 (four MFMA k-steps, one per k-group
// wave) for WK = 4, else 8 (two k-steps); smaller chunks keep more
// workgroups resident.
constexpr int chunk_k(int WK) { return WK == 4 ? 16 : 8; }

template <int WM, int WN, int WK>
struct Tile {
    static constexpr int KC = chunk_k(WK);
    static constexpr int KSTEPS = KC / 4 / WK;  // MFMA k-steps per wave per chunk
    static constexpr int TM = 32 * WM, TN = 32 * WN;
    static constexpr int AE = TM * KC / THREADS;  // A elements per thread per chunk
    static constexpr int BE = TN * KC / THREADS;
    static constexpr int A_BYTES = 2 * 2 * KC * TM * 8;  // [buffer][re/im][k][m]
    static constexpr int B_BYTES = 2 * 2 * KC * TN * 8;
    static constexpr int RED_BYTES = WK > 1 ? WM * WN * 64 * 32 * 8 : 0;  // one partial per output block
    static constexpr int LDS = A_BYTES + B_BYTES > RED_BYTES ? A_BYTES + B_BYTES : RED_BYTES;
    static_assert(WM * WN * WK == 4, "four waves");
    static_assert(KSTEPS >= 1 && KSTEPS * 4 * WK == KC, "k-steps per chunk split evenly");
    static_assert(AE >= 1 && BE >= 1, "tile too small for the thread count");
};

__device__ __forceinline__ long long batch_off(const BatchOff &o, int b)
{
    return (long long)((b / o.d0) % o.m0) * o.s0 + (long long)((b / o.d1) % o.m1) * o.s1;
}

template <int WM, int WN, int WK>
__global__ void __launch_bounds__(THREADS, 2) zgemm(ZgemmArgs a)
{
    using T = Tile<WM, WN, WK>;
    constexpr int TM = T::TM, TN = T::TN, KC = T::KC;
    __shared__ __align__(16) unsigned char smem[T::LDS];
    auto As = reinterpret_cast<double (*)[2][KC][TM]>(smem);                // [buffer][re/im][k][m]
    auto Bs = reinterpret_cast<double (*)[2][KC][TN]>(smem + T::A_BYTES);  // [buffer][re/im][k][n]

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = (wave / WM) % WN, wk = wave / (WM * WN);

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

    const d2_t *A = reinterpret_cast<const d2_t *>(a.A) + batch_off(a.a_b, b);
    const d2_t *B = reinterpret_cast<const d2_t *>(a.B) + batch_off(a.b_b, b);
    const long long c_base = batch_off(a.c_b, b);

    // Element -> (row, k) of the loads: k fastest when k is the contiguous
    // axis of the operand, the row (column) fastest otherwise.  Two register
    // sets: the loads of chunk c + 2 are in flight while chunk c is
    // multiplied and chunk c + 1 is written to LDS.
    const bool a_kfast = a.a_sk == 1, b_kfast = a.b_sk == 1 && a.b_sn != 1;
    d2_t ra[2][T::AE], rb[2][T::BE];
    auto load = [&](auto set, int k0) {
        constexpr int S = decltype(set)::value;
#pragma unroll
        for (int j = 0; j < T::AE; ++j) {
            const int e = tid + THREADS * j;
            const int m = a_kfast ? e / KC : e % TM, k = a_kfast ? e % KC : e / TM;
            const int gm = m0 + m, gk = k0 + k;
            ra[S][j] = gm < a.M && gk < a.K ? A[(long long)gm * a.a_sm + (long long)gk * a.a_sk] : d2_t{0.0, 0.0};
        }
#pragma unroll
        for (int j = 0; j < T::BE; ++j) {
            const int e = tid + THREADS * j;
            const int n = b_kfast ? e / KC : e % TN, k = b_kfast ? e % KC : e / TN;
            const int gn = n0 + n, gk = k0 + k;
            rb[S][j] = gn < a.N && gk < a.K ? B[(long long)gk * a.b_sk + (long long)gn * a.b_sn] : d2_t{0.0, 0.0};
        }
    };
    auto store = [&](auto set, int buf) {
        constexpr int S = decltype(set)::value;
#pragma unroll
        for (int j = 0; j < T::AE; ++j) {
            const int e = tid + THREADS * j;
            const int m = a_kfast ? e / KC : e % TM, k = a_kfast ? e % KC : e / TM;
            As[buf][0][k][m] = ra[S][j].x;
            As[buf][1][k][m] = ra[S][j].y;
        }
#pragma unroll
        for (int j = 0; j < T::BE; ++j) {
            const int e = tid + THREADS * j;
            const int n = b_kfast ? e / KC : e % TN, k = b_kfast ? e % KC : e / TN;
            Bs[buf][0][k][n] = rb[S][j].x;
            Bs[buf][1][k][n] = rb[S][j].y;
        }
    };

    d4_t cr[2][2], ci[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) cr[i][j] = ci[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

    // Fragment operands: A(row, k) from lane row + 16 k, B(k, col) from lane col + 16 k.
    const int fr = lane & 15, fk = lane >> 4;
    auto multiply = [&](int buf) {
#pragma unroll
        for (int j = 0; j < T::KSTEPS; ++j) {
            const int k = 4 * (wk + WK * j) + fk;
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
                for (int jj = 0; jj < 2; ++jj) {
                    cr[i][jj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[jj], cr[i][jj], 0, 0, 0);
                    cr[i][jj] = __builtin_amdgcn_mfma_f64_16x16x4f64(nai[i], bi[jj], cr[i][jj], 0, 0, 0);
                    ci[i][jj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi[jj], ci[i][jj], 0, 0, 0);
                    ci[i][jj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br[jj], ci[i][jj], 0, 0, 0);
                }
        }
    };
    using S0 = std::integral_constant<int, 0>;
    using S1 = std::integral_constant<int, 1>;
    const int n_chunks = (a.K + KC - 1) / KC;
    load(S0{}, 0);
    store(S0{}, 0);
    if (n_chunks > 1) load(S1{}, KC);
    if (n_chunks > 2) load(S0{}, 2 * KC);
    __syncthreads();
    // Chunk c: LDS buffer c & 1; its successor's registers are set (c + 1) & 1,
    // which then takes chunk c + 3.
    auto step = [&](auto par, int c) {
        constexpr int P = decltype(par)::value;
        using Next = std::integral_constant<int, P ^ 1>;
        multiply(P);
        if (c + 1 < n_chunks) store(Next{}, P ^ 1);
        if (c + 3 < n_chunks) load(Next{}, (c + 3) * KC);
        __syncthreads();
    };
    int c = 0;
    for (; c + 2 <= n_chunks; c += 2) {
        step(S0{}, c);
        step(S1{}, c + 1);
    }
    if (c < n_chunks) step(S0{}, c);

    // Sum of the WK partial blocks, in order of wk (the staging buffers are
    // free after the loop's last barrier): wave wk > 0 posts its partial, the
    // wk = 0 wave of the same block adds it.
    if constexpr (WK > 1) {
        d2_t *red = reinterpret_cast<d2_t *>(smem) + (wm + WM * wn) * 64 * 16 + lane;
        for (int r = 1; r < WK; ++r) {
            if (wk == r) {
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int jj = 0; jj < 2; ++jj)
#pragma unroll
                        for (int e = 0; e < 4; ++e) red[64 * ((i * 2 + jj) * 4 + e)] = d2_t{cr[i][jj][e], ci[i][jj][e]};
            }
            __syncthreads();
            if (wk == 0) {
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int jj = 0; jj < 2; ++jj)
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const d2_t v = red[64 * ((i * 2 + jj) * 4 + e)];
                            cr[i][jj][e] += v.x;
                            ci[i][jj][e] += v.y;
                        }
            }
            __syncthreads();
        }
        if (wk != 0) return;
    }

    // Accumulator register r of a 16x16 f64 fragment holds (row 4 r + lane / 16, col lane % 16).
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm * 32 + i * 16 + 4 * r + fk;
                const int gn = n0 + wn * 32 + jj * 16 + fr;
                if (gm >= a.M || gn >= a.N) continue;
                const long long off = c_base + (long long)gm * a.c_sm +
                                      (long long)(gn / a.c_ng) * a.c_sg + (long long)(gn % a.c_ng) * a.c_sn;
                if (a.c_c64)
                    reinterpret_cast<float2 *>(a.C)[off] = make_float2((float)cr[i][jj][r], (float)ci[i][jj][r]);
                else
                    reinterpret_cast<d2_t *>(a.C)[off] = d2_t{cr[i][jj][r], ci[i][jj][r]};
            }
}

template <int WM, int WN, int WK>
hipError_t run(ZgemmArgs a, hipStream_t st)
{
    using T = Tile<WM, WN, WK>;
    a.tiles_m = (a.M + T::TM - 1) / T::TM;
    a.tiles_n = (a.N + T::TN - 1) / T::TN;
    const long long grid = (long long)a.batch * a.tiles_m * a.tiles_n;
    if (grid <= 0 || grid > 0x7fffffffLL) return hipErrorInvalidValue;
    zgemm<WM, WN, WK><<<dim3((unsigned)grid), dim3(THREADS), 0, st>>>(a);
    return hipGetLastError();
}

// Wave layouts (WM, WN, WK), in order of preference on equal estimates.
constexpr int SHAPES[6][3] = {{2, 2, 1}, {1, 4, 1}, {4, 1, 1}, {1, 2, 2}, {2, 1, 2}, {1, 1, 4}};

}  // namespace zg

// The layout with the fewest MFMA k-steps per SIMD: k-steps per wave
// (ceil(K / 4) / WK) times the rounds of one wave per SIMD the grid needs
// (4 waves per workgroup, 1024 SIMDs).
int zgemm_shape(int M, int N, int K, int batch)
{
    int best = 0;
    double best_est = 0.0;
    for (int i = 0; i < 6; ++i) {
        const int WM = zg::SHAPES[i][0], WN = zg::SHAPES[i][1], WK = zg::SHAPES[i][2];
        const double wgs = (double)batch * ((M + 32 * WM - 1) / (32 * WM)) * ((N + 32 * WN - 1) / (32 * WN));
        const double rounds = std::ceil(wgs * 4.0 / 1024.0);
        const double est = std::ceil((K + 3) / 4 / (double)WK) * rounds;
        if (i == 0 || est < best_est) {
            best = i;
            best_est = est;
        }
    }
    return best;
}

hipError_t launch_zgemm(const ZgemmArgs &a, hipStream_t st)
{
    if (a.M < 1 || a.N < 1 || a.K < 1 || a.batch < 1 || a.c_ng < 1) return hipErrorInvalidValue;
    int layout = zgemm_shape(a.M, a.N, a.K, a.batch);
    if (const char *f = std::getenv("BBLOCK_ZGEMM_LAYOUT")) {  // forced layout 0..5 (tests, tuning)
        const int v = std::atoi(f);
        if (v >= 0 && v < 6) layout = v;
    }
    switch (layout) {
    case 0: return zg::run<2, 2, 1>(a, st);
    case 1: return zg::run<1, 4, 1>(a, st);
    case 2: return zg::run<4, 1, 1>(a, st);
    case 3: return zg::run<1, 2, 2>(a, st);
    case 4: return zg::run<2, 1, 2>(a, st);
    default: return zg::run<1, 1, 4>(a, st);
    }
}

}  // namespace bb
