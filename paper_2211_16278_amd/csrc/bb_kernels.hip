// HIP kernels of libbblock.so for gfx950 (MI355X).
//
// The baryon block of the paper (Sec. 2, eq. (3)),
//   B[p][d1][d2][d3] = sum_x exp(-i p.x) eps_abc q1[x][a][d1] q2[x][b][d2] q3[x][c][d3],
// is evaluated as one complex GEMM per block
//   C[(d1,d2), (p,d3)] = sum_{kappa=(c,x)} D[kappa, (d1,d2)] * W[kappa, (p,d3)]
// with the colour cross product ("diquark") D_c = eps_abc q1_a q2_b of
// Algorithm 1 (Sec. 3, the diquark loop) and the phase-weighted third quark
// W = q3_c(x, d3) exp(-i p.x).  Summing D_c q3_c over c is the singlet of
// Algorithm 1 and the sum over sites with the phase is its momentum GEMM; here
// the two are fused into one contraction over kappa = (colour, site) so that
// the whole block is a single dense GEMM on the matrix cores, with the momenta
// folded into the N dimension.
//
// Workgroup = 4 wave64.  A workgroup owns an (m-tile, n-tile, site-split) of a
// block.  Sites are streamed in chunks of CHUNK_SITES: the workgroup builds the
// chunk's D tile and W tile in LDS (never in HBM), then every wave multiplies
// its rows of D against all columns of W with MFMA.  The complex product is
// embedded in real arithmetic on the row side: real row (m, re) holds
// (Re D, -Im D) and real row (m, im) holds (Im D, Re D) against the column
// (Re W, Im W), so each output row yields Re C or Im C directly.
//
// Precision paths (template parameter P):
//   FP64   - complex double D and W, v_mfma_f64_16x16x4_f64, FP64 partials;
//   FP32   - complex float  D and W, v_mfma_f32_32x32x2_f32, FP32 partials;
//   BF16X3 - complex float  D and W split into bf16 hi + lo, three
//            v_mfma_f32_32x32x16_bf16 products (lo*hi, hi*lo, hi*hi) per
//            fragment pair, FP32 accumulation, FP32 partials.
// Partials of a split are summed in FP64 by bb_reduce (paper, Algorithm 1:
// the accumulation over site blocks into tmpBuf and the final write-out).

#include <algorithm>

#include "bb_internal.h"

namespace bb {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f16_t __attribute__((ext_vector_type(16)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf2_t __attribute__((ext_vector_type(2)));

template <class R>
struct cx {
    R re, im;
};

template <class R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

template <class R>
__device__ __forceinline__ cx<R> csub(cx<R> a, cx<R> b)
{
    return {a.re - b.re, a.im - b.im};
}

// ------------------------------------------------------------- traits ---
template <int P>
struct Tr;

template <>
struct Tr<FP64> {
    using R = double;            // arithmetic of D and W
    using E = double;            // LDS element (planes: Re, Im)
    using Acc = d4_t;            // 16x16 f64 accumulator fragment
    using Part = double;         // split-K partial element
    static constexpr int FRAG = 16;   // real rows / columns per fragment
    static constexpr int MT = 64;     // complex rows per workgroup (16 per wave)
    static constexpr int KP = CHUNK_KAPPA + 1;  // padded kappa stride, bank spread
};

template <>
struct Tr<FP32> {
    using R = float;
    using E = float;
    using Acc = f16_t;
    using Part = float;
    static constexpr int FRAG = 32;
    static constexpr int MT = 128;    // 32 per wave
    static constexpr int KP = CHUNK_KAPPA + 1;
};

template <>
struct Tr<BF16X3> {
    using R = float;
    using E = uint32_t;          // packed bf16 (Re low half, Im high half); planes: hi, lo
    using Acc = f16_t;
    using Part = float;
    static constexpr int FRAG = 32;
    static constexpr int MT = 128;
    static constexpr int KP = CHUNK_KAPPA + 4;  // 16-byte rows, 8 b128 lanes hit disjoint banks
};

// ----------------------------------------------------- element storage ---
__device__ __forceinline__ uint32_t pack_bf16(float a, float b)
{
    bf2_t v = {(__bf16)a, (__bf16)b};  // v_cvt_pk_bf16_f32, round to nearest even
    return __builtin_bit_cast(uint32_t, v);
}

template <int P>
__device__ __forceinline__ void store_elem(typename Tr<P>::E *p0, typename Tr<P>::E *p1, int idx,
                                           cx<typename Tr<P>::R> v)
{
    if constexpr (P == BF16X3) {
        const uint32_t hi = pack_bf16(v.re, v.im);
        const float rre = v.re - __uint_as_float(hi << 16);
        const float rim = v.im - __uint_as_float(hi & 0xffff0000u);
        p0[idx] = hi;
        p1[idx] = pack_bf16(rre, rim);
    } else {
        p0[idx] = v.re;
        p1[idx] = v.im;
    }
}

template <class R>
__device__ __forceinline__ cx<R> load_q(const void *base, size_t idx, int c64)
{
    if (c64) {
        const float2 v = reinterpret_cast<const float2 *>(base)[idx];
        return {R(v.x), R(v.y)};
    }
    const double2 v = reinterpret_cast<const double2 *>(base)[idx];
    return {R(v.x), R(v.y)};
}

// ----------------------------------------------------- MFMA multiplies ---
// Each wave owns 2 row fragments (wave rows) and NB column fragments.  Row
// fragment f of wave w covers complex rows w*WR + f*(FRAG/2) + [0, FRAG/2):
// real rows [0, FRAG/2) are the Re-rows, [FRAG/2, FRAG) the Im-rows.

template <int NB>
__device__ __forceinline__ void mma_chunk(Tr<FP64>, const double *D0, const double *D1,
                                          const double *W0, const double *W1,
                                          d4_t (&acc)[2][NB], int lane, int wave)
{
    constexpr int KP = Tr<FP64>::KP;
    // A[i][k] from lane i + 16k, B[k][j] from lane j + 16k, k = 2h + t:
    // kappa = h * (CHUNK_KAPPA/2) + step, t selects Re/Im of kappa.
    const int g = lane >> 4, h = g >> 1, t = g & 1;
    const int r = lane & 15, s = r >> 3;
    const double *Ap = (s ^ t) ? D1 : D0;
    const double sign = (s == 0 && t == 1) ? -1.0 : 1.0;
    const int arow = wave * 16 + (r & 7);
    const double *Bp = t ? W1 : W0;
    const int bcol = lane & 15;
#pragma unroll 2
    for (int j = 0; j < CHUNK_KAPPA / 2; ++j) {
        const int kap = h * (CHUNK_KAPPA / 2) + j;
        double a[2];
#pragma unroll
        for (int f = 0; f < 2; ++f) a[f] = sign * Ap[(arow + f * 8) * KP + kap];
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            const double b = Bp[(n * 16 + bcol) * KP + kap];
#pragma unroll
            for (int f = 0; f < 2; ++f) acc[f][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[f], b, acc[f][n], 0, 0, 0);
        }
    }
}

template <int NB>
__device__ __forceinline__ void mma_chunk(Tr<FP32>, const float *D0, const float *D1,
                                          const float *W0, const float *W1,
                                          f16_t (&acc)[2][NB], int lane, int wave)
{
    constexpr int KP = Tr<FP32>::KP;
    // A[i][k] from lane i + 32k, B[k][j] from lane j + 32k; k = t (Re/Im of kappa).
    const int t = lane >> 5;
    const int r = lane & 31, s = r >> 4;
    const float *Ap = (s ^ t) ? D1 : D0;
    const float sign = (s == 0 && t == 1) ? -1.0f : 1.0f;
    const int arow = wave * 32 + (r & 15);
    const float *Bp = t ? W1 : W0;
    const int bcol = lane & 31;
#pragma unroll 4
    for (int kap = 0; kap < CHUNK_KAPPA; ++kap) {
        float a[2];
#pragma unroll
        for (int f = 0; f < 2; ++f) a[f] = sign * Ap[(arow + f * 16) * KP + kap];
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            const float b = Bp[(n * 32 + bcol) * KP + kap];
#pragma unroll
            for (int f = 0; f < 2; ++f) acc[f][n] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[f], b, acc[f][n], 0, 0, 0);
        }
    }
}

__device__ __forceinline__ uint4 row_embed(uint4 v, bool im_row)
{
    // Re-row: (Re, -Im) -> flip the sign bit of the high half.
    // Im-row: (Im, Re)  -> swap the halves.
    uint4 o;
    o.x = im_row ? __builtin_amdgcn_alignbit(v.x, v.x, 16) : (v.x ^ 0x80000000u);
    o.y = im_row ? __builtin_amdgcn_alignbit(v.y, v.y, 16) : (v.y ^ 0x80000000u);
    o.z = im_row ? __builtin_amdgcn_alignbit(v.z, v.z, 16) : (v.z ^ 0x80000000u);
    o.w = im_row ? __builtin_amdgcn_alignbit(v.w, v.w, 16) : (v.w ^ 0x80000000u);
    return o;
}

template <int NB>
__device__ __forceinline__ void mma_chunk(Tr<BF16X3>, const uint32_t *Dh, const uint32_t *Dl,
                                          const uint32_t *Wh, const uint32_t *Wl,
                                          f16_t (&acc)[2][NB], int lane, int wave)
{
    constexpr int KP = Tr<BF16X3>::KP;
    // Lane i + 32g holds 8 bf16 of one row (A) or column (B): 4 kappas of
    // group g, each as an (Re, Im) pair.  The same (g, slot) -> kappa map is
    // used on both sides, so the hardware's k order inside the instruction
    // does not matter.
    const int g = lane >> 5;
    const int r = lane & 31;
    const bool im_row = (r >> 4) != 0;
    const int arow = wave * 32 + (r & 15);
    const int bcol = lane & 31;
#pragma unroll
    for (int j = 0; j < CHUNK_KAPPA / 8; ++j) {
        const int kap = 8 * j + 4 * g;
        bf8_t ah[2], al[2];
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            const int off = (arow + f * 16) * KP + kap;
            ah[f] = __builtin_bit_cast(bf8_t, row_embed(*reinterpret_cast<const uint4 *>(Dh + off), im_row));
            al[f] = __builtin_bit_cast(bf8_t, row_embed(*reinterpret_cast<const uint4 *>(Dl + off), im_row));
        }
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            const int off = (n * 32 + bcol) * KP + kap;
            const bf8_t bh = __builtin_bit_cast(bf8_t, *reinterpret_cast<const uint4 *>(Wh + off));
            const bf8_t bl = __builtin_bit_cast(bf8_t, *reinterpret_cast<const uint4 *>(Wl + off));
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                acc[f][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[f], bh, acc[f][n], 0, 0, 0);
                acc[f][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[f], bl, acc[f][n], 0, 0, 0);
                acc[f][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[f], bh, acc[f][n], 0, 0, 0);
            }
        }
    }
}

// Output element (real row, column) of accumulator register reg, as measured
// on gfx950 with a one-hot probe:
// 16x16x4 f64: row = 4*reg + lane/16, col = lane%16.
// 32x32 f32:   row = 8*(reg/4) + 4*(lane/32) + reg%4, col = lane%32.
template <int P>
__device__ __forceinline__ int acc_row(int lane, int reg)
{
    if constexpr (P == FP64)
        return 4 * reg + (lane >> 4);
    else
        return 8 * (reg >> 2) + 4 * (lane >> 5) + (reg & 3);
}

// --------------------------------------------------------- GEMM kernel ---
template <int P, int NB>
struct Geom {
    static constexpr int MT = Tr<P>::MT;
    static constexpr int NT = NB * Tr<P>::FRAG;  // complex columns per workgroup
    static constexpr int KP = Tr<P>::KP;
    static constexpr size_t d_bytes = 2ull * MT * KP * sizeof(typename Tr<P>::E);
    static constexpr size_t w_bytes = 2ull * NT * KP * sizeof(typename Tr<P>::E);
    static size_t lds(int n_mom, int L)
    {
        return d_bytes + w_bytes + (2ull * n_mom * CHUNK_SITES + L) * sizeof(cx<typename Tr<P>::R>);
    }
};

template <int P, int NB>
__global__ void __launch_bounds__(THREADS, 1) bb_gemm(GemmArgs a)
{
    using T = Tr<P>;
    using R = typename T::R;
    using E = typename T::E;
    using G = Geom<P, NB>;
    constexpr int MT = G::MT, NT = G::NT, KP = G::KP;
    constexpr int DJ = MT * CHUNK_SITES / THREADS;             // D items per thread
    constexpr int WJ = (NT * CHUNK_SITES + THREADS - 1) / THREADS;  // W items per thread
    static_assert(THREADS % MT == 0, "D item mapping needs MT | THREADS");

    extern __shared__ __align__(16) unsigned char smem[];
    E *D0 = reinterpret_cast<E *>(smem);
    E *D1 = D0 + MT * KP;
    E *W0 = D1 + MT * KP;
    E *W1 = W0 + NT * KP;
    cx<R> *ph = reinterpret_cast<cx<R> *>(smem + G::d_bytes + G::w_bytes);  // [2][n_mom][CHUNK_SITES]
    cx<R> *roots = ph + 2 * a.n_mom * CHUNK_SITES;                            // [L]
    __shared__ int s_tile;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int L = a.L, n_mom = a.n_mom;

    for (int k = tid; k < L; k += THREADS) roots[k] = {R(a.roots[2 * k]), R(a.roots[2 * k + 1])};
    __syncthreads();

    auto next_tile = [&](int current) -> int {
        if (a.counter == nullptr) return current < 0 ? (int)blockIdx.x : a.n_tiles;
        __syncthreads();
        if (tid == 0) s_tile = atomicAdd(&a.counter[0], 1);
        __syncthreads();
        return s_tile;
    };

    // Phase table of one chunk: ph[p][xl] = roots[(n_p . x) mod L].
    auto phases = [&](cx<R> *dst, int x0) {
        for (int i = tid; i < n_mom * CHUNK_SITES; i += THREADS) {
            const int p = i / CHUNK_SITES, xl = i - p * CHUNK_SITES;
            const int x = x0 + xl;
            const int ix = x % L, iy = (x / L) % L, iz = x / (L * L);
            const int k = (a.mom[3 * p] * ix + a.mom[3 * p + 1] * iy + a.mom[3 * p + 2] * iz) % L;
            dst[i] = roots[k];
        }
    };

    // A walking tile runs every split of its block in order: the loop
    // stays on tile t and steps its split (wsp) up to the block's last.
    for (int t = next_tile(-1), wsp = 0; t < a.n_tiles;) {
        const int4 tl0 = wave_uniform(a.tiles[t]);
        const BlockDesc bd = wave_uniform(a.blocks[tl0.x]);
        const int4 tl = make_int4(tl0.x, tl0.y, tl0.z, tl0.w + wsp);
        const int m0 = tl.y * MT, nu0 = tl.z * NT;
        const int xs = tl.w * bd.sps;
        const int xe = min(a.V, xs + bd.sps);
        const int n_chunks = (xe - xs + CHUNK_SITES - 1) / CHUNK_SITES;

        // D work of this thread: one row (d1, d2), DJ sites per chunk.
        const int dm = tid % MT;
        const bool dvalid = (m0 + dm) < bd.M;
        const int d1 = dvalid ? (m0 + dm) / bd.n2 : 0;
        const int d2 = dvalid ? (m0 + dm) % bd.n2 : 0;
        // W work of this thread: WJ (column, site) items per chunk.
        int wnl[WJ], wxl[WJ], wp[WJ], wd3[WJ];
        bool wv[WJ];
#pragma unroll
        for (int j = 0; j < WJ; ++j) {
            const int item = tid + THREADS * j;
            wnl[j] = item % NT;
            wxl[j] = item / NT;
            const int nu = nu0 + wnl[j];
            wv[j] = item < NT * CHUNK_SITES && nu < bd.N;
            wp[j] = wv[j] ? nu / bd.n3 : 0;
            wd3[j] = wv[j] ? nu % bd.n3 : 0;
        }

        typename T::Acc acc[2][NB];
#pragma unroll
        for (int f = 0; f < 2; ++f)
#pragma unroll
            for (int n = 0; n < NB; ++n)
#pragma unroll
                for (int e = 0; e < (int)(sizeof(typename T::Acc) / sizeof(acc[0][0][0])); ++e) acc[f][n][e] = 0;

        phases(ph, xs);
        __syncthreads();
        for (int c = 0; c < n_chunks; ++c) {
            const int x0 = xs + c * CHUNK_SITES;
            const cx<R> *phc = ph + (c & 1) * n_mom * CHUNK_SITES;
            // Diquark D_c(x; d1, d2) = eps_abc q1_a q2_b (Algorithm 1, the diquark loop).
#pragma unroll
            for (int j = 0; j < DJ; ++j) {
                const int xl = tid / MT + j * (THREADS / MT);
                const int x = x0 + xl;
                cx<R> dq[3] = {{0, 0}, {0, 0}, {0, 0}};
                if (dvalid && x < xe) {
                    cx<R> u[3], v[3];
#pragma unroll
                    for (int col = 0; col < 3; ++col) {
                        u[col] = load_q<R>(bd.q1, ((size_t)x * 3 + col) * bd.n1 + d1, a.in_c64);
                        v[col] = load_q<R>(bd.q2, ((size_t)x * 3 + col) * bd.n2 + d2, a.in_c64);
                    }
                    dq[0] = csub(cmul(u[1], v[2]), cmul(u[2], v[1]));
                    dq[1] = csub(cmul(u[2], v[0]), cmul(u[0], v[2]));
                    dq[2] = csub(cmul(u[0], v[1]), cmul(u[1], v[0]));
                }
#pragma unroll
                for (int col = 0; col < 3; ++col) store_elem<P>(D0, D1, dm * KP + col * CHUNK_SITES + xl, dq[col]);
            }
            // Phase-weighted third quark W_c(x; p, d3) = q3_c(x, d3) exp(-i p.x).
#pragma unroll
            for (int j = 0; j < WJ; ++j) {
                if (tid + THREADS * j >= NT * CHUNK_SITES) break;
                const int x = x0 + wxl[j];
                cx<R> w[3] = {{0, 0}, {0, 0}, {0, 0}};
                if (wv[j] && x < xe) {
                    const cx<R> e = phc[wp[j] * CHUNK_SITES + wxl[j]];
#pragma unroll
                    for (int col = 0; col < 3; ++col)
                        w[col] = cmul(load_q<R>(bd.q3, ((size_t)x * 3 + col) * bd.n3 + wd3[j], a.in_c64), e);
                }
#pragma unroll
                for (int col = 0; col < 3; ++col) store_elem<P>(W0, W1, wnl[j] * KP + col * CHUNK_SITES + wxl[j], w[col]);
            }
            __syncthreads();
            if (c + 1 < n_chunks) phases(ph + ((c + 1) & 1) * n_mom * CHUNK_SITES, x0 + CHUNK_SITES);
            mma_chunk<NB>(T{}, D0, D1, W0, W1, acc, lane, wave);
            __syncthreads();
        }

        // Epilogue: Re-rows and Im-rows of complex row m, column nu = p*n3 + d3.
        with_put_mode(bd, tl.w, [&](auto mode) {
            constexpr int REGS = sizeof(typename T::Acc) / sizeof(acc[0][0][0]);
            constexpr int HALF = T::FRAG / 2;
            constexpr int WR = 2 * HALF;  // complex rows per wave
#pragma unroll
            for (int n = 0; n < NB; ++n) {
                const int nu = nu0 + n * T::FRAG + (lane % T::FRAG);
                if (nu >= bd.N) continue;
                const int p = nu / bd.n3, d3 = nu - (nu / bd.n3) * bd.n3;
#pragma unroll
                for (int f = 0; f < 2; ++f)
#pragma unroll
                    for (int e = 0; e < REGS; ++e) {
                        const int row = acc_row<P>(lane, e);
                        const int m = m0 + wave * WR + f * HALF + (row % HALF);
                        const int s = row / HALF;
                        if (m >= bd.M) continue;
                        put_result<decltype(mode)::value, typename T::Part>(bd, tl.w, m, nu, p, d3, s, (double)acc[f][n][e]);
                    }
            }
        });
        if (bd.walk && tl.w + 1 < bd.S) {
            ++wsp;
            __syncthreads();  // the split's last LDS reads come before the next split's writes
        } else {
            wsp = 0;
            t = next_tile(t);
        }
    }

    if (a.counter != nullptr && tid == 0) {
        // The last workgroup out resets both counters for the next launch
        // (also when the launch is replayed from a captured graph).
        __threadfence();
        if (atomicAdd(&a.counter[1], 1) == (int)gridDim.x - 1) {
            atomicExch(&a.counter[0], 0);
            atomicExch(&a.counter[1], 0);
        }
    }
}

// --------------------------------------------------------- FP64 reduce ---
// B[p][d1][d2][d3] = sum over splits of the partials, in FP64, in split order.
template <class PartT>
__global__ void __launch_bounds__(256) bb_reduce(ReduceArgs a)
{
    const BlockDesc bd = a.blocks[a.list[blockIdx.y]];
    const PartT *ws = reinterpret_cast<const PartT *>(bd.ws);
    const size_t MN = (size_t)bd.M * bd.N;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < MN; idx += (size_t)gridDim.x * blockDim.x) {
        const int m = (int)(idx / bd.N), nu = (int)(idx - (size_t)m * bd.N);
        double re = 0.0, im = 0.0;
        // Unrolled so that the loads of several splits are in flight at once;
        // the additions stay in split order.
#pragma unroll 8
        for (int s = 0; s < bd.S; ++s) {
            re += (double)ws[(size_t)(2 * s) * MN + idx];
            im += (double)ws[(size_t)(2 * s + 1) * MN + idx];
        }
        const int p = nu / bd.n3, d3 = nu - p * bd.n3;
        reinterpret_cast<double2 *>(bd.out)[((size_t)p * bd.M + m) * bd.n3 + d3] = make_double2(re, im);
    }
}

// ---------------------------------------------------- spin projection ---
// Output group g (paper, eq. (1): the spin-projected block is a linear
// combination of baryon blocks): out = sum_i c_i * (sum_s partials_i[s]), in
// FP64, members in list order and splits in split order, so the result is
// reproducible; with accumulate[g] set the sum is added to out (the group's
// earlier members ran in an earlier launch).
template <class PartT>
__global__ void __launch_bounds__(256) bb_combine(CombineArgs a)
{
    const int g = blockIdx.y;
    const int i0 = a.gstart[g], i1 = a.gstart[g + 1];
    const BlockDesc b0 = a.blocks[a.list[i0]];
    const size_t MN = (size_t)b0.M * b0.N;
    double2 *out = reinterpret_cast<double2 *>(b0.out);
    const bool acc = a.accumulate[g] != 0;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < MN; idx += (size_t)gridDim.x * blockDim.x) {
        const int m = (int)(idx / b0.N), nu = (int)(idx - (size_t)m * b0.N);
        const int p = nu / b0.n3, d3 = nu - p * b0.n3;
        const size_t o = ((size_t)p * b0.M + m) * b0.n3 + d3;
        double re = 0.0, im = 0.0;
        if (acc) {
            const double2 v = out[o];
            re = v.x;
            im = v.y;
        }
        for (int i = i0; i < i1; ++i) {
            const BlockDesc bd = a.blocks[a.list[i]];
            const PartT *ws = reinterpret_cast<const PartT *>(bd.ws);
            double br = 0.0, bi = 0.0;
            for (int s = 0; s < bd.S; ++s) {
                br += (double)ws[(size_t)(2 * s) * MN + idx];
                bi += (double)ws[(size_t)(2 * s + 1) * MN + idx];
            }
            const double cr = a.coef[2 * i], ci = a.coef[2 * i + 1];
            re += cr * br - ci * bi;
            im += cr * bi + ci * br;
        }
        out[o] = make_double2(re, im);
    }
}

// ------------------------------------------------------- host launchers ---
static const int kNbFp64[] = {1, 2, 4, 7, 14};
static const int kNbF32[] = {1, 2, 4, 7};

int nb_options(int prec, const int **list)
{
    if (prec == FP64) {
        *list = kNbFp64;
        return 5;
    }
    *list = kNbF32;
    return 4;
}

template <int P, int NB>
static hipError_t launch_one(const GemmArgs &a, int grid, hipStream_t st)
{
    const size_t lds = Geom<P, NB>::lds(a.n_mom, a.L);
    hipLaunchKernelGGL((bb_gemm<P, NB>), dim3(grid), dim3(THREADS), lds, st, a);
    return hipGetLastError();
}

template <int P, int NB>
static hipError_t raise_lds(int bytes)
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&bb_gemm<P, NB>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <int P>
static KernelGeom geom_of(int nb, int n_mom, int L)
{
    KernelGeom g{Tr<P>::MT, Tr<P>::FRAG, 0};
    switch (nb) {
    case 1: g.lds_bytes = (int)Geom<P, 1>::lds(n_mom, L); break;
    case 2: g.lds_bytes = (int)Geom<P, 2>::lds(n_mom, L); break;
    case 4: g.lds_bytes = (int)Geom<P, 4>::lds(n_mom, L); break;
    case 7: g.lds_bytes = (int)Geom<P, 7>::lds(n_mom, L); break;
    case 14: g.lds_bytes = (int)Geom<P, 14>::lds(n_mom, L); break;
    default: g.lds_bytes = -1;
    }
    return g;
}

KernelGeom kernel_geom(int prec, int nb, int n_mom, int L)
{
    switch (prec) {
    case FP64: return geom_of<FP64>(nb, n_mom, L);
    case FP32: return (nb == 14) ? KernelGeom{0, 0, -1} : geom_of<FP32>(nb, n_mom, L);
    default: return (nb == 14) ? KernelGeom{0, 0, -1} : geom_of<BF16X3>(nb, n_mom, L);
    }
}

hipError_t launch_gemm(int prec, int nb, const GemmArgs &a, int grid, hipStream_t st)
{
#define BB_CASE(P, NB) \
    if (prec == P && nb == NB) return launch_one<P, NB>(a, grid, st);
    BB_CASE(FP64, 1) BB_CASE(FP64, 2) BB_CASE(FP64, 4) BB_CASE(FP64, 7) BB_CASE(FP64, 14)
    BB_CASE(FP32, 1) BB_CASE(FP32, 2) BB_CASE(FP32, 4) BB_CASE(FP32, 7)
    BB_CASE(BF16X3, 1) BB_CASE(BF16X3, 2) BB_CASE(BF16X3, 4) BB_CASE(BF16X3, 7)
#undef BB_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_reduce(int prec, const ReduceArgs &a, int max_mn, hipStream_t st)
{
    if (a.n_list <= 0) return hipSuccess;
    const int gx = (int)std::min<long>(1024, ((long)max_mn + 255) / 256);
    if (prec == FP64)
        hipLaunchKernelGGL(bb_reduce<double>, dim3(gx, a.n_list), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(bb_reduce<float>, dim3(gx, a.n_list), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_combine(int prec, const CombineArgs &a, int max_mn, hipStream_t st)
{
    if (a.n_groups <= 0) return hipSuccess;
    if (a.n_groups > 65535) return hipErrorInvalidValue;
    const int gx = (int)std::min<long>(1024, ((long)max_mn + 255) / 256);
    if (prec == FP64)
        hipLaunchKernelGGL(bb_combine<double>, dim3(gx, a.n_groups), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(bb_combine<float>, dim3(gx, a.n_groups), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t prepare_kernels(int lds_bytes)
{
    hipError_t e = hipSuccess;
#define BB_RAISE(P, NB) \
    if (e == hipSuccess) e = raise_lds<P, NB>(lds_bytes);
    BB_RAISE(FP64, 1) BB_RAISE(FP64, 2) BB_RAISE(FP64, 4) BB_RAISE(FP64, 7) BB_RAISE(FP64, 14)
    BB_RAISE(FP32, 1) BB_RAISE(FP32, 2) BB_RAISE(FP32, 4) BB_RAISE(FP32, 7)
    BB_RAISE(BF16X3, 1) BB_RAISE(BF16X3, 2) BB_RAISE(BF16X3, 4) BB_RAISE(BF16X3, 7)
#undef BB_RAISE
    return e;
}

}  // namespace bb
