// FP32 paper-order contraction kernels of libbblock.so (gfx950, plan kernels
// 7 and 9).
//
// The block of the paper (Sec. 2, eq. (3)) in the order of Algorithm 1, as
// FP64 kernel 6 does it, in single precision: per site the singlet
//   S[x; (d1,d2), d3] = sum_c D_c[x; d1,d2] q3_c[x; d3],  D_c = eps_abc q1_a q2_b,
// formed per lane in the MFMA operand layout, then the momentum projection
//   B[p][(d1,d2)][d3] = sum_x S[x; (d1,d2), d3] exp(-i p.x)
// on v_mfma_f32_16x16x4_f32 (kernel 7, fragments of 16 momenta) or
// v_mfma_f32_4x4x1_16b_f32 (kernel 9, fragments of 4: few momenta pad to a
// multiple of 4, not of 16) with three real products up to two momentum
// fragments (P1 = (Sr + Si)(er + ei), P2 = Sr er, P3 = Si ei; Re = P2 - P3,
// Im = P1 - P2 - P3) and the real embedding above (four: Re += Sr er -
// Si ei, Im += Sr ei + Si er), FP32 accumulation over a site split of at
// most 4096 sites, the splits summed in FP64.  As with FP64, the
// counters show no co-execution of vector work with these MFMAs: the second
// workgroup per CU of the narrow tiles is what covers the vector work's and
// the LDS's latencies.
//
// Workgroup: eight wave64, two per SIMD (two workgroups per CU for tiles
// of one or two momentum fragments and d3 blocks of 16).  Tile: 128 rows = NPAIR (d1,d2)
// pairs x a block of B3 d3 values, W CF momenta, one site split; wave w
// owns rows 16 w to 16 w + 15 (16 d3 values of one pair) and all momenta:
// CF accumulator fragments per real product.  With W = 4 each of the 16
// blocks of an MFMA holds 4 rows at one site of the k-step; the epilogue
// adds the four sites' blocks across lanes.  Chunks of 32 sites, double
// buffered in LDS: the diquark of the tile's pairs, q3 of its d3 block, the
// phases of its momenta, built from registers loaded a chunk earlier.
//
// Zero momentum (instantiation Z, kernel 7 only, a.p_skip >= 0), as in kernel 6: summed
// per lane on the vector unit, reduced across the k-groups at the end and
// written by the tiles of column block 0; the columns hold the other
// momenta.  Z kernels of two workgroups per CU are held to 128 VGPRs by
// their launch bounds (four waves per SIMD); with complex128 inputs and two
// fragments that spills two values outside the chunk loop.
#include <algorithm>

#include "bb_fast.h"
#include "bb_internal.h"

namespace bb {
namespace f32p {

typedef float f4_t __attribute__((ext_vector_type(4)));

constexpr int WG = 512;       // eight waves
constexpr int MT = 128;       // rows (pair, d3) per tile, 16 per wave
constexpr int SITES = 32;     // sites per chunk
constexpr int KS = SITES / 4; // k-steps per chunk
constexpr uint32_t OOB = 0x80000000u;  // a buffer offset past any range: loads return zero

// W: momenta per column fragment, 16 (v_mfma_f32_16x16x4_f32) or 4
// (v_mfma_f32_4x4x1_16b_f32, plan kernel 9).
template <int CF, int B3, int W = 16>
struct Shape {
    static constexpr int NPAIR = MT / B3;                     // (d1,d2) pairs per tile
    static constexpr int NC = W * CF;                         // momenta per tile
    // Site stride of the phase planes (floats): the k-groups 0 and 1 of a
    // half-wave read 16 floats apart modulo 32 banks.
    static constexpr int PS = W == 4 ? 16 : (NC % 32 == 0) ? NC + 16 : NC;
    static constexpr int ND = NPAIR * SITES;                  // diquark items per chunk
    static constexpr int NQ = SITES * 3 * B3;                 // q3 values per chunk
    static constexpr int NP = SITES * NC;                     // phases per chunk
    static constexpr int JQ = (NQ + WG - 1) / WG, JP = (NP + WG - 1) / WG;
    // Complex products: three real products (Gauss, as in the FP64 kernels,
    // with the phase's Re + Im formed per k-step) up to two momentum
    // fragments, where the third accumulator still leaves two workgroups per
    // CU; four (the real embedding) above.
    static constexpr bool G3 = CF <= 2;
    static constexpr int NPL = 2;                             // phase planes
    // One buffer (floats): D [3][SITES][NPAIR] and q3 [3][SITES][B3] as
    // (re, im) pairs, then the phase planes Re, Im [SITES][PS].
    static constexpr int DOFF = 0, QOFF = 2 * 3 * SITES * NPAIR, POFF = QOFF + 2 * 3 * SITES * B3;
    static constexpr int BUF = POFF + NPL * SITES * PS;
    static constexpr size_t lds = (size_t)2 * BUF * 4 + (size_t)MAX_L * 8;
    static_assert(PS % 32 == 16, "the two k-groups of a half-wave must read disjoint banks");
    static_assert(B3 % 16 == 0 && MT % B3 == 0, "a wave's 16 rows are d3 values of one pair");
    static_assert(ND % 64 == 0 && ND <= WG, "diquark items end on a wave boundary, one per thread");
    static_assert(NQ % 256 == 0 && NP % 64 == 0, "q3 and phase items end on a wave boundary");
    static_assert(W == 16 || (W == 4 && B3 == 16), "fragments of 4 momenta with d3 blocks of 16");
    static_assert(lds <= 160 * 1024, "two buffers fit the LDS");
    // Workgroups per CU: two for the narrow tiles with d3 blocks of 16 (their
    // LDS and at most 128 VGPRs let both fit, and four waves per SIMD hide
    // more latency than two), one otherwise.
    static constexpr int WGS = (B3 == 16 && CF <= 2) ? 2 : 1;
    static_assert(WGS == 1 || 2 * lds <= 160 * 1024, "two workgroups fit the LDS");
};

template <bool C64>
struct In {
    static constexpr int ESZ = 16;
};
template <>
struct In<true> {
    static constexpr int ESZ = 8;
};

template <bool C64>
__device__ __forceinline__ float2 ldq(__amdgpu_buffer_rsrc_t rs, uint32_t off)
{
    if constexpr (C64) {
        return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
    } else {
        const double2 v = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
        return make_float2((float)v.x, (float)v.y);
    }
}

// Resource over sites [x0, x0 + SITES) of a field [V][3][n] (bytes in range:
// the sites below xe only; none when x0 >= xe).
template <bool C64>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t chunk_rsrc(const void *q, int n, int x0, int xe)
{
    constexpr int ESZ = In<C64>::ESZ;
    const int ns = __builtin_amdgcn_readfirstlane(min(max(xe - x0, 0), SITES));  // wave-uniform: no waterfall
    const unsigned char *base = static_cast<const unsigned char *>(q) + (size_t)x0 * 3 * n * ESZ;
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, ns * 3 * n * ESZ, 0x00020000);
}

// One MFMA of the projection: a 16 x 16 fragment over 4 sites (W = 16), or
// 16 blocks of 4 x 4 over one site each (W = 4: block b holds rows
// 4 (b % 4) .. 4 (b % 4) + 3 at site b / 4 of the k-step, the sites summed
// across blocks in the epilogue).
template <int W>
__device__ __forceinline__ f4_t mfma(float a, float b, f4_t c)
{
    if constexpr (W == 16)
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

// Launch bounds: held to the registers of WGS workgroups per CU (2 WGS
// waves per SIMD).
template <int CF, int B3, bool C64, bool Z, int W = 16>
__global__ void __launch_bounds__(WG, (2 * Shape<CF, B3, W>::WGS)) contract(GemmArgs a)
{
    static_assert(!Z || W == 16, "fragments of 4 keep the zero momentum a column");
    using Sh = Shape<CF, B3, W>;
    constexpr int NPAIR = Sh::NPAIR, NC = Sh::NC, PS = Sh::PS, BUF = Sh::BUF;
    constexpr int ESZ = In<C64>::ESZ;
    __shared__ __align__(16) float lds[2 * BUF];
    __shared__ float2 roots[MAX_L];
    __shared__ int s_tile;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int k = tid; k < a.L; k += WG) roots[k] = make_float2((float)a.roots[2 * k], (float)a.roots[2 * k + 1]);

    auto next_tile = [&](int current) -> int {
        if (a.counter == nullptr) return current < 0 ? (int)blockIdx.x : a.n_tiles;
        __syncthreads();
        if (tid == 0) s_tile = atomicAdd(&a.counter[0], 1);
        __syncthreads();
        return __builtin_amdgcn_readfirstlane(s_tile);
    };
    __syncthreads();

    // A walking tile runs every split of its block in order: the loop
    // stays on tile t and steps its split (wsp) up to the block's last.
    for (int t = next_tile(-1), wsp = 0; t < a.n_tiles;) {
        const int4 tl0 = wave_uniform(a.tiles[t]);
        const BlockDesc bd = wave_uniform(a.blocks[tl0.x]);
        const int4 tl = make_int4(tl0.x, tl0.y, tl0.z, tl0.w + wsp);
        // m-tile = (pair block, d3 block); n_mt2 holds the number of d3 blocks.
        const int m12_0 = (tl.y / bd.n_mt2) * NPAIR, d3_0 = (tl.y % bd.n_mt2) * B3;
        const int p0 = tl.z * NC;
        const int M12 = bd.M;
        const int xs = tl.w * bd.sps;
        const int xe = min(a.V, xs + bd.sps);
        const int n_chunks = (xe - xs + SITES - 1) / SITES;

        // ---- generation items of this thread (tile invariant) ----
        // Diquark item: pair tid % NPAIR at site tid / NPAIR (threads past ND: none).
        const bool has_d = wave * 64 < Sh::ND;  // wave-uniform
        const int dp = tid % NPAIR, ds = tid / NPAIR;
        const int m = m12_0 + dp;
        const bool mok = has_d && m < M12;
        const int d1 = mok ? m / bd.n2 : 0, d2 = mok ? m - (m / bd.n2) * bd.n2 : 0;
        uint32_t o1[3], o2[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            o1[c] = mok ? (uint32_t)(((ds * 3 + c) * bd.n1 + d1) * ESZ) : OOB;
            o2[c] = mok ? (uint32_t)(((ds * 3 + c) * bd.n2 + d2) * ESZ) : OOB;
        }
        // q3 items q = tid + WG j = ((s 3 + c) B3 + d): offsets in the chunk.
        uint32_t o3[Sh::JQ];
#pragma unroll
        for (int j = 0; j < Sh::JQ; ++j) {
            const int q = tid + WG * j;
            const int d = q % B3, sc = q / B3;
            o3[j] = (q < Sh::NQ && d3_0 + d < bd.n3) ? (uint32_t)((sc * bd.n3 + d3_0 + d) * ESZ) : OOB;
        }
        // Momentum columns: every momentum but, with Z, a.p_skip (the zero
        // momentum, summed on the vector unit and written by the tiles of
        // column block 0).
        const int ps = Z ? a.p_skip : -1, n_col = a.n_mom - (Z ? 1 : 0);
        const bool zsum = Z && tl.z == 0;  // wave-uniform
        // Phase items q = tid + WG j = (s NC + jc): column p0 + jc at site s.
        uint32_t ok[Sh::JP];
#pragma unroll
        for (int j = 0; j < Sh::JP; ++j) {
            const int q = tid + WG * j;
            const int jc = q % NC, s = q / NC, col = p0 + jc;
            const int pm = col + (Z && col >= ps ? 1 : 0);
            ok[j] = (q < Sh::NP && col < n_col) ? (uint32_t)(pm * a.kstride + s) : OOB;
        }
        const int krec = a.n_mom * a.kstride;

        float2 u[3], v[3], w[Sh::JQ];
        uint32_t kk[Sh::JP];
        auto issue = [&](int ci) {
            const int x0 = __builtin_amdgcn_readfirstlane(xs + ci * SITES);
            if (has_d) {
                const __amdgpu_buffer_rsrc_t rs1 = chunk_rsrc<C64>(bd.q1, bd.n1, x0, xe);
                const __amdgpu_buffer_rsrc_t rs2 = chunk_rsrc<C64>(bd.q2, bd.n2, x0, xe);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    u[c] = ldq<C64>(rs1, o1[c]);
                    v[c] = ldq<C64>(rs2, o2[c]);
                }
            }
            const __amdgpu_buffer_rsrc_t rs3 = chunk_rsrc<C64>(bd.q3, bd.n3, x0, xe);
#pragma unroll
            for (int j = 0; j < Sh::JQ; ++j) w[j] = ldq<C64>(rs3, o3[j]);
            const __amdgpu_buffer_rsrc_t rsk = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(a.kidx + min(x0, krec)), (short)0, max(krec - x0, 0), 0x00020000);
#pragma unroll
            for (int j = 0; j < Sh::JP; ++j) kk[j] = __builtin_amdgcn_raw_buffer_load_b8(rsk, ok[j], 0, 0);
        };
        // The loaded chunk into buffer b: the diquark u_a v_b - u_b v_a
        // (eps_{a b c} = +1) per colour with the fixed rounding of
        // fast::cmulf, q3 as loaded, the phases roots[k] = exp(-2 pi i k / L).
        auto build = [&](int b) {
            asm volatile("" : "+s"(b));  // one base register per buffer, immediate offsets from it
            float *base = lds + b * BUF;
            float2 *Dt = reinterpret_cast<float2 *>(base + Sh::DOFF);
            float2 *Qt = reinterpret_cast<float2 *>(base + Sh::QOFF);
            float *Pr = base + Sh::POFF, *Pi = Pr + SITES * PS;
            if (has_d) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float2 x = fast::cmulf(u[(c + 1) % 3], v[(c + 2) % 3]);
                    const float2 y = fast::cmulf(u[(c + 2) % 3], v[(c + 1) % 3]);
                    Dt[(c * SITES + ds) * NPAIR + dp] = make_float2(x.x - y.x, x.y - y.y);
                }
            }
#pragma unroll
            for (int j = 0; j < Sh::JQ; ++j) {
                const int q = tid + WG * j;
                if (q < Sh::NQ) {
                    const int d = q % B3, sc = q / B3, s = sc / 3, c = sc - 3 * s;
                    Qt[(c * SITES + s) * B3 + d] = w[j];
                }
            }
#pragma unroll
            for (int j = 0; j < Sh::JP; ++j) {
                const int q = tid + WG * j;
                if (q < Sh::NP) {
                    const int jc = q % NC, s = q / NC;
                    const float2 e = roots[kk[j]];
                    Pr[s * PS + jc] = e.x;
                    Pi[s * PS + jc] = e.y;
                }
            }
        };

        constexpr int NACC = Sh::G3 ? 3 : 2;  // (P1, P2, P3) or (Re, Im)
        f4_t acc[NACC][CF];
#pragma unroll
        for (int q = 0; q < NACC; ++q)
#pragma unroll
            for (int n = 0; n < CF; ++n) acc[q][n] = f4_t{0.f, 0.f, 0.f, 0.f};
        // A[i][k] from lane i + 16 k: row 16 wave + i at site k of the k-step.
        const int li = lane & 15, kg = lane >> 4;
        const int rw = wave * 16 + li;
        const int pair_l = rw / B3, d3_l = rw % B3;

        // One chunk from buffer b: per k-step the singlets of this lane's
        // (row, site) from LDS, then 4 CF MFMAs; after the first k-step the
        // next chunk's tiles go into buffer b ^ 1 and the loads of the chunk
        // after it are issued.
        float zr = 0.f, zi = 0.f;  // this lane's (row, site) singlets summed: the zero momentum
        auto chunk = [&](int b, int ci_next) {
            asm volatile("" : "+s"(b));
            const float *base = lds + b * BUF;
            const float2 *Dl = reinterpret_cast<const float2 *>(base + Sh::DOFF) + kg * NPAIR + pair_l;
            const float2 *Ql = reinterpret_cast<const float2 *>(base + Sh::QOFF) + kg * B3 + d3_l;
            // B[k][j] (W = 16) or B[b][0][j] (W = 4, j = lane % 4): the
            // phase of column j at the lane's site.
            const float *Pl = base + Sh::POFF + kg * PS + (W == 16 ? li : (lane & 3));
            float2 dv[2][3], qv[2][3];
            float br[2][CF], bi[2][CF];
            auto read_s = [&](int ks, int slot) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    dv[slot][c] = Dl[(c * SITES + 4 * ks) * NPAIR];
                    qv[slot][c] = Ql[(c * SITES + 4 * ks) * B3];
                }
#pragma unroll
                for (int n = 0; n < CF; ++n) {
                    br[slot][n] = Pl[4 * ks * PS + n * W];
                    bi[slot][n] = Pl[(SITES + 4 * ks) * PS + n * W];
                }
            };
            read_s(0, 0);
            fast::static_for<0, KS>([&](auto kk_) {
                constexpr int ks = kk_, slot = ks & 1;
                // Singlet S = sum_c D_c q3_c (complex).
                float sr = __builtin_fmaf(dv[slot][0].x, qv[slot][0].x, -(dv[slot][0].y * qv[slot][0].y));
                float si = __builtin_fmaf(dv[slot][0].x, qv[slot][0].y, dv[slot][0].y * qv[slot][0].x);
#pragma unroll
                for (int c = 1; c < 3; ++c) {
                    sr = __builtin_fmaf(dv[slot][c].x, qv[slot][c].x, sr);
                    sr = __builtin_fmaf(-dv[slot][c].y, qv[slot][c].y, sr);
                    si = __builtin_fmaf(dv[slot][c].x, qv[slot][c].y, si);
                    si = __builtin_fmaf(dv[slot][c].y, qv[slot][c].x, si);
                }
                const float nsi = -si, ss = sr + si;
                if constexpr (Z) {
                    zr += sr;
                    zi += si;
                }
                if constexpr (ks + 1 < KS) read_s(ks + 1, slot ^ 1);
#pragma unroll
                for (int n = 0; n < CF; ++n) {
                    if constexpr (Sh::G3) {
                        acc[0][n] = mfma<W>(ss, br[slot][n] + bi[slot][n], acc[0][n]);
                        acc[1][n] = mfma<W>(sr, br[slot][n], acc[1][n]);
                        acc[NACC - 1][n] = mfma<W>(si, bi[slot][n], acc[NACC - 1][n]);
                    } else {
                        acc[0][n] = mfma<W>(sr, br[slot][n], acc[0][n]);
                        acc[1][n] = mfma<W>(sr, bi[slot][n], acc[1][n]);
                        acc[0][n] = mfma<W>(nsi, bi[slot][n], acc[0][n]);
                        acc[1][n] = mfma<W>(si, br[slot][n], acc[1][n]);
                    }
                }
                if constexpr (ks == 0) {
                    build(b ^ 1);
                    issue(ci_next);  // past the split the loads are out of range (zeros)
                }
            });
        };

        // Prologue: chunk 0 into buffer 0, chunk 1 in registers.
        issue(0);
        build(0);
        issue(1);
        __syncthreads();
        for (int i = 0; i < n_chunks; ++i) {
            chunk(i & 1, i + 2);
            __syncthreads();
        }
        if constexpr (Z) {
            // The four sites of a k-step sit in lanes l, l + 16, l + 32, l + 48.
            zr += __shfl_xor(zr, 16);
            zi += __shfl_xor(zi, 16);
            zr += __shfl_xor(zr, 32);
            zi += __shfl_xor(zi, 32);
        }

        if constexpr (W == 4) {
            // Block b = lane / 4 summed over the sites of its k-group only:
            // add the four k-groups (lanes l, l ^ 16, l ^ 32, l ^ 48).
#pragma unroll
            for (int q = 0; q < NACC; ++q)
#pragma unroll
                for (int n = 0; n < CF; ++n)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        float x = acc[q][n][e];
                        x += __shfl_xor(x, 16);
                        x += __shfl_xor(x, 32);
                        acc[q][n][e] = x;
                    }
        }

        // Epilogue.  Accumulator register e of a 16x16 f32 fragment holds
        // row 4 (lane / 16) + e, column lane % 16; of the 4 x 4 blocks (the
        // k-groups added above), row 4 ((lane / 4) % 4) + e, column lane % 4:
        // there k-group kg writes register kg.
        with_put_mode(bd, tl.w, [&](auto mode) {
            if constexpr (W == 4) {
#pragma unroll
                for (int n = 0; n < CF; ++n) {
                    const int col = p0 + n * 4 + (lane & 3);
                    if (col >= n_col) continue;
                    const int r = wave * 16 + 4 * ((lane >> 2) & 3) + kg;
                    const int mo = m12_0 + r / B3, d3 = d3_0 + r % B3;
                    if (mo >= M12 || d3 >= bd.n3) continue;
                    const int nu = col * bd.n3 + d3;
                    float x[NACC];
#pragma unroll
                    for (int q = 0; q < NACC; ++q) {
                        const f4_t v = acc[q][n];
                        x[q] = kg == 0 ? v[0] : kg == 1 ? v[1] : kg == 2 ? v[2] : v[3];
                    }
                    float re = x[0], im = x[1];
                    if constexpr (Sh::G3) {  // Re = P2 - P3, Im = P1 - P2 - P3
                        re = x[1] - x[NACC - 1];
                        im = (x[0] - x[1]) - x[NACC - 1];
                    }
                    put_result<decltype(mode)::value, float>(bd, tl.w, mo, nu, col, d3, 0, (double)re);
                    put_result<decltype(mode)::value, float>(bd, tl.w, mo, nu, col, d3, 1, (double)im);
                }
            } else {
#pragma unroll
                for (int n = 0; n < CF; ++n) {
                    const int col = p0 + n * 16 + li;
                    if (col >= n_col) continue;
                    const int p = col + (Z && col >= ps ? 1 : 0);
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int r = wave * 16 + 4 * kg + e;
                        const int mo = m12_0 + r / B3, d3 = d3_0 + r % B3;
                        if (mo >= M12 || d3 >= bd.n3) continue;
                        const int nu = p * bd.n3 + d3;
                        float re = acc[0][n][e], im = acc[1][n][e];
                        if constexpr (Sh::G3) {  // Re = P2 - P3, Im = P1 - P2 - P3
                            const float p3 = acc[NACC - 1][n][e];
                            re = acc[1][n][e] - p3;
                            im = (acc[0][n][e] - acc[1][n][e]) - p3;
                        }
                        put_result<decltype(mode)::value, float>(bd, tl.w, mo, nu, p, d3, 0, (double)re);
                        put_result<decltype(mode)::value, float>(bd, tl.w, mo, nu, p, d3, 1, (double)im);
                    }
                }
                if (Z && zsum && kg == 0) {
                    const int mo = m12_0 + pair_l, d3 = d3_0 + d3_l;
                    if (mo < M12 && d3 < bd.n3) {
                        const int nu = ps * bd.n3 + d3;
                        put_result<decltype(mode)::value, float>(bd, tl.w, mo, nu, ps, d3, 0, (double)zr);
                        put_result<decltype(mode)::value, float>(bd, tl.w, mo, nu, ps, d3, 1, (double)zi);
                    }
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
        // The last workgroup out resets both counters for the next launch.
        __threadfence();
        if (atomicAdd(&a.counter[1], 1) == (int)gridDim.x - 1) {
            atomicExch(&a.counter[0], 0);
            atomicExch(&a.counter[1], 0);
        }
    }
}

template <int CF, int B3, bool C64>
hipError_t run(const GemmArgs &a, int grid, hipStream_t st)
{
    if (a.p_skip >= 0)
        contract<CF, B3, C64, true><<<dim3(grid), dim3(WG), 0, st>>>(a);
    else
        contract<CF, B3, C64, false><<<dim3(grid), dim3(WG), 0, st>>>(a);
    return hipGetLastError();
}

// Fragments of 4 momenta (plan kernel 9): every momentum is a column.
template <int CF, bool C64>
hipError_t run_narrow(const GemmArgs &a, int grid, hipStream_t st)
{
    if (a.p_skip >= 0) return hipErrorInvalidValue;
    contract<CF, 16, C64, false, 4><<<dim3(grid), dim3(WG), 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace f32p

int f32p_lds_bytes(int cf, int b3, int w)
{
#define BBR_SIZE(CF_, B3_, W_) \
    if (cf == CF_ && b3 == B3_ && w == W_) return (int)f32p::Shape<CF_, B3_, W_>::lds;
    BBR_SIZE(1, 16, 16) BBR_SIZE(2, 16, 16) BBR_SIZE(3, 16, 16) BBR_SIZE(4, 16, 16)
    BBR_SIZE(1, 32, 16) BBR_SIZE(2, 32, 16) BBR_SIZE(3, 32, 16) BBR_SIZE(4, 32, 16)
    BBR_SIZE(1, 16, 4) BBR_SIZE(2, 16, 4) BBR_SIZE(3, 16, 4) BBR_SIZE(4, 16, 4)
#undef BBR_SIZE
    return -1;
}

int f32p_pairs(int b3) { return b3 == 16 || b3 == 32 ? f32p::MT / b3 : -1; }

int f32p_wgs(int cf, int b3, int w)
{
#define BBR_WGS(CF_, B3_, W_) \
    if (cf == CF_ && b3 == B3_ && w == W_) return f32p::Shape<CF_, B3_, W_>::WGS;
    BBR_WGS(1, 16, 16) BBR_WGS(2, 16, 16) BBR_WGS(3, 16, 16) BBR_WGS(4, 16, 16)
    BBR_WGS(1, 32, 16) BBR_WGS(2, 32, 16) BBR_WGS(3, 32, 16) BBR_WGS(4, 32, 16)
    BBR_WGS(1, 16, 4) BBR_WGS(2, 16, 4) BBR_WGS(3, 16, 4) BBR_WGS(4, 16, 4)
#undef BBR_WGS
    return 1;
}

hipError_t launch_f32p(int cf, int b3, int c64, const GemmArgs &a, int grid, hipStream_t st)
{
#define BBR_CASE(CF_, B3_)      \
    if (cf == CF_ && b3 == B3_) \
        return c64 ? f32p::run<CF_, B3_, true>(a, grid, st) : f32p::run<CF_, B3_, false>(a, grid, st);
    BBR_CASE(1, 16) BBR_CASE(2, 16) BBR_CASE(3, 16) BBR_CASE(4, 16)
    BBR_CASE(1, 32) BBR_CASE(2, 32) BBR_CASE(3, 32) BBR_CASE(4, 32)
#undef BBR_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_f32n(int cf, int c64, const GemmArgs &a, int grid, hipStream_t st)
{
#define BBR_CASE(CF_) \
    if (cf == CF_) return c64 ? f32p::run_narrow<CF_, true>(a, grid, st) : f32p::run_narrow<CF_, false>(a, grid, st);
    BBR_CASE(1) BBR_CASE(2) BBR_CASE(3) BBR_CASE(4)
#undef BBR_CASE
    return hipErrorInvalidValue;
}

}  // namespace bb
