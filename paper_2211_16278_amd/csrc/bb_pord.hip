// Paper-order BF16X3 contraction (gfx950): the singlet first, then the
// momentum projection as a small GEMM (paper, Algorithm 1: the singlet loop
// forms S(x; d1,d2,d3) = sum_c D_c(x; d1,d2) q3_c(x; d3), and the projection
// multiplies the singlets by the phases, GEMM with m = (d1,d2,d3), n = momenta,
// k = sites).
//
// Per chunk of 8 sites a workgroup builds the diquark D (Algorithm 1, diquark
// loop) of its (d1,d2) pairs in LDS and stages q3 of its d3 block; each lane
// then forms the singlets of its own GEMM row (one (d1,d2,d3)) for the 4
// sites of its k-group on the VALU, splits them into BF16 hi/lo and feeds
// them as the A operand of v_mfma_f32_32x32x16_bf16 directly from registers.
// The B operand is conj(exp(-i p.x)) over the chunk's sites for 32 momenta
// per column fragment, also built in registers (the phases do not depend on
// the row).  The MFMA work per (site, row) is 8 x 32 NB real flops x 3
// (BF16x3) instead of 24 N_mom for the fused GEMM, at the cost of 3 complex
// multiply-adds and a BF16 split per (site, row) on the VALU; two
// workgroups per CU let one wave's VALU work run under another's MFMAs.
//
// Real embedding on the column side (the B operand is built once per chunk
// and shared by all row fragments): A = (Re S, Im S) along k; the real part
// of S ph comes from B = (Re ph, -Im ph), the imaginary part from
// B = (Im ph, Re ph).
#include "bb_fast.h"

namespace bb {
namespace pord {

using fast::bf8_t;
using fast::cmulf;
using fast::f16_t;
using fast::pack_bf16;
using fast::pin;
using fast::split_lo;
using fast::static_for;

typedef const void __attribute__((address_space(1))) *gvoid;

typedef float f2v_t __attribute__((ext_vector_type(2)));
typedef float f4v_t __attribute__((ext_vector_type(4)));

// Tile shape: NB column fragments of 32 momenta; F row fragments of 32 rows
// per wave (rows = PPF pairs x B3 d3 values); 4 waves.
template <int NB, int B3>
struct Shape {
    static constexpr int F = NB == 1 ? 4 : 2;
    static constexpr int PPF = 32 / B3;        // (d1,d2) pairs per row fragment
    static constexpr int NPAIR = 4 * F * PPF;  // pairs per workgroup
    static constexpr int NCOL = 32 * NB;       // momenta per workgroup
    static constexpr int ND = NPAIR * CHUNK_SITES;       // diquark items per chunk (one per thread at most)
    static constexpr int NQ = 3 * CHUNK_SITES * B3;     // staged q3 values per chunk
    static constexpr int JQ = (NQ + THREADS - 1) / THREADS;
    static_assert(ND <= THREADS, "one diquark item per thread");
};

template <int NB, int B3, bool C64, bool Z>
__global__ void __launch_bounds__(THREADS, 2) contract(GemmArgs a)
{
    static_assert(!Z || NB == 1, "the zero momentum off the matrix cores saves the second fragment");
    using Sh = Shape<NB, B3>;
    using IT = typename fast::InT<C64>::T;
    constexpr int F = Sh::F, PPF = Sh::PPF, NPAIR = Sh::NPAIR;
    constexpr int ESZ = sizeof(IT);
    // D[pair][site][colour] and q3[site][colour][d3], double-buffered over chunks.
    __shared__ __align__(16) float2 dtile[2][NPAIR * CHUNK_SITES * 3];
    __shared__ __align__(16) float2 q3s[2][3 * CHUNK_SITES * B3];
    // Column operands per phase index k: conj(exp(-2 pi i k / L)) split into
    // BF16 hi/lo, as the four dwords (Re-part hi, Re-part lo, Im-part hi,
    // Im-part lo) a lane needs for one site: the real output takes
    // (Re ph, -Im ph), the imaginary one (Im ph, Re ph).
    __shared__ __align__(16) uint32_t bops[MAX_L][4];
    // Z: the zero momentum's site sums of each wave's rows, (Re, Im) per
    // (fragment, row, k-group), accumulated per chunk.
    __shared__ __align__(8) float2 zacc[Z ? 4 * Sh::F * 64 : 1];
    __shared__ int s_tile;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 5, r = lane & 31;
    const int V = a.V, L = a.L;
    for (int k = tid; k < L; k += THREADS) {
        const float c = (float)a.roots[2 * k], sn = (float)a.roots[2 * k + 1];
        const uint32_t hr = pack_bf16(c, -sn), hi = pack_bf16(sn, c);
        bops[k][0] = hr;
        bops[k][1] = split_lo(c, -sn, hr);
        bops[k][2] = hi;
        bops[k][3] = split_lo(sn, c, hi);
    }
    __syncthreads();

    auto next_tile = [&](int current) -> int {
        if (a.counter == nullptr) return current < 0 ? (int)blockIdx.x : a.n_tiles;
        __syncthreads();
        if (tid == 0) s_tile = atomicAdd(&a.counter[0], 1);
        __syncthreads();
        return __builtin_amdgcn_readfirstlane(s_tile);
    };

    // A walking tile runs every split of its block in order: the loop
    // stays on tile t and steps its split (wsp) up to the block's last.
    for (int t = next_tile(-1), wsp = 0; t < a.n_tiles;) {
        const int4 tl0 = wave_uniform(a.tiles[t]);
        const BlockDesc bd = wave_uniform(a.blocks[tl0.x]);
        const int4 tl = make_int4(tl0.x, tl0.y, tl0.z, tl0.w + wsp);
        // m-tile = (pair block, d3 block); n_mt2 holds the number of d3 blocks.
        const int pb = tl.y / bd.n_mt2, d3_0 = (tl.y % bd.n_mt2) * B3;
        const int m12_0 = pb * NPAIR, M12 = bd.n1 * bd.n2;
        const int p0 = tl.z * Sh::NCOL;
        const int xs = tl.w * bd.sps;
        const int xe = min(V, xs + bd.sps);
        const int n_chunks = (xe - xs + CHUNK_SITES - 1) / CHUNK_SITES;

        // Buffer resources over this split's sites (out of range -> 0).
        const int nrec1 = (xe - xs) * 3 * bd.n1 * ESZ, nrec2 = (xe - xs) * 3 * bd.n2 * ESZ;
        const int nrec3 = (xe - xs) * 3 * bd.n3 * ESZ;
        const __amdgpu_buffer_rsrc_t rs1 = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(reinterpret_cast<const IT *>(bd.q1) + (size_t)xs * 3 * bd.n1), (short)0, nrec1, 0x00020000);
        const __amdgpu_buffer_rsrc_t rs2 = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(reinterpret_cast<const IT *>(bd.q2) + (size_t)xs * 3 * bd.n2), (short)0, nrec2, 0x00020000);
        const __amdgpu_buffer_rsrc_t rs3 = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(reinterpret_cast<const IT *>(bd.q3) + (size_t)xs * 3 * bd.n3), (short)0, nrec3, 0x00020000);
        auto ld = [&](__amdgpu_buffer_rsrc_t rs, uint32_t off) -> IT {
            if constexpr (C64)
                return __builtin_bit_cast(IT, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
            else
                return __builtin_bit_cast(IT, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
        };

        // Diquark item of this thread: (pair dp, site dx).
        const int dp = tid / CHUNK_SITES, dx = tid % CHUNK_SITES;
        const int m12 = m12_0 + dp;
        const bool d_ok = tid < Sh::ND && m12 < M12;
        const int d1 = d_ok ? m12 / bd.n2 : 0, d2 = d_ok ? m12 % bd.n2 : 0;
        const uint32_t o1 = d_ok ? (uint32_t)((dx * 3 * bd.n1 + d1) * ESZ) : 0x80000000u;
        const uint32_t o2 = d_ok ? (uint32_t)((dx * 3 * bd.n2 + d2) * ESZ) : 0x80000000u;
        const uint32_t c1 = (uint32_t)(bd.n1 * ESZ), c2 = (uint32_t)(bd.n2 * ESZ);  // colour strides
        const uint32_t s1 = 24u * bd.n1 * ESZ, s2 = 24u * bd.n2 * ESZ, s3 = 24u * bd.n3 * ESZ;  // chunk strides
        // q3 staging slots: element e = tid + 256 j -> (site, colour, d3l).
        uint32_t o3[Sh::JQ];
#pragma unroll
        for (int j = 0; j < Sh::JQ; ++j) {
            const int e = tid + THREADS * j;
            const int d3l = e % B3, c = (e / B3) % 3, x = e / (3 * B3);
            const bool ok = e < Sh::NQ && d3_0 + d3l < bd.n3;
            o3[j] = ok ? (uint32_t)(((x * 3 + c) * bd.n3 + d3_0 + d3l) * ESZ) : 0x80000000u;
        }

        // Phase indices of the lane's column: kidx[p][x] of its 4 sites as one
        // dword (rows padded to 4 bytes; momenta past the set read 0).
        const __amdgpu_buffer_rsrc_t rsk = __builtin_amdgcn_make_buffer_rsrc(
            (void *)a.kidx, (short)0, (int)((uint32_t)a.n_mom * (uint32_t)a.kstride), 0x00020000);
        // Z: the columns hold every momentum but a.p_skip (the zero one).
        const int ps = Z ? a.p_skip : -1, n_col = a.n_mom - (Z ? 1 : 0);
        const int pcol = p0 + r;
        uint32_t ko[NB];
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            const int col = pcol + 32 * n, pm = col + (Z && col >= ps ? 1 : 0);
            ko[n] = col < n_col ? (uint32_t)(pm * a.kstride + xs + 4 * g) : 0x80000000u;
        }
        float2 *zw = zacc + (Z ? wave * F * 64 : 0);  // this wave's rows: [f][g][r]
        if constexpr (Z) {
            for (int i = lane; i < F * 64; i += 64) zw[i] = make_float2(0.f, 0.f);
        }

        IT u[3], v[3], w[Sh::JQ];
        uint32_t kw[NB], kn[NB];
        auto load_chunk = [&](int ci) {
#pragma unroll
            for (int n = 0; n < NB; ++n)
                kn[n] = __builtin_amdgcn_raw_buffer_load_b32(rsk, ko[n] + (uint32_t)ci * CHUNK_SITES, 0, 0);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                u[c] = ld(rs1, o1 + c * c1 + (uint32_t)ci * s1);
                v[c] = ld(rs2, o2 + c * c2 + (uint32_t)ci * s2);
            }
#pragma unroll
            for (int j = 0; j < Sh::JQ; ++j) w[j] = ld(rs3, o3[j] + (uint32_t)ci * s3);
        };
        // D_c = eps_abc q1_a q2_b of the thread's item, and the q3 staging, into buffer b.
        auto store_chunk = [&](int b) {
            float2 uf[3], vf[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                uf[c] = make_float2((float)u[c].x, (float)u[c].y);
                vf[c] = make_float2((float)v[c].x, (float)v[c].y);
            }
            if (tid < Sh::ND) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int a_ = (c + 1) % 3, b_ = (c + 2) % 3;  // eps_{a b c} = +1
                    const float2 d = fast::diqf(uf[a_], uf[b_], vf[a_], vf[b_]);
                    *reinterpret_cast<f2v_t *>(&dtile[b][(dp * CHUNK_SITES + dx) * 3 + c]) = f2v_t{d.x, d.y};
                }
            }
#pragma unroll
            for (int j = 0; j < Sh::JQ; ++j) {
                const int e = tid + THREADS * j;
                if (e < Sh::NQ)
                    *reinterpret_cast<f2v_t *>(&q3s[b][e]) = f2v_t{(float)w[j].x, (float)w[j].y};
            }
        };


        f16_t acc[F][NB][2];
#pragma unroll
        for (int f = 0; f < F; ++f)
#pragma unroll
            for (int n = 0; n < NB; ++n)
#pragma unroll
                for (int s = 0; s < 2; ++s)
#pragma unroll
                    for (int e = 0; e < 16; ++e) acc[f][n][s][e] = 0.f;

        load_chunk(0);
        store_chunk(0);
#pragma unroll
        for (int n = 0; n < NB; ++n) kw[n] = kn[n];
        load_chunk(1);
        __syncthreads();

        for (int i = 0; i < n_chunks; ++i) {
            const int b = i & 1;
            // B operands of the lane's column over its 4 sites: (Re ph, -Im ph)
            // gives the real part of S ph, (Im ph, Re ph) the imaginary part.
            uint4 bh[NB][2], bl[NB][2];
#pragma unroll
            for (int n = 0; n < NB; ++n) {
                uint32_t k4[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) k4[j] = (kw[n] >> (8 * j)) & 0xffu;
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    bh[n][s] = make_uint4(bops[k4[0]][2 * s], bops[k4[1]][2 * s], bops[k4[2]][2 * s], bops[k4[3]][2 * s]);
                    bl[n][s] = make_uint4(bops[k4[0]][2 * s + 1], bops[k4[1]][2 * s + 1], bops[k4[2]][2 * s + 1],
                                          bops[k4[3]][2 * s + 1]);
                }
            }
            // q3 of the lane's d3 for its 4 sites, reused by all row fragments.
            const int d3l = r % B3;
            float2 q[4][3];
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const f2v_t t = *reinterpret_cast<const f2v_t *>(&q3s[b][((4 * g + j) * 3 + c) * B3 + d3l]);
                    q[j][c] = make_float2(t.x, t.y);
                }
            if constexpr (NB == 1) {
                // Singlet S = sum_c D_c q3_c of row fragment f split into BF16
                // hi/lo, in 17 steps: the 12 D reads, then per site the Re chain,
                // the Im chain, the hi pack and the lo split.  Fragment 0's runs
                // before its MFMAs, fragment f+1's between fragment f's (double-
                // buffered hi/lo): the D reads alone after the first MFMA, so
                // that their latency runs under the second, the 16 arithmetic
                // steps spread over the five slots after it.
                float2 dvf[12];
                float sre = 0.f, sim = 0.f;
                float zre = 0.f, zim = 0.f;  // Z: the fragment's singlets over the lane's 4 sites
                uint32_t sh[2][4], sl[2][4];
                auto singlet = [&](auto ff, auto ss) {
                    constexpr int f = ff, st = ss, B = f & 1;
                    if constexpr (Z && st == 0) {
                        zre = 0.f;
                        zim = 0.f;
                    }
                    if constexpr (Z && st == 16) {
                        // Each lane adds its k-group's sums into a slot of its
                        // own (the lane's (f, g, r)): no two lanes meet.
                        float2 *zp = &zw[f * 64 + lane];
                        const float2 z = *zp;
                        *zp = make_float2(z.x + zre, z.y + zim);
                    }
                    if constexpr (st == 0) {
                        const int pi = (wave * F + f) * PPF + r / B3;  // pair of the lane's row
                        const float2 *D = &dtile[b][(pi * CHUNK_SITES + 4 * g) * 3];
#pragma unroll
                        for (int k = 0; k < 12; ++k) dvf[k] = D[k];
                    } else {
                        constexpr int s1 = st - 1, j = s1 / 4, part = s1 % 4;
                        if constexpr (part == 0) {
                            sre = 0.f;
#pragma unroll
                            for (int c = 0; c < 3; ++c) {
                                sre = __builtin_fmaf(dvf[j * 3 + c].x, q[j][c].x, sre);
                                sre = __builtin_fmaf(-dvf[j * 3 + c].y, q[j][c].y, sre);
                            }
                            pin(sre);
                            if constexpr (Z) zre += sre;
                        } else if constexpr (part == 1) {
                            sim = 0.f;
#pragma unroll
                            for (int c = 0; c < 3; ++c) {
                                sim = __builtin_fmaf(dvf[j * 3 + c].x, q[j][c].y, sim);
                                sim = __builtin_fmaf(dvf[j * 3 + c].y, q[j][c].x, sim);
                            }
                            pin(sim);
                            if constexpr (Z) zim += sim;
                        } else if constexpr (part == 2) {
                            sh[B][j] = pack_bf16(sre, sim);
                            pin(sh[B][j]);
                        } else {
                            sl[B][j] = split_lo(sre, sim, sh[B][j]);
                            pin(sl[B][j]);
                        }
                    }
                };
                constexpr int NSTEP = 17, NSLOT = 6 * NB;
                static_for<0, NSTEP>([&](auto ss) { singlet(std::integral_constant<int, 0>{}, ss); });
                static_for<0, F>([&](auto ff) {
                    constexpr int f = ff, B = f & 1;
                    const bf8_t Ah = __builtin_bit_cast(bf8_t, make_uint4(sh[B][0], sh[B][1], sh[B][2], sh[B][3]));
                    const bf8_t Al = __builtin_bit_cast(bf8_t, make_uint4(sl[B][0], sl[B][1], sl[B][2], sl[B][3]));
                    // Products in the order lo.hi, hi.lo, hi.hi for every
                    // accumulator, the accumulators interleaved.
                    static_for<0, NSLOT>([&](auto kk) {
                        constexpr int k = kk, prod = k / (2 * NB), n = (k % (2 * NB)) / 2, sp = k % 2;
                        // Steps of fragment f+1 after this MFMA: step 0 (the D
                        // reads) after the first, steps 1..16 over the rest.
                        constexpr int s_lo = k == 0 ? 0 : 1 + ((k - 1) * (NSTEP - 1) + NSLOT - 2) / (NSLOT - 1);
                        constexpr int s_hi = 1 + (k * (NSTEP - 1) + NSLOT - 2) / (NSLOT - 1);
                        const bf8_t Bh = __builtin_bit_cast(bf8_t, bh[n][sp]), Bl = __builtin_bit_cast(bf8_t, bl[n][sp]);
                        acc[f][n][sp] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(prod == 0 ? Al : Ah, prod == 1 ? Bl : Bh,
                                                                                 acc[f][n][sp], 0, 0, 0);
                        __builtin_amdgcn_sched_barrier(0);
                        if constexpr (f + 1 < F)
                            static_for<s_lo, s_hi>([&](auto ss) { singlet(std::integral_constant<int, f + 1>{}, ss); });
                        __builtin_amdgcn_sched_barrier(0);
                    });
                });
            } else {
                // Two column fragments: the pipelined form above needs more
                // registers than the two-workgroup occupancy leaves (it spills
                // in the loop and runs slower), so the singlet of each row
                // fragment is formed before its MFMAs.
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    const int pi = (wave * F + f) * PPF + r / B3;  // pair of the lane's row
                    const float2 *D = &dtile[b][(pi * CHUNK_SITES + 4 * g) * 3];
                    uint32_t sh[4], sl[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        float re = 0.f, im = 0.f;
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            const float2 dv = D[j * 3 + c];
                            re = __builtin_fmaf(dv.x, q[j][c].x, re);
                            re = __builtin_fmaf(-dv.y, q[j][c].y, re);
                            im = __builtin_fmaf(dv.x, q[j][c].y, im);
                            im = __builtin_fmaf(dv.y, q[j][c].x, im);
                        }
                        sh[j] = pack_bf16(re, im);
                        sl[j] = split_lo(re, im, sh[j]);
                    }
                    const bf8_t Ah = __builtin_bit_cast(bf8_t, make_uint4(sh[0], sh[1], sh[2], sh[3]));
                    const bf8_t Al = __builtin_bit_cast(bf8_t, make_uint4(sl[0], sl[1], sl[2], sl[3]));
#pragma unroll
                    for (int n = 0; n < NB; ++n)
#pragma unroll
                        for (int s = 0; s < 2; ++s) {
                            const bf8_t Bh = __builtin_bit_cast(bf8_t, bh[n][s]), Bl = __builtin_bit_cast(bf8_t, bl[n][s]);
                            acc[f][n][s] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Al, Bh, acc[f][n][s], 0, 0, 0);
                            acc[f][n][s] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah, Bl, acc[f][n][s], 0, 0, 0);
                            acc[f][n][s] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah, Bh, acc[f][n][s], 0, 0, 0);
                        }
                }
            }
            // Next chunk's diquark and q3 into the other buffer; loads two ahead.
            store_chunk(b ^ 1);
#pragma unroll
            for (int n = 0; n < NB; ++n) kw[n] = kn[n];
            load_chunk(i + 2);
            __syncthreads();
        }

        // Epilogue: row (pair, d3), column p; Re/Im fragment s.  A later
        // split of a walking tile adds to out (put_result's PUT_ADD);
        // otherwise the tile stores to out (one split, or a walking tile's
        // first) or its split partial.  Written out here rather than through
        // put_result: in this kernel that form, or one copy of the loops per
        // write mode, makes the compiler spill in the contraction loops.
        if (bd.walk && tl.w > 0) {
#pragma unroll
            for (int f = 0; f < F; ++f)
#pragma unroll
                for (int n = 0; n < NB; ++n) {
                    const int col = pcol + 32 * n, p = col + (Z && col >= ps ? 1 : 0);
                    if (col >= n_col) continue;
#pragma unroll
                    for (int s = 0; s < 2; ++s)
#pragma unroll
                        for (int e = 0; e < 16; ++e) {
                            const int row = 8 * (e >> 2) + 4 * g + (e & 3);
                            const int pi = (wave * F + f) * PPF + row / B3;
                            const int m = m12_0 + pi, d3 = d3_0 + row % B3;
                            if (m >= M12 || d3 >= bd.n3) continue;
                            (void)unsafeAtomicAdd(bd.out + (((size_t)p * M12 + m) * bd.n3 + d3) * 2 + s,
                                                  (double)acc[f][n][s][e]);
                        }
                }
            if constexpr (Z) {
                if (tl.z == 0) {
#pragma unroll
                    for (int f = 0; f < F; ++f) {
                        const int pi = (wave * F + f) * PPF + r / B3;
                        const int m = m12_0 + pi, d3 = d3_0 + r % B3;
                        if (m >= M12 || d3 >= bd.n3) continue;
                        const float2 z0 = zw[f * 64 + r], z1 = zw[f * 64 + 32 + r];
                        const float v = g ? z0.y + z1.y : z0.x + z1.x;
                        (void)unsafeAtomicAdd(bd.out + (((size_t)ps * M12 + m) * bd.n3 + d3) * 2 + g, (double)v);
                    }
                }
            }
        } else {
#pragma unroll
            for (int f = 0; f < F; ++f)
#pragma unroll
                for (int n = 0; n < NB; ++n) {
                    const int col = pcol + 32 * n, p = col + (Z && col >= ps ? 1 : 0);
                    if (col >= n_col) continue;
#pragma unroll
                    for (int s = 0; s < 2; ++s)
#pragma unroll
                        for (int e = 0; e < 16; ++e) {
                            const int row = 8 * (e >> 2) + 4 * g + (e & 3);
                            const int pi = (wave * F + f) * PPF + row / B3;
                            const int m = m12_0 + pi, d3 = d3_0 + row % B3;
                            if (m >= M12 || d3 >= bd.n3) continue;
                            if (bd.direct || bd.walk)
                                bd.out[(((size_t)p * M12 + m) * bd.n3 + d3) * 2 + s] = (double)acc[f][n][s][e];
                            else
                                reinterpret_cast<float *>(bd.ws)[(((size_t)tl.w * 2 + s) * M12 + m) * bd.N + p * bd.n3 + d3] =
                                    acc[f][n][s][e];
                        }
                }
            if constexpr (Z) {
                // The zero momentum's sums: lanes of k-group g write part g.
                if (tl.z == 0) {
#pragma unroll
                    for (int f = 0; f < F; ++f) {
                        const int pi = (wave * F + f) * PPF + r / B3;
                        const int m = m12_0 + pi, d3 = d3_0 + r % B3;
                        if (m >= M12 || d3 >= bd.n3) continue;
                        const float2 z0 = zw[f * 64 + r], z1 = zw[f * 64 + 32 + r];
                        const float v = g ? z0.y + z1.y : z0.x + z1.x;
                        if (bd.direct || bd.walk)
                            bd.out[(((size_t)ps * M12 + m) * bd.n3 + d3) * 2 + g] = (double)v;
                        else
                            reinterpret_cast<float *>(bd.ws)[(((size_t)tl.w * 2 + g) * M12 + m) * bd.N + ps * bd.n3 + d3] = v;
                    }
                }
            }
        }
        if (bd.walk && tl.w + 1 < bd.S) {
            ++wsp;
            __syncthreads();  // the split's last LDS reads come before the next split's writes
        } else {
            wsp = 0;
            t = next_tile(t);
        }
    }

    if (a.counter != nullptr && tid == 0) {
        __threadfence();
        if (atomicAdd(&a.counter[1], 1) == (int)gridDim.x - 1) {
            atomicExch(&a.counter[0], 0);
            atomicExch(&a.counter[1], 0);
        }
    }
}

template <int NB, int B3, bool C64>
hipError_t run(const GemmArgs &a, int grid, hipStream_t st)
{
    if constexpr (NB == 1) {
        if (a.p_skip >= 0) {
            contract<NB, B3, C64, true><<<dim3(grid), dim3(THREADS), 0, st>>>(a);
            return hipGetLastError();
        }
    } else if (a.p_skip >= 0) {
        return hipErrorInvalidValue;
    }
    contract<NB, B3, C64, false><<<dim3(grid), dim3(THREADS), 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace pord

int pord_pairs(int nb, int b3)
{
    if (nb == 1 && b3 == 32) return pord::Shape<1, 32>::NPAIR;
    if (nb == 1 && b3 == 16) return pord::Shape<1, 16>::NPAIR;
    if (nb == 2 && b3 == 32) return pord::Shape<2, 32>::NPAIR;
    if (nb == 2 && b3 == 16) return pord::Shape<2, 16>::NPAIR;
    return -1;
}

hipError_t launch_pord(int nb, int b3, int c64, const GemmArgs &a, int grid, hipStream_t st)
{
#define BBP_CASE(NB_, B3_) \
    if (nb == NB_ && b3 == B3_) return c64 ? pord::run<NB_, B3_, true>(a, grid, st) : pord::run<NB_, B3_, false>(a, grid, st);
    BBP_CASE(1, 32) BBP_CASE(1, 16) BBP_CASE(2, 32) BBP_CASE(2, 16)
#undef BBP_CASE
    return hipErrorInvalidValue;
}

}  // namespace bb
