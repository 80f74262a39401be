// Pipelined contraction kernel of libbblock.so for the FP32 and BF16X3 paths
// (gfx950).  Same contraction as bb_kernels.hip (paper, Sec. 2, eq. (3) as
// one complex GEMM over kappa = (colour, site) with the diquark of
// Algorithm 1 as the row operand and the phase-weighted third quark as the
// column operand), organised so that every stage overlaps another:
//
//   global -> registers : the unique quark values of chunk i+3 are loaded
//                         while chunk i is multiplied;
//   registers -> staging: one LDS staging tile (complex FP32) per chunk;
//   staging -> D/W tiles: the diquark and W tiles of chunk i+1 are built
//                         (VALU) into one of two LDS buffers while the MFMAs
//                         of chunk i read the other buffer.
//
// Tiles are rectangles: rows (d1, d2) in a B1 x B2 block (B1*B2 = 128),
// columns (p, d3) in a bp x B3 block (bp*B3 <= 32*NB).  A workgroup of 4
// wave64 owns one (m-tile, n-tile, site split); wave w owns complex rows
// [32w, 32w+32) and all columns.  The phase exp(-i p.x) comes from the
// per-momentum-set table kidx[p][x] = (n_p . x) mod L and the L roots of
// unity (paper, Sec. 3: the phase is precomputed and reused).
#pragma once

#include <algorithm>
#include <type_traits>

#include "bb_internal.h"

namespace bb {
namespace fast {

typedef float f16_t __attribute__((ext_vector_type(16)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf2_t __attribute__((ext_vector_type(2)));

constexpr int MT = 128;  // complex rows per workgroup

// u32 offsets of tile rows (24 words = one chunk of kappa per row, plus
// padding).  The fragment accesses put row r = lane % 32 (and k-group
// lane / 32, +4 words) on each lane; on gfx950 these 128-bit accesses are
// free of LDS bank conflicts (SQ_LDS_BANK_CONFLICT = 0, measured per layout
// with a probe kernel) for
//   W tiles, read as B fragments: 24 r + 4 (r >> 4);
//   D tiles, read as A fragments and written row per lane: 28 r;
// while the earlier 24 r + 4 (r >> 2) costs about four conflict cycles per
// read.  Both are additive over 32-row fragments: f(32 n + r) = f(32 n) + f(r).
__host__ __device__ constexpr int wrow(int r) { return r * 24 + (r >> 4) * 4; }
__host__ __device__ constexpr int drow(int r) { return r * 28; }

template <int NB, int B2, int B3>
struct Layout {
    static constexpr int NT = 32 * NB;        // complex columns per workgroup
    static constexpr int B1 = MT / B2;
    static constexpr int BPM = NT / B3;       // momentum slots per n-tile
    static constexpr int IPW = 32 / B3;       // momentum slots per wave per W round
    static constexpr int JW = (BPM + 4 * IPW - 1) / (4 * IPW);  // W rounds
    static constexpr int DPL = drow(MT);   // u32 per D plane
    static constexpr int WPL = wrow(NT);   // u32 per W plane
    static constexpr int DW = 2 * DPL + 2 * WPL;
    static constexpr int E1 = 24 * B1, E2 = 24 * B2, E3 = 24 * B3, EPH = 8 * BPM;
    static constexpr int SG = E1 + E2 + E3 + EPH;  // float2 per staging tile
    static constexpr int SINK = 64;                 // float2 slots written by idle lanes
    static constexpr int J1 = (E1 + 255) / 256, J2 = (E2 + 255) / 256, J3 = (E3 + 255) / 256;
    static constexpr int JL = J1 + J2 + J3;
    static_assert(EPH <= 256, "phase slots per chunk exceed one per thread");
    static_assert(B1 % 4 == 0 || B1 == 4, "rows must split over four waves");
    static size_t bytes(int L) { return (size_t)2 * DW * 4 + (size_t)(SG + SINK) * 8 + (size_t)L * 8; }
};

__device__ __forceinline__ uint32_t pack_bf16(float a, float b)
{
    bf2_t v = {(__bf16)a, (__bf16)b};  // round to nearest even
    return __builtin_bit_cast(uint32_t, v);
}

// Residual of the BF16 split of (a, b) given hi = pack_bf16(a, b).  The low
// half is widened with a byte permute so that the compiler keeps using hi.
__device__ __forceinline__ uint32_t split_lo(float a, float b, uint32_t hi)
{
    const float ha = __uint_as_float(__builtin_amdgcn_perm(hi, hi, 0x01000c0cu));
    const float hb = __uint_as_float(hi & 0xffff0000u);
    return pack_bf16(a - ha, b - hb);
}

// Keeps a computed value at this point of the instruction stream: the empty
// asm statement reads and rewrites it, so the arithmetic that produces it
// cannot sink past the scheduling barrier that follows (work spread one step
// per MFMA slot would otherwise gather next to its first use).
template <class T>
__device__ __forceinline__ void pin(T &x)
{
    asm volatile("" : "+v"(x));
}

// Complex product with a fixed rounding sequence (one rounded product, then
// one fused multiply-add per part), so that every kernel that forms the same
// product gets the same bits whatever the compiler's contraction choices.
__device__ __forceinline__ float2 cmulf(float2 a, float2 b)
{
    return make_float2(__builtin_fmaf(a.x, b.x, -(a.y * b.y)), __builtin_fmaf(a.x, b.y, a.y * b.x));
}

// Diquark colour component ua vb - ub va (Algorithm 1's cross product) as two
// chains of one product and three fused multiply-adds: 8 VALU operations
// instead of the 10 of two complex products and a difference, with the same
// fixed rounding sequence in every kernel.
__device__ __forceinline__ float diq_re(float2 ua, float2 ub, float2 va, float2 vb)
{
    return __builtin_fmaf(ua.x, vb.x, __builtin_fmaf(-ua.y, vb.y, __builtin_fmaf(-ub.x, va.x, ub.y * va.y)));
}
__device__ __forceinline__ float diq_im(float2 ua, float2 ub, float2 va, float2 vb)
{
    return __builtin_fmaf(ua.x, vb.y, __builtin_fmaf(ua.y, vb.x, __builtin_fmaf(-ub.x, va.y, -(ub.y * va.x))));
}
__device__ __forceinline__ float2 diqf(float2 ua, float2 ub, float2 va, float2 vb)
{
    return make_float2(diq_re(ua, ub, va, vb), diq_im(ua, ub, va, vb));
}

// Four complex values of one tile row (4 consecutive kappa) into the two planes.
template <int P>
__device__ __forceinline__ void store4(uint32_t *p0, uint32_t *p1, int off, const float2 (&v)[4])
{
    uint4 a, b;
    if constexpr (P == BF16X3) {
        uint32_t hi[4], lo[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            hi[i] = pack_bf16(v[i].x, v[i].y);
            lo[i] = pack_bf16(v[i].x - __uint_as_float(hi[i] << 16), v[i].y - __uint_as_float(hi[i] & 0xffff0000u));
        }
        a = make_uint4(hi[0], hi[1], hi[2], hi[3]);
        b = make_uint4(lo[0], lo[1], lo[2], lo[3]);
    } else {
        a = make_uint4(__float_as_uint(v[0].x), __float_as_uint(v[1].x), __float_as_uint(v[2].x), __float_as_uint(v[3].x));
        b = make_uint4(__float_as_uint(v[0].y), __float_as_uint(v[1].y), __float_as_uint(v[2].y), __float_as_uint(v[3].y));
    }
    *reinterpret_cast<uint4 *>(p0 + off) = a;
    *reinterpret_cast<uint4 *>(p1 + off) = b;
}

// Diquark tile of one chunk from the staging tile: lane -> (i1, i2, site
// group of 4); D_c = eps_abc q1_a q2_b for the 3 colours and 4 sites.
template <int P, int NB, int B2, int B3>
__device__ __forceinline__ void gen_d(uint32_t *buf, const float2 *stg, int lane, int wave)
{
    using Lt = Layout<NB, B2, B3>;
    const float2 *S1 = stg, *S2 = stg + Lt::E1;
    uint32_t *D0 = buf, *D1 = buf + Lt::DPL;
    const int i2 = lane % B2, xg = (lane / B2) & 1, i1 = wave * (Lt::B1 / 4) + lane / (2 * B2);
    const int off = drow(i1 * B2 + i2) + 4 * xg;
    float2 d[3][4];
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        float2 u[3], v[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            u[a] = S1[(a * 8 + 4 * xg + x) * Lt::B1 + i1];
            v[a] = S2[(a * 8 + 4 * xg + x) * B2 + i2];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int a = (c + 1) % 3, b = (c + 2) % 3;  // eps_{a b c} = +1
            d[c][x] = diqf(u[a], u[b], v[a], v[b]);
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) store4<P>(D0, D1, off + 8 * c, d[c]);
}

// Round j of the W tile: lane -> (i3, site group, momentum slot);
// W_c = q3_c * exp(-i p.x).  Waves past the last momentum slot redo round 0
// (identical data to identical addresses) instead of branching.
template <int P, int NB, int B2, int B3>
__device__ __forceinline__ void gen_w(uint32_t *buf, const float2 *stg, int j, int lane, int wave)
{
    using Lt = Layout<NB, B2, B3>;
    const float2 *S3 = stg + Lt::E1 + Lt::E2, *PH = S3 + Lt::E3;
    uint32_t *W0 = buf + 2 * Lt::DPL, *W1 = W0 + Lt::WPL;
    const int i3 = lane % B3, xg = (lane / B3) & 1, ipl = lane / (2 * B3);
    const bool live = (wave + 4 * j) < NB;
    const int ip = wave * Lt::IPW + ipl + (live ? 4 * Lt::IPW * j : 0);
    const int off = wrow(ip * B3 + i3) + 4 * xg;
    float2 ph[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) ph[x] = PH[ip * 8 + 4 * xg + x];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float2 w[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) w[x] = cmulf(S3[(c * 8 + 4 * xg + x) * B3 + i3], ph[x]);
        store4<P>(W0, W1, off + 8 * c, w);
    }
}

// MFMAs of colour c of one chunk (8 kappa).
template <int P, int NB, int B2, int B3>
__device__ __forceinline__ void multiply(const uint32_t *buf, int c, f16_t (&acc)[2][NB], int lane, int wave)
{
    using Lt = Layout<NB, B2, B3>;
    const uint32_t *D0 = buf, *D1 = buf + Lt::DPL, *W0 = buf + 2 * Lt::DPL, *W1 = W0 + Lt::WPL;
    const int g = lane >> 5, r = lane & 31;
    const bool im_row = r >= 16;
    if constexpr (P == BF16X3) {
        // Lane i + 32g holds 4 kappa (Re, Im pairs) of one row / column.
        // Row side real embedding: Re-row (Re, -Im), Im-row (Im, Re).
        const uint32_t sel = im_row ? 0x01000302u : 0x03020100u;
        const uint32_t flip = im_row ? 0u : 0x80000000u;
        const int aoff = drow(wave * 32 + (r & 15)) + 4 * g + 8 * c;
        const int boff = wrow(r) + 4 * g + 8 * c;
        bf8_t ah[2], al[2];
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            uint4 h = *reinterpret_cast<const uint4 *>(D0 + aoff + f * drow(16));
            uint4 l = *reinterpret_cast<const uint4 *>(D1 + aoff + f * drow(16));
            h = make_uint4(__builtin_amdgcn_perm(h.x, h.x, sel) ^ flip, __builtin_amdgcn_perm(h.y, h.y, sel) ^ flip,
                           __builtin_amdgcn_perm(h.z, h.z, sel) ^ flip, __builtin_amdgcn_perm(h.w, h.w, sel) ^ flip);
            l = make_uint4(__builtin_amdgcn_perm(l.x, l.x, sel) ^ flip, __builtin_amdgcn_perm(l.y, l.y, sel) ^ flip,
                           __builtin_amdgcn_perm(l.z, l.z, sel) ^ flip, __builtin_amdgcn_perm(l.w, l.w, sel) ^ flip);
            ah[f] = __builtin_bit_cast(bf8_t, h);
            al[f] = __builtin_bit_cast(bf8_t, l);
        }
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            const bf8_t bh = __builtin_bit_cast(bf8_t, *reinterpret_cast<const uint4 *>(W0 + boff + n * wrow(32)));
            const bf8_t bl = __builtin_bit_cast(bf8_t, *reinterpret_cast<const uint4 *>(W1 + boff + n * wrow(32)));
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                acc[f][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[f], bh, acc[f][n], 0, 0, 0);
                acc[f][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[f], bl, acc[f][n], 0, 0, 0);
                acc[f][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[f], bh, acc[f][n], 0, 0, 0);
            }
        }
    } else {
        // FP32: A[i][k] from lane i + 32k, k = t = Re/Im part of one kappa.
        const int t = g, s = im_row ? 1 : 0;
        const uint32_t *Ap = (s ^ t) ? D1 : D0;
        const uint32_t flip = (s == 0 && t == 1) ? 0x80000000u : 0u;
        const uint32_t *Bp = t ? W1 : W0;
        const int aoff = drow(wave * 32 + (r & 15)) + 8 * c;
        const int boff = wrow(r) + 8 * c;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            float av[2][4];
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                const uint4 v = *reinterpret_cast<const uint4 *>(Ap + aoff + f * drow(16) + 4 * h);
                av[f][0] = __uint_as_float(v.x ^ flip);
                av[f][1] = __uint_as_float(v.y ^ flip);
                av[f][2] = __uint_as_float(v.z ^ flip);
                av[f][3] = __uint_as_float(v.w ^ flip);
            }
#pragma unroll
            for (int n = 0; n < NB; ++n) {
                const uint4 v = *reinterpret_cast<const uint4 *>(Bp + boff + n * wrow(32) + 4 * h);
                const float bv[4] = {__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z), __uint_as_float(v.w)};
#pragma unroll
                for (int k = 0; k < 4; ++k)
#pragma unroll
                    for (int f = 0; f < 2; ++f)
                        acc[f][n] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[f][k], bv[k], acc[f][n], 0, 0, 0);
            }
        }
    }
}

// Global-memory (address space 1) pointers: loads through them are
// global_load, which count only on vmcnt, so LDS waits never wait on HBM.
template <class T>
using gptr = const T __attribute__((address_space(1))) *;

// Compile-time loop: f(integral_constant<int, I>) for I in [B, E).
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Slot K of SLOTS runs the sub-steps [ceil(K*NSUB/SLOTS), ceil((K+1)*NSUB/SLOTS))
// of a piece of work split into NSUB sub-steps.
template <int K, int SLOTS, int NSUB, class F>
__device__ __forceinline__ void slot_steps(F &&f)
{
    static_for<(K * NSUB + SLOTS - 1) / SLOTS, ((K + 1) * NSUB + SLOTS - 1) / SLOTS>(f);
}

__device__ __forceinline__ bf8_t embed(uint4 v, uint32_t sel, uint32_t flip)
{
    return __builtin_bit_cast(bf8_t, make_uint4(__builtin_amdgcn_perm(v.x, v.x, sel) ^ flip,
                                                __builtin_amdgcn_perm(v.y, v.y, sel) ^ flip,
                                                __builtin_amdgcn_perm(v.z, v.z, sel) ^ flip,
                                                __builtin_amdgcn_perm(v.w, v.w, sel) ^ flip));
}

// Scheduling pattern of one section: each MFMA followed by NV VALU and ND LDS
// instructions, so the VALU work of the generation issues while the matrix
// core is busy (one wave per SIMD: overlap has to come from within the wave).
template <int NM, int NV, int ND>
__device__ __forceinline__ void interleave()
{
#pragma unroll
    for (int k = 0; k < NM; ++k) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
        if constexpr (NV > 0) __builtin_amdgcn_sched_group_barrier(0x002, NV, 0);  // VALU
        if constexpr (ND > 0) __builtin_amdgcn_sched_group_barrier(0x080, ND, 0);  // LDS
    }
}

// Instruction estimates per section and wave, for the interleave patterns.
template <int P, int NB, int B2, int B3>
struct Sched {
    using Lt = Layout<NB, B2, B3>;
    static constexpr int SPLIT = P == BF16X3 ? 7 : 0;  // VALU per complex hi/lo split
    static constexpr int XFORM = P == BF16X3 ? 32 : 16; // row-embedding VALU per colour
    static constexpr int MF = P == BF16X3 ? 6 * NB : 16 * NB;  // MFMAs per colour
    static constexpr int V_D = 12 * (10 + SPLIT) + XFORM;
    static constexpr int V_W = Lt::JW * 12 * (4 + SPLIT) + XFORM;
    static constexpr int V_S = 4 * Lt::JL + 12 + XFORM;
    static constexpr int cd(int a, int b) { return (a + b - 1) / b; }
    static constexpr int NV_D = cd(V_D, MF), NV_W = cd(V_W, MF), NV_S = cd(V_S, MF);
};

// Complex input element as a native vector (loads through address-space-1
// pointers need a trivially copyable type).
template <bool C64>
struct InT {
    using T = double __attribute__((ext_vector_type(2)));
};
template <>
struct InT<true> {
    using T = float __attribute__((ext_vector_type(2)));
};

template <int P, int NB, int B2, int B3, bool C64>
__global__ void __launch_bounds__(THREADS, 1) bb_fast(GemmArgs a)
{
    using Lt = Layout<NB, B2, B3>;
    using IT = typename InT<C64>::T;
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *dwbuf = reinterpret_cast<uint32_t *>(smem);
    float2 *stg = reinterpret_cast<float2 *>(smem + 2 * Lt::DW * 4);
    float2 *roots = stg + Lt::SG + Lt::SINK;
    __shared__ int s_tile;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int V = a.V;
    for (int k = tid; k < a.L; k += THREADS) roots[k] = make_float2((float)a.roots[2 * k], (float)a.roots[2 * k + 1]);
    __syncthreads();

    auto next_tile = [&](int current) -> int {
        if (a.counter == nullptr) return current < 0 ? (int)blockIdx.x : a.n_tiles;
        __syncthreads();
        if (tid == 0) s_tile = atomicAdd(&a.counter[0], 1);
        __syncthreads();
        return s_tile;
    };

    // A walking tile runs every split of its block in order: the loop
    // stays on tile t and steps its split (wsp) up to the block's last.
    for (int t = next_tile(-1), wsp = 0; t < a.n_tiles;) {
        const int4 tl0 = wave_uniform(a.tiles[t]);
        const BlockDesc bd = wave_uniform(a.blocks[tl0.x]);
        const int4 tl = make_int4(tl0.x, tl0.y, tl0.z, tl0.w + wsp);
        const int d1_0 = (tl.y / bd.n_mt2) * Lt::B1, d2_0 = (tl.y % bd.n_mt2) * B2;
        const int p0 = (tl.z / bd.n_nt3) * bd.bp, d3_0 = (tl.z % bd.n_nt3) * B3;
        const int xs = tl.w * bd.sps;
        const int xe = min(V, xs + bd.sps);
        const int n_chunks = (xe - xs + CHUNK_SITES - 1) / CHUNK_SITES;

        // Per-thread staging elements (tile invariant part): element e of
        // array k is (colour c, site x, index i) with e = i + B_k (x + 8c).
        // Slots [0, J1) load q1, [J1, J1+J2) q2, the rest q3.
        // Packed per slot: bits 0-13 element offset c*n + d0 + i (< 3*4096),
        // 14-25 staging destination, 26-28 site, 29 index in range.
        unsigned plan[Lt::JL];
        auto plan_slot = [&](int q, int j, int n_k, int d0_k, int B_k, int E_k, int sofs_k) {
            const int e = tid + 256 * j;
            const int i = e % B_k, x = (e / B_k) % 8, c = e / (8 * B_k);
            const bool live = e < E_k;
            const bool dok = live && (d0_k + i < n_k);
            const unsigned ofs = dok ? (unsigned)(c * n_k + d0_k + i) : 0u;
            const unsigned dst = live ? (unsigned)(sofs_k + e) : (unsigned)(Lt::SG + lane);
            plan[q] = ofs | (dst << 14) | ((unsigned)x << 26) | (dok ? (1u << 29) : 0u);
        };
#pragma unroll
        for (int j = 0; j < Lt::J1; ++j) plan_slot(j, j, bd.n1, d1_0, Lt::B1, Lt::E1, 0);
#pragma unroll
        for (int j = 0; j < Lt::J2; ++j) plan_slot(Lt::J1 + j, j, bd.n2, d2_0, B2, Lt::E2, Lt::E1);
#pragma unroll
        for (int j = 0; j < Lt::J3; ++j) plan_slot(Lt::J1 + Lt::J2 + j, j, bd.n3, d3_0, B3, Lt::E3, Lt::E1 + Lt::E2);
        // Phase slot of this thread: (momentum slot ip, site x).
        const int ph_ip = (tid / 8), ph_x = tid % 8;
        const bool ph_live = tid < Lt::EPH;
        const bool ph_ok = ph_live && ph_ip < bd.bp && (p0 + ph_ip) < a.n_mom;
        const int ph_dst = ph_live ? Lt::E1 + Lt::E2 + Lt::E3 + tid : Lt::SG + lane;
        const gptr<unsigned char> kp = (gptr<unsigned char>)(a.kidx + (size_t)(ph_ok ? p0 + ph_ip : 0) * a.kstride);
        const gptr<IT> q1p = (gptr<IT>)bd.q1;
        const gptr<IT> q2p = (gptr<IT>)bd.q2;
        const gptr<IT> q3p = (gptr<IT>)bd.q3;

        IT rv[Lt::JL];
        unsigned okbits = 0;
        int kval = 0;
        // Out-of-range elements load element 0 (always valid) and are
        // zeroed at the staging store; masks instead of branches keep the
        // whole loop body one scheduling region.
        auto load_slot = [&](int q, gptr<IT> basep, int n_k, int x0) {
            const int xa = x0 + (int)((plan[q] >> 26) & 7u);
            const unsigned ok = ((plan[q] >> 29) & 1u) & (unsigned)(xa < xe);
            const int idx = (xa * 3 * n_k + (int)(plan[q] & 0x3fffu)) & -(int)ok;
            rv[q] = basep[idx];
            okbits |= ok << q;
        };
        auto issue_loads = [&](int ci) {
            const int x0 = xs + ci * CHUNK_SITES;
            okbits = 0;
#pragma unroll
            for (int j = 0; j < Lt::J1; ++j) load_slot(j, q1p, bd.n1, x0);
#pragma unroll
            for (int j = 0; j < Lt::J2; ++j) load_slot(Lt::J1 + j, q2p, bd.n2, x0);
#pragma unroll
            for (int j = 0; j < Lt::J3; ++j) load_slot(Lt::J1 + Lt::J2 + j, q3p, bd.n3, x0);
            const int xa = x0 + ph_x;
            const unsigned ok = (unsigned)ph_ok & (unsigned)(xa < V);
            kval = kp[xa & -(int)ok];
            okbits |= ok << 31;
        };
        auto store_staging = [&]() {
#pragma unroll
            for (int q = 0; q < Lt::JL; ++q) {
                const float m = (float)((okbits >> q) & 1u);
                stg[(plan[q] >> 14) & 0xfffu] = make_float2(m * (float)rv[q].x, m * (float)rv[q].y);
            }
            const float m = (float)(okbits >> 31);
            const float2 r = roots[kval];
            stg[ph_dst] = make_float2(m * r.x, m * r.y);
        };

        f16_t acc[2][NB];
#pragma unroll
        for (int f = 0; f < 2; ++f)
#pragma unroll
            for (int n = 0; n < NB; ++n)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[f][n][e] = 0.f;

        // Prologue: D/W of chunk 0 in buffer 0, staging holds chunk 1,
        // registers hold chunk 2.
        issue_loads(0);
        store_staging();
        __syncthreads();
        gen_d<P, NB, B2, B3>(dwbuf, stg, lane, wave);
#pragma unroll
        for (int j = 0; j < Lt::JW; ++j) gen_w<P, NB, B2, B3>(dwbuf, stg, j, lane, wave);
        issue_loads(1);
        __syncthreads();
        store_staging();
        issue_loads(2);
        __syncthreads();

        if constexpr (P == BF16X3) {
            // Steady state, one wave per SIMD: each of the 126 MFMAs of a chunk
            // is followed (in program order, fenced by scheduling barriers) by
            // a slice of VALU/LDS work, so the matrix core and the VALU run
            // concurrently.  Section c multiplies colour c of chunk i; its
            // slices build the diquark tile (c = 0) and the W tile (c = 1) of
            // chunk i+1, or stage chunk i+2 and load chunk i+3 (c = 2), and
            // prefetch the A fragments of the next section.
            constexpr int SLOTS = 6 * NB;
            const int g = lane >> 5, r = lane & 31;
            const uint32_t sel = r >= 16 ? 0x01000302u : 0x03020100u;
            const uint32_t flip = r >= 16 ? 0u : 0x80000000u;
            const int aoff = drow(wave * 32 + (r & 15)) + 4 * g;
            const int boff = wrow(r) + 4 * g;
            const int i2 = lane % B2, xgd = (lane / B2) & 1, i1 = wave * (Lt::B1 / 4) + lane / (2 * B2);
            const int doff = drow(i1 * B2 + i2) + 4 * xgd;
            const int i3 = lane % B3, xgw = (lane / B3) & 1, ipl = lane / (2 * B3);
            const float2 *S1 = stg, *S2 = stg + Lt::E1, *S3 = S2 + Lt::E2, *PH = S3 + Lt::E3;

            bf8_t ah[2], al[2], ahn[2], aln[2];
            uint4 rah[2], ral[2];
            auto load_a = [&](const uint32_t *buf, int c) {
#pragma unroll
                for (int f = 0; f < 2; ++f) {
                    rah[f] = *reinterpret_cast<const uint4 *>(buf + aoff + 8 * c + f * drow(16));
                    ral[f] = *reinterpret_cast<const uint4 *>(buf + Lt::DPL + aoff + 8 * c + f * drow(16));
                }
            };
            // A prefetch for the next section: raw loads at mid-section, the
            // row embedding in the last four slots.
            auto a_prefetch = [&](auto kk, const uint32_t *buf, int c) {
                constexpr int k = kk;
                if constexpr (k == SLOTS / 2) load_a(buf, c);
                if constexpr (k == SLOTS - 4) ahn[0] = embed(rah[0], sel, flip);
                if constexpr (k == SLOTS - 3) aln[0] = embed(ral[0], sel, flip);
                if constexpr (k == SLOTS - 2) ahn[1] = embed(rah[1], sel, flip);
                if constexpr (k == SLOTS - 1) aln[1] = embed(ral[1], sel, flip);
            };
            // One colour of MFMAs: 6 per column fragment (lo*hi, hi*lo, hi*hi
            // for both row fragments).  B fragments are prefetched one ahead;
            // the first one of the next section (colour nc of buffer nbuf) is
            // loaded during this section's last column fragment.
            uint4 b0h, b0l;
            auto load_b0 = [&](const uint32_t *buf, int c) {
                b0h = *reinterpret_cast<const uint4 *>(buf + 2 * Lt::DPL + boff + 8 * c);
                b0l = *reinterpret_cast<const uint4 *>(buf + 2 * Lt::DPL + Lt::WPL + boff + 8 * c);
            };
            auto run_section = [&](const uint32_t *buf, auto cc, auto &&pre, auto &&work, const uint32_t *nbuf, int nc) {
                constexpr int c = cc;
                const uint32_t *W0 = buf + 2 * Lt::DPL, *W1 = W0 + Lt::WPL;
                uint4 bh[2], bl[2];
                bh[0] = b0h;
                bl[0] = b0l;
                pre();
                static_for<0, NB>([&](auto nn) {
                    constexpr int n = nn;
                    if constexpr (n + 1 < NB) {
                        bh[(n + 1) & 1] = *reinterpret_cast<const uint4 *>(W0 + boff + 8 * c + (n + 1) * wrow(32));
                        bl[(n + 1) & 1] = *reinterpret_cast<const uint4 *>(W1 + boff + 8 * c + (n + 1) * wrow(32));
                    } else {
                        load_b0(nbuf, nc);
                    }
                    static_for<0, 6>([&](auto kk) {
                        constexpr int k = kk, f = k & 1, prod = k >> 1;
                        const bf8_t A = prod == 0 ? al[f] : ah[f];
                        const bf8_t Bv = __builtin_bit_cast(bf8_t, prod == 1 ? bl[n & 1] : bh[n & 1]);
                        acc[f][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, Bv, acc[f][n], 0, 0, 0);
                        __builtin_amdgcn_sched_barrier(0);
                        work(std::integral_constant<int, n * 6 + k>{});
                        __builtin_amdgcn_sched_barrier(0);
                    });
                });
#pragma unroll
                for (int f = 0; f < 2; ++f) {
                    ah[f] = ahn[f];
                    al[f] = aln[f];
                }
            };
            // Generation slices start two MFMAs into a section, once the
            // staging reads issued at its start have landed.
            constexpr int GEN0 = 2;

            load_a(dwbuf, 0);
            load_b0(dwbuf, 0);
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                ah[f] = embed(rah[f], sel, flip);
                al[f] = embed(ral[f], sel, flip);
            }
            for (int i = 0; i < n_chunks; ++i) {
                const uint32_t *cur = dwbuf + (i & 1) * Lt::DW;
                uint32_t *nxt = dwbuf + ((i + 1) & 1) * Lt::DW;

                // Colour 0 + diquark tile of chunk i+1: 12 values (3 colours
                // x 4 sites), 4 sub-steps each.
                {
                    float2 u[3][4], v[3][4], t1[12];
                    uint32_t dh[3][4], dl[3][4];
                    auto pre = [&]() {
#pragma unroll
                        for (int x = 0; x < 4; ++x)
#pragma unroll
                            for (int q = 0; q < 3; ++q) {
                                u[q][x] = S1[(q * 8 + 4 * xgd + x) * Lt::B1 + i1];
                                v[q][x] = S2[(q * 8 + 4 * xgd + x) * B2 + i2];
                            }
                    };
                    auto step = [&](auto ss) {
                        constexpr int st = ss, t = st / 4, part = st % 4, x = t / 3, c = t % 3;
                        constexpr int a_ = (c + 1) % 3, b_ = (c + 2) % 3;  // eps_{a b c} = +1
                        if constexpr (part == 0) {
                            t1[t].x = diq_re(u[a_][x], u[b_][x], v[a_][x], v[b_][x]);
                        } else if constexpr (part == 1) {
                            t1[t].y = diq_im(u[a_][x], u[b_][x], v[a_][x], v[b_][x]);
                        } else if constexpr (part == 2) {
                            const float2 d = t1[t];
                            const uint32_t hi = pack_bf16(d.x, d.y);
                            dh[c][x] = hi;
                            t1[t] = make_float2(d.x - __uint_as_float(hi << 16), d.y - __uint_as_float(hi & 0xffff0000u));
                        } else {
                            dl[c][x] = pack_bf16(t1[t].x, t1[t].y);
                            if constexpr (x == 3) {
                                *reinterpret_cast<uint4 *>(nxt + doff + 8 * c) = make_uint4(dh[c][0], dh[c][1], dh[c][2], dh[c][3]);
                                *reinterpret_cast<uint4 *>(nxt + Lt::DPL + doff + 8 * c) =
                                    make_uint4(dl[c][0], dl[c][1], dl[c][2], dl[c][3]);
                            }
                        }
                    };
                    run_section(cur, std::integral_constant<int, 0>{}, pre, [&](auto kk) {
                        constexpr int k = kk;
                        if constexpr (k >= GEN0) slot_steps<k - GEN0, SLOTS - GEN0, 48>(step);
                        a_prefetch(kk, cur, 1);
                    }, cur, 1);
                }
                // Colour 1 + W tile of chunk i+1: JW rounds x 3 colours x 4
                // sites, 2 sub-steps each.
                {
                    float2 s3[3][4], ph[Lt::JW][4], wt[12 * Lt::JW];
                    uint32_t wh[Lt::JW][3][4], wl[Lt::JW][3][4];
                    int ip[Lt::JW];
#pragma unroll
                    for (int j = 0; j < Lt::JW; ++j) {
                        const bool live = (wave + 4 * j) < NB;
                        ip[j] = wave * Lt::IPW + ipl + (live ? 4 * Lt::IPW * j : 0);
                    }
                    auto pre = [&]() {
#pragma unroll
                        for (int x = 0; x < 4; ++x) {
#pragma unroll
                            for (int q = 0; q < 3; ++q) s3[q][x] = S3[(q * 8 + 4 * xgw + x) * B3 + i3];
#pragma unroll
                            for (int j = 0; j < Lt::JW; ++j) ph[j][x] = PH[ip[j] * 8 + 4 * xgw + x];
                        }
                    };
                    auto step = [&](auto ss) {
                        constexpr int st = ss, t = st / 2, part = st % 2, x = t % 4, c = (t / 4) % 3, j = t / 12;
                        if constexpr (part == 0) {
                            wt[t] = cmulf(s3[c][x], ph[j][x]);
                        } else {
                            const uint32_t hi = pack_bf16(wt[t].x, wt[t].y);
                            wh[j][c][x] = hi;
                            wl[j][c][x] = pack_bf16(wt[t].x - __uint_as_float(hi << 16), wt[t].y - __uint_as_float(hi & 0xffff0000u));
                            if constexpr (x == 3) {
                                const int off = wrow(ip[j] * B3 + i3) + 4 * xgw + 8 * c;
                                *reinterpret_cast<uint4 *>(nxt + 2 * Lt::DPL + off) =
                                    make_uint4(wh[j][c][0], wh[j][c][1], wh[j][c][2], wh[j][c][3]);
                                *reinterpret_cast<uint4 *>(nxt + 2 * Lt::DPL + Lt::WPL + off) =
                                    make_uint4(wl[j][c][0], wl[j][c][1], wl[j][c][2], wl[j][c][3]);
                            }
                        }
                    };
                    run_section(cur, std::integral_constant<int, 1>{}, pre, [&](auto kk) {
                        constexpr int k = kk;
                        if constexpr (k >= GEN0) slot_steps<k - GEN0, SLOTS - GEN0, 24 * Lt::JW>(step);
                        a_prefetch(kk, cur, 2);
                    }, cur, 2);
                }
                __syncthreads();
                // Colour 2 + staging of chunk i+2 and loads of chunk i+3.
                {
                    const int x0 = xs + (i + 3) * CHUNK_SITES;
                    auto step = [&](auto ss) {
                        constexpr int st = ss;
                        if constexpr (st < Lt::JL) {
                            const float m = (float)((okbits >> st) & 1u);
                            stg[(plan[st] >> 14) & 0xfffu] = make_float2(m * (float)rv[st].x, m * (float)rv[st].y);
                        } else if constexpr (st == Lt::JL) {
                            const float m = (float)(okbits >> 31);
                            const float2 rr = roots[kval];
                            stg[ph_dst] = make_float2(m * rr.x, m * rr.y);
                            okbits = 0;
                        } else if constexpr (st < 2 * Lt::JL + 1) {
                            constexpr int q = st - Lt::JL - 1;
                            if constexpr (q < Lt::J1)
                                load_slot(q, q1p, bd.n1, x0);
                            else if constexpr (q < Lt::J1 + Lt::J2)
                                load_slot(q, q2p, bd.n2, x0);
                            else
                                load_slot(q, q3p, bd.n3, x0);
                        } else {
                            const int xa = x0 + ph_x;
                            const unsigned ok = (unsigned)ph_ok & (unsigned)(xa < V);
                            kval = kp[xa & -(int)ok];
                            okbits |= ok << 31;
                        }
                    };
                    run_section(cur, std::integral_constant<int, 2>{}, [] {}, [&](auto kk) {
                        slot_steps<decltype(kk)::value, SLOTS, 2 * Lt::JL + 2>(step);
                        a_prefetch(kk, nxt, 0);
                    }, nxt, 0);
                }
                __syncthreads();
            }
        } else {
        // Steady state: each colour's MFMAs of chunk i are interleaved with one
        // piece of the generation of chunk i+1 (or the staging of chunk i+2);
        // the scheduling barriers bound the live registers of each piece.
        using Sc = Sched<P, NB, B2, B3>;
        for (int i = 0; i < n_chunks; ++i) {
            const uint32_t *cur = dwbuf + (i & 1) * Lt::DW;
            uint32_t *nxt = dwbuf + ((i + 1) & 1) * Lt::DW;
            gen_d<P, NB, B2, B3>(nxt, stg, lane, wave);
            multiply<P, NB, B2, B3>(cur, 0, acc, lane, wave);
            interleave<Sc::MF, Sc::NV_D, 1>();
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < Lt::JW; ++j) gen_w<P, NB, B2, B3>(nxt, stg, j, lane, wave);
            multiply<P, NB, B2, B3>(cur, 1, acc, lane, wave);
            interleave<Sc::MF, Sc::NV_W, 1>();
            __builtin_amdgcn_sched_barrier(0);
            __syncthreads();
            store_staging();
            issue_loads(i + 3);
            multiply<P, NB, B2, B3>(cur, 2, acc, lane, wave);
            interleave<Sc::MF, Sc::NV_S, 1>();
            __syncthreads();
        }
        }

        // Epilogue: real row -> (complex row, Re/Im), column -> (p, d3).
        with_put_mode(bd, tl.w, [&](auto mode) {
#pragma unroll
            for (int n = 0; n < NB; ++n) {
                const int nl = n * 32 + (lane & 31);
                const int ip = nl / B3, d3 = d3_0 + nl % B3, p = p0 + ip;
                if (ip >= bd.bp || p >= a.n_mom || d3 >= bd.n3) continue;
                const int nu = p * bd.n3 + d3;
#pragma unroll
                for (int f = 0; f < 2; ++f)
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        const int row = 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                        const int ml = wave * 32 + f * 16 + (row & 15);
                        const int s = row >> 4;
                        const int d1 = d1_0 + ml / B2, d2 = d2_0 + ml % B2;
                        if (d1 >= bd.n1 || d2 >= bd.n2) continue;
                        const int m = d1 * bd.n2 + d2;
                        put_result<decltype(mode)::value, float>(bd, tl.w, m, nu, p, d3, s, (double)acc[f][n][e]);
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
        __threadfence();
        if (atomicAdd(&a.counter[1], 1) == (int)gridDim.x - 1) {
            atomicExch(&a.counter[0], 0);
            atomicExch(&a.counter[1], 0);
        }
    }
}

// Instantiation table of one precision.
template <int P>
struct Launcher {
    template <int NB, int B2, int B3, bool C64>
    static hipError_t run(const GemmArgs &a, int grid, hipStream_t st)
    {
        const size_t lds = Layout<NB, B2, B3>::bytes(a.L);
        bb_fast<P, NB, B2, B3, C64><<<dim3(grid), dim3(THREADS), lds, st>>>(a);
        return hipGetLastError();
    }
    template <int NB, int B2, int B3, bool C64>
    static hipError_t raise(int bytes)
    {
        return hipFuncSetAttribute(reinterpret_cast<const void *>(&bb_fast<P, NB, B2, B3, C64>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    }
    static hipError_t launch(int nb, int b2, int b3, int c64, const GemmArgs &a, int grid, hipStream_t st)
    {
#define BBF_CASE(NB_, B2_, B3_)                                                                     \
    if (nb == NB_ && b2 == B2_ && b3 == B3_)                                                        \
        return c64 ? run<NB_, B2_, B3_, true>(a, grid, st) : run<NB_, B2_, B3_, false>(a, grid, st);
        BBF_CASE(7, 32, 32) BBF_CASE(7, 32, 16) BBF_CASE(7, 16, 32) BBF_CASE(7, 16, 16)
        BBF_CASE(4, 32, 32) BBF_CASE(4, 32, 16) BBF_CASE(4, 16, 32) BBF_CASE(4, 16, 16)
#undef BBF_CASE
        return hipErrorInvalidValue;
    }
    static hipError_t prepare(int bytes)
    {
        hipError_t e = hipSuccess;
#define BBF_RAISE(NB_, B2_, B3_)                                   \
    if (e == hipSuccess) e = raise<NB_, B2_, B3_, true>(bytes);    \
    if (e == hipSuccess) e = raise<NB_, B2_, B3_, false>(bytes);
        BBF_RAISE(7, 32, 32) BBF_RAISE(7, 32, 16) BBF_RAISE(7, 16, 32) BBF_RAISE(7, 16, 16)
        BBF_RAISE(4, 32, 32) BBF_RAISE(4, 32, 16) BBF_RAISE(4, 16, 32) BBF_RAISE(4, 16, 16)
#undef BBF_RAISE
        return e;
    }
};

inline int lds_bytes(int nb, int b2, int b3, int L)
{
#define BBF_SIZE(NB_, B2_, B3_) \
    if (nb == NB_ && b2 == B2_ && b3 == B3_) return (int)Layout<NB_, B2_, B3_>::bytes(L);
    BBF_SIZE(7, 32, 32) BBF_SIZE(7, 32, 16) BBF_SIZE(7, 16, 32) BBF_SIZE(7, 16, 16)
    BBF_SIZE(4, 32, 32) BBF_SIZE(4, 32, 16) BBF_SIZE(4, 16, 32) BBF_SIZE(4, 16, 16)
#undef BBF_SIZE
    return -1;
}

}  // namespace fast
}  // namespace bb
