// BF16X3 contraction with the phase-weighted third quark precomputed
// (gfx950).  Same contraction as the other kernels (paper, Sec. 2, eq. (3) as
// one complex GEMM over kappa = (colour, site)), split in two launches:
//
//   w_image : W[p][x][c][d3] = exp(-i p.x) q3[x][c][d3] of every (split,
//             n-tile, chunk), split into BF16 hi/lo planes and written to the
//             workspace in exactly the byte layout of the W tile in LDS.
//             Every m-tile of a split reads the same images, so the phase
//             multiplication and the split run once per column instead of
//             once per m-tile, and the contraction kernel copies W with
//             direct-to-LDS loads (no registers, no VALU).
//   contract: the diquark tile D = eps q1 q2 (Algorithm 1) is built in LDS
//             from staged q1/q2 (it never reaches HBM) while the MFMAs of the
//             previous chunk run; one barrier per chunk.
//
// Real embedding of the complex product: the W image holds conj(W), so the
// Re rows of a 32-row MFMA fragment take D as stored, (Re D, Im D), and the
// Im rows take (Im D, -Re D):
//   Re(D W) = Re D Re W + Im D (-Im W),   Im(D W) = Im D Re W + (-Re D)(-Im W).
// Fragment f = 0 holds the Re rows and f = 1 the Im rows of the same 32
// complex rows, so one LDS read feeds both.
#include "bb_fast.h"

namespace bb {
namespace w3 {

using fast::bf8_t;
using fast::cmulf;
using fast::f16_t;
using fast::MT;
using fast::pack_bf16;
using fast::drow;
using fast::wrow;
using fast::pin;
using fast::split_lo;
using fast::static_for;

// One W image: the hi and lo planes of an n-tile of NT columns over one chunk
// (24 kappa per column, wrow padding), padded to whole 4 KiB rounds of the
// direct-to-LDS copy (4 waves x 64 lanes x 16 bytes).
template <int NB>
struct WImg {
    static constexpr int NT = 32 * NB;
    static constexpr int WPL = wrow(NT);                 // u32 per plane
    static constexpr int DW = (2 * WPL + 1023) / 1024 * 1024; // u32 per image
    static constexpr int ROUNDS = DW / 1024;                 // copy instructions per wave
};

template <int NB, int B2>
struct CLayout {
    static constexpr int B1 = MT / B2;
    static constexpr int DPL = drow(MT);  // u32 per D plane
    static constexpr int E1 = 24 * B1, E2 = 24 * B2;
    static constexpr int SG = E1 + E2;       // float2 per staging buffer
    static constexpr int SINK = 64;          // slots written by lanes without an element
    static constexpr int J1 = (E1 + 255) / 256, J2 = (E2 + 255) / 256, JL = J1 + J2;
    static constexpr size_t lds_bytes()
    {
        return (size_t)2 * WImg<NB>::DW * 4 + (size_t)2 * 2 * DPL * 4 + (size_t)2 * (SG + SINK) * 8 + 16;
    }
};

// (Im, -Re) of four packed (Re, Im) BF16 pairs: the Im-row operand.
__device__ __forceinline__ bf8_t im_rows(uint4 v)
{
    return __builtin_bit_cast(bf8_t, make_uint4(__builtin_amdgcn_perm(v.x, v.x, 0x01000302u) ^ 0x80000000u,
                                                __builtin_amdgcn_perm(v.y, v.y, 0x01000302u) ^ 0x80000000u,
                                                __builtin_amdgcn_perm(v.z, v.z, 0x01000302u) ^ 0x80000000u,
                                                __builtin_amdgcn_perm(v.w, v.w, 0x01000302u) ^ 0x80000000u));
}

// Staged complex values move as one 8-byte LDS access (a float2 struct would
// be split into two 4-byte accesses, and the compiler's alias information for
// the second one is lost, which makes it wait for the W copy before it).
typedef float f2v_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 lds_get(const float2 *p)
{
    const f2v_t v = *reinterpret_cast<const f2v_t *>(p);
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ void lds_put(float2 *p, float x, float y) { *reinterpret_cast<f2v_t *>(p) = f2v_t{x, y}; }

typedef const void __attribute__((address_space(1))) *gvoid;
typedef void __attribute__((address_space(3))) *lvoid;

// ------------------------------------------------------------- W images ---
// One workgroup per (image entry, chunk).  blockIdx.y = entry (block, n-tile,
// split), blockIdx.x = chunk of that split.
template <int NB, bool C64>
__global__ void __launch_bounds__(THREADS) w_image(WImageArgs a)
{
    using Wi = WImg<NB>;
    using IT = typename fast::InT<C64>::T;
    constexpr int BPM_MAX = Wi::NT / 16;
    __shared__ float2 q3s[24 * 32];
    __shared__ float2 phs[BPM_MAX * 8];

    const int4 en = wave_uniform(a.entries[blockIdx.y]);
    const BlockDesc bd = wave_uniform(a.blocks[en.x]);
    const int ci = blockIdx.x;
    const int xs = en.z * bd.sps, xe = min(a.V, xs + bd.sps);
    if (ci * CHUNK_SITES >= xe - xs) return;  // whole workgroup: chunk past the split
    const int B3 = bd.b3, bpm = Wi::NT / B3;
    const int p0 = (en.y / bd.n_nt3) * bd.bp, d3_0 = (en.y % bd.n_nt3) * B3;
    const int x0 = xs + ci * CHUNK_SITES;
    const int tid = threadIdx.x, L = a.L;
    const IT *q3 = reinterpret_cast<const IT *>(bd.q3);

    for (int e = tid; e < 24 * B3; e += THREADS) {
        const int kap = e / B3, i3 = e - kap * B3, c = kap >> 3, xa = x0 + (kap & 7), d3 = d3_0 + i3;
        float2 v = make_float2(0.f, 0.f);
        if (xa < xe && d3 < bd.n3) {
            const IT w = q3[((size_t)xa * 3 + c) * bd.n3 + d3];
            v = make_float2((float)w.x, (float)w.y);
        }
        q3s[e] = v;
    }
    for (int e = tid; e < BPM_MAX * 8; e += THREADS) {  // columns past bp * B3 get zero phases
        const int ip = e >> 3, xa = x0 + (e & 7), p = p0 + ip;
        float2 v = make_float2(0.f, 0.f);
        if (ip < bd.bp && p < a.n_mom && xa < a.V) {
            const int ix = xa % L, iy = (xa / L) % L, iz = xa / (L * L);
            const int k = (a.mom[3 * p] * ix + a.mom[3 * p + 1] * iy + a.mom[3 * p + 2] * iz) % L;
            v = make_float2((float)a.roots[2 * k], (float)a.roots[2 * k + 1]);
        }
        phs[e] = v;
    }
    __syncthreads();

    uint32_t *img = reinterpret_cast<uint32_t *>(bd.wimg) +
                    (((size_t)(en.z - bd.img_s0) * bd.n_nt + en.y) * bd.cps + ci) * (size_t)Wi::DW;
    for (int it = tid; it < Wi::NT * 6; it += THREADS) {
        const int col = it / 6, r6 = it - col * 6, c = r6 >> 1, xg = r6 & 1;
        const int ip = col / B3, i3 = col - ip * B3;
        uint32_t hi[4], lo[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int x = 4 * xg + j;
            const float2 w = cmulf(q3s[(c * 8 + x) * B3 + i3], phs[ip * 8 + x]);
            const float wr = w.x, wi = -w.y;  // conj(W)
            hi[j] = pack_bf16(wr, wi);
            lo[j] = split_lo(wr, wi, hi[j]);
        }
        const int off = wrow(col) + 8 * c + 4 * xg;
        *reinterpret_cast<uint4 *>(img + off) = make_uint4(hi[0], hi[1], hi[2], hi[3]);
        *reinterpret_cast<uint4 *>(img + Wi::WPL + off) = make_uint4(lo[0], lo[1], lo[2], lo[3]);
    }
}

// ------------------------------------------------------------ contract ---
template <int NB, int B2, bool C64>
__global__ void __launch_bounds__(THREADS, 1) contract(GemmArgs a)
{
    using Lt = CLayout<NB, B2>;
    using Wi = WImg<NB>;
    using IT = typename fast::InT<C64>::T;
    constexpr int ESZ = sizeof(IT);
    constexpr int B1 = Lt::B1;
    constexpr int FR = 3 * NB;  // B fragments per chunk (colour, column fragment)
    // The two W buffers are separate objects: the direct-to-LDS copy into one
    // then never makes the compiler wait before reads of the other.
    __shared__ __align__(16) uint32_t w_a[Wi::DW];
    __shared__ __align__(16) uint32_t w_b[Wi::DW];
    __shared__ __align__(16) uint32_t dtile[2][2 * Lt::DPL];
    __shared__ __align__(16) float2 stg[2][Lt::SG + Lt::SINK];
    __shared__ int s_tile;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 5, r = lane & 31;
    const int V = a.V;

    auto next_tile = [&](int current) -> int {
        if (a.counter == nullptr) return current < 0 ? (int)blockIdx.x : a.n_tiles;
        __syncthreads();
        if (tid == 0) s_tile = atomicAdd(&a.counter[0], 1);
        __syncthreads();
        return __builtin_amdgcn_readfirstlane(s_tile);  // uniform: tile data go to scalar registers
    };

    // A walking tile runs every split of its block in order: the loop
    // stays on tile t and steps its split (wsp) up to the block's last.
    for (int t = next_tile(-1), wsp = 0; t < a.n_tiles;) {
        const int4 tl0 = wave_uniform(a.tiles[t]);
        const BlockDesc bd = wave_uniform(a.blocks[tl0.x]);
        const int4 tl = make_int4(tl0.x, tl0.y, tl0.z, tl0.w + wsp);
        const int d1_0 = (tl.y / bd.n_mt2) * B1, d2_0 = (tl.y % bd.n_mt2) * B2;
        const int p0 = (tl.z / bd.n_nt3) * bd.bp, d3_0 = (tl.z % bd.n_nt3) * bd.b3;
        const int xs = tl.w * bd.sps;
        const int xe = min(V, xs + bd.sps);
        const int n_chunks = (xe - xs + CHUNK_SITES - 1) / CHUNK_SITES;
        const uint32_t *img = reinterpret_cast<const uint32_t *>(bd.wimg) +
                              ((size_t)(tl.w - bd.img_s0) * bd.n_nt + tl.z) * bd.cps * (size_t)Wi::DW;

        // q1/q2 of this split through buffer resources: loads past the
        // split's sites (or of slots without an element) are out of range and
        // return zero, so no masks are needed.
        const __amdgpu_buffer_rsrc_t rs1 = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(reinterpret_cast<const IT *>(bd.q1) + (size_t)xs * 3 * bd.n1), (short)0,
            (xe - xs) * 3 * bd.n1 * ESZ, 0x00020000);
        const __amdgpu_buffer_rsrc_t rs2 = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(reinterpret_cast<const IT *>(bd.q2) + (size_t)xs * 3 * bd.n2), (short)0,
            (xe - xs) * 3 * bd.n2 * ESZ, 0x00020000);
        const uint32_t cstep1 = 24u * bd.n1 * ESZ, cstep2 = 24u * bd.n2 * ESZ;  // bytes per chunk

        // Staging slots: element e = tid + 256 j of array k is (colour c,
        // site x, index i) with e = i + B_k (x + 8c).
        uint32_t voff[Lt::JL];
        int sdst[Lt::JL];
        auto plan_slot = [&](int q, int j, int n_k, int d0_k, int B_k, int E_k, int sofs_k) {
            const int e = tid + 256 * j;
            const int i = e % B_k, x = (e / B_k) % 8, c = e / (8 * B_k);
            const bool live = e < E_k;
            const bool ok = live && (d0_k + i < n_k);
            voff[q] = ok ? (uint32_t)(((x * 3 + c) * n_k + d0_k + i) * ESZ) : 0x80000000u;
            sdst[q] = live ? sofs_k + e : Lt::SG + lane;
        };
#pragma unroll
        for (int j = 0; j < Lt::J1; ++j) plan_slot(j, j, bd.n1, d1_0, B1, Lt::E1, 0);
#pragma unroll
        for (int j = 0; j < Lt::J2; ++j) plan_slot(Lt::J1 + j, j, bd.n2, d2_0, B2, Lt::E2, Lt::E1);

        IT rv[Lt::JL];
        auto qload = [&](int q, int ci) {
            const bool first = q < Lt::J1;
            const uint32_t off = voff[q] + (uint32_t)ci * (first ? cstep1 : cstep2);
            if constexpr (C64)
                rv[q] = __builtin_bit_cast(IT, __builtin_amdgcn_raw_buffer_load_b64(first ? rs1 : rs2, off, 0, 0));
            else
                rv[q] = __builtin_bit_cast(IT, __builtin_amdgcn_raw_buffer_load_b128(first ? rs1 : rs2, off, 0, 0));
        };
        auto qstore = [&](int q, float2 *s) { lds_put(s + sdst[q], (float)rv[q].x, (float)rv[q].y); };
        // Direct-to-LDS copy of round k of image ci into W buffer wbuf.
        // The image of chunk ci is addressed through a buffer resource built
        // from scalar values (the image base, uniform per chunk), the wave's
        // slice by a scalar offset and the lane by one fixed vector offset,
        // so a copy costs no vector instructions.
        const int swave = __builtin_amdgcn_readfirstlane(wave);
        const uint32_t lane_off = (uint32_t)lane * 16u;
        auto wcopy = [&](uint32_t *wbuf, int k, int ci) {
            const int ro = (k * 4 + swave) * 256;  // u32 offset of this wave's 1 KiB slice of round k
            const __amdgpu_buffer_rsrc_t rsi = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(img + (size_t)ci * Wi::DW), (short)0, Wi::DW * 4, 0x00020000);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rsi, (lvoid)(wbuf + ro), 16, lane_off, (uint32_t)ro * 4u, 0, 0);
        };

        // Diquark generation: lane -> (i1, i2, site group of 4).
        const int i2 = lane % B2, xgd = (lane / B2) & 1, i1 = wave * (B1 / 4) + lane / (2 * B2);
        const int doff = drow(i1 * B2 + i2) + 4 * xgd;
        const int aoff = drow(wave * 32 + r) + 4 * g;
        const int boff = wrow(r) + 4 * g;

        f16_t acc[2][NB];
#pragma unroll
        for (int f = 0; f < 2; ++f)
#pragma unroll
            for (int n = 0; n < NB; ++n)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[f][n][e] = 0.f;

        // Operand registers: A of the current colour (hi/lo x Re/Im rows), A
        // of the next colour, B fragments double-buffered across the chunk.
        bf8_t A[4], An[4];
        uint4 ra[2];
        uint4 bh[2], bl[2];
        auto load_a = [&](const uint32_t *dbuf, int c) {
            ra[0] = *reinterpret_cast<const uint4 *>(dbuf + aoff + 8 * c);
            ra[1] = *reinterpret_cast<const uint4 *>(dbuf + Lt::DPL + aoff + 8 * c);
        };
        auto load_b = [&](const uint32_t *wbuf, int c, int n, int slot) {
            bh[slot] = *reinterpret_cast<const uint4 *>(wbuf + boff + 8 * c + n * wrow(32));
            bl[slot] = *reinterpret_cast<const uint4 *>(wbuf + Wi::WPL + boff + 8 * c + n * wrow(32));
        };
        // An[0..3] = (hi Re rows, lo Re rows, hi Im rows, lo Im rows)
        auto embed_step = [&](int s) {
            if (s == 0) An[0] = __builtin_bit_cast(bf8_t, ra[0]);
            if (s == 1) An[1] = __builtin_bit_cast(bf8_t, ra[1]);
            if (s == 2) An[2] = im_rows(ra[0]);
            if (s == 3) An[3] = im_rows(ra[1]);
        };

        // Diquark generation of one chunk in 52 sub-steps: for each of the 4
        // sites, one read step (6 staged values) and 12 arithmetic steps (3
        // colours x 4); site x+1 is read one site ahead.
        float2 u[2][3], v[2][3], t1[3];
        uint32_t dh[3][4], dl[3][4];
        auto dgen = [&](auto ss, const float2 *sd, uint32_t *dn) {
            constexpr int st = ss;
            const float2 *S1 = sd, *S2 = sd + Lt::E1;
            auto read_site = [&](int x) {
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    u[x & 1][q] = lds_get(S1 + (q * 8 + 4 * xgd + x) * B1 + i1);
                    v[x & 1][q] = lds_get(S2 + (q * 8 + 4 * xgd + x) * B2 + i2);
                }
            };
            // Step layout: 0: read site 0; 1: read site 1; then per site x:
            // 12 arithmetic steps, followed (x < 2) by the read of site x+2.
            if constexpr (st == 0) {
                read_site(0);
            } else if constexpr (st == 1) {
                read_site(1);
            } else {
                constexpr int s2 = st - 2, x = s2 / 13, w = s2 % 13;
                if constexpr (w == 12) {
                    if constexpr (x + 2 < 4) read_site(x + 2);
                } else {
                    constexpr int c = w / 4, part = w % 4;
                    constexpr int a_ = (c + 1) % 3, b_ = (c + 2) % 3;  // eps_{a b c} = +1
                    const float2 *uu = u[x & 1], *vv = v[x & 1];
                    if constexpr (part == 0) {
                        t1[c].x = fast::diq_re(uu[a_], uu[b_], vv[a_], vv[b_]);
                        pin(t1[c].x);
                    } else if constexpr (part == 1) {
                        t1[c].y = fast::diq_im(uu[a_], uu[b_], vv[a_], vv[b_]);
                        pin(t1[c].y);
                    } else if constexpr (part == 2) {
                        dh[c][x] = pack_bf16(t1[c].x, t1[c].y);
                        pin(dh[c][x]);
                    } else {
                        dl[c][x] = split_lo(t1[c].x, t1[c].y, dh[c][x]);
                        if constexpr (x == 3) {
                            *reinterpret_cast<uint4 *>(dn + doff + 8 * c) = make_uint4(dh[c][0], dh[c][1], dh[c][2], dh[c][3]);
                            *reinterpret_cast<uint4 *>(dn + Lt::DPL + doff + 8 * c) =
                                make_uint4(dl[c][0], dl[c][1], dl[c][2], dl[c][3]);
                        }
                    }
                }
            }
        };
        constexpr int NDGEN = 2 + 4 * 13;

        // ---- prologue: chunk 0 staged, D(0) and W(0) built, chunk 1 staged,
        // chunk 2 in registers.
#pragma unroll
        for (int q = 0; q < Lt::JL; ++q) qload(q, 0);
#pragma unroll
        for (int k = 0; k < Wi::ROUNDS; ++k) wcopy(w_a, k, 0);
        __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0)
#pragma unroll
        for (int q = 0; q < Lt::JL; ++q) qstore(q, stg[0]);
#pragma unroll
        for (int q = 0; q < Lt::JL; ++q) qload(q, 1);
        __syncthreads();
        static_for<0, NDGEN>([&](auto ss) { dgen(ss, stg[0], dtile[0]); });
        __builtin_amdgcn_s_waitcnt(0x0f70);
#pragma unroll
        for (int q = 0; q < Lt::JL; ++q) qstore(q, stg[1]);
#pragma unroll
        for (int q = 0; q < Lt::JL; ++q) qload(q, 2);
        __syncthreads();
        load_a(dtile[0], 0);
        load_b(w_a, 0, 0, 0);
#pragma unroll
        for (int s = 0; s < 4; ++s) embed_step(s);
#pragma unroll
        for (int s = 0; s < 4; ++s) A[s] = An[s];

        // ---- steady state.  Chunk i (buffer parity P = i & 1): the MFMAs
        // read D/W buffer P; the slices stage chunk i+2, copy W(i+1), load
        // chunk i+3 and build D(i+1) into buffer P^1.  The barrier sits
        // before the last column fragment so that the A/B reads of chunk i+1
        // overlap its MFMAs.
        constexpr int NSLOT = 6 * FR - 6;                      // slots before the barrier
        constexpr int NQ = Lt::JL, NW = Wi::ROUNDS;
        // Work items in order: staging stores (their registers were loaded a
        // chunk ago), the W copies, the staging loads, the diquark steps.
        // The staging stores precede the copies because any wait for the
        // stores' registers while a copy is in flight would wait for the copy.
        constexpr int W_STAGE = 0, W_COPY = NQ, W_LOAD = NQ + NW, W_DGEN = 2 * NQ + NW;
        constexpr int NFIRST = NQ + NW;  // items issued one per slot from the start of the chunk
        constexpr int NWORK = W_DGEN + NDGEN;
        auto chunk = [&](auto par, int i) {
            constexpr int P = decltype(par)::value;
            uint32_t *Wc = P ? w_b : w_a;
            uint32_t *Wn = P ? w_a : w_b;
            const uint32_t *Dc = dtile[P];
            uint32_t *Dn = dtile[P ^ 1];
            const float2 *Sd = stg[P ^ 1];
            float2 *Ss = stg[P];
            const int cnext = min(i + 1, n_chunks - 1);
            auto work = [&](auto ww) {
                constexpr int w = ww;
                if constexpr (w < W_COPY)
                    qstore(w - W_STAGE, Ss);
                else if constexpr (w < W_LOAD)
                    wcopy(Wn, w - W_COPY, cnext);
                else if constexpr (w < W_DGEN)
                    qload(w - W_LOAD, i + 3);
                else
                    dgen(std::integral_constant<int, w - W_DGEN>{}, Sd, Dn);
            };
            static_for<0, 3>([&](auto cc) {
                constexpr int c = cc;
                static_for<0, NB>([&](auto nn) {
                    constexpr int n = nn;
                    constexpr int fr = c * NB + n;                 // fragment index in the chunk
                    constexpr int slot_b = (P * FR + fr) & 1;      // B register set of this fragment
                    if constexpr (fr == FR - 1) {
                        // Publish D/W(i+1).  The barrier waits for all of
                        // this wave's loads (the copies write LDS), so the
                        // staging loads are issued first in the chunk.
                        __builtin_amdgcn_sched_barrier(0);
                        __syncthreads();
                        __builtin_amdgcn_sched_barrier(0);
                    }
                    // Prefetch of the next B fragment (next colour's first,
                    // or chunk i+1's first after the barrier).
                    if constexpr (fr + 1 < FR)
                        load_b(Wc, (fr + 1) / NB, (fr + 1) % NB, slot_b ^ 1);
                    static_for<0, 6>([&](auto kk) {
                        constexpr int k = kk, f = k & 1, prod = k >> 1;
                        // prod 0: lo x hi, 1: hi x lo, 2: hi x hi
                        const bf8_t Av = A[2 * f + (prod == 0 ? 1 : 0)];
                        const bf8_t Bv = __builtin_bit_cast(bf8_t, prod == 1 ? bl[slot_b] : bh[slot_b]);
                        acc[f][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Av, Bv, acc[f][n], 0, 0, 0);
                        __builtin_amdgcn_sched_barrier(0);
                        constexpr int s = fr * 6 + k;  // slot
                        if constexpr (fr < FR - 1) {
                            // Stores and copies one per slot from the start
                            // (the copies' latency is the longest), the rest
                            // of the work spread evenly over the other slots.
                            if constexpr (s < NFIRST) {
                                work(std::integral_constant<int, s>{});
                            } else {
                                constexpr int s2 = s - NFIRST, NS2 = NSLOT - NFIRST, NW2 = NWORK - NFIRST;
                                static_for<NFIRST + (s2 * NW2 + NS2 - 1) / NS2, NFIRST + ((s2 + 1) * NW2 + NS2 - 1) / NS2>(work);
                            }
                            // A of the next colour: read at mid-colour, turned
                            // into the four operands in the colour's last slots.
                            constexpr int cs = s - c * 6 * NB;  // slot within the colour
                            if constexpr (c < 2) {
                                if constexpr (cs == 3 * NB) load_a(Dc, c + 1);
                                if constexpr (cs >= 6 * NB - 4) embed_step(cs - (6 * NB - 4));
                            }
                        } else {
                            // After the barrier: chunk i+1's first operands.
                            if constexpr (k == 0) {
                                load_a(Dn, 0);
                                load_b(Wn, 0, 0, slot_b ^ 1);
                            }
                            if constexpr (k >= 2) embed_step(k - 2);
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    });
                    if constexpr (n == NB - 1) {
#pragma unroll
                        for (int s = 0; s < 4; ++s) A[s] = An[s];
                    }
                });
            });
        };
        int i = 0;
        for (; i + 2 <= n_chunks; i += 2) {
            chunk(std::integral_constant<int, 0>{}, i);
            chunk(std::integral_constant<int, 1>{}, i + 1);
        }
        if (i < n_chunks) chunk(std::integral_constant<int, 0>{}, i);

        // Epilogue: fragment f = Re (0) / Im (1) part of complex row
        // 32 wave + row; column -> (p, d3).
        with_put_mode(bd, tl.w, [&](auto mode) {
            const int B3 = bd.b3;
#pragma unroll
            for (int n = 0; n < NB; ++n) {
                const int nl = n * 32 + r;
                const int ip = nl / B3, d3 = d3_0 + nl % B3, p = p0 + ip;
                if (ip >= bd.bp || p >= a.n_mom || d3 >= bd.n3) continue;
                const int nu = p * bd.n3 + d3;
#pragma unroll
                for (int f = 0; f < 2; ++f)
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        const int row = 8 * (e >> 2) + 4 * g + (e & 3);
                        const int ml = wave * 32 + row;
                        const int d1 = d1_0 + ml / B2, d2 = d2_0 + ml % B2;
                        if (d1 >= bd.n1 || d2 >= bd.n2) continue;
                        const int m = d1 * bd.n2 + d2;
                        put_result<decltype(mode)::value, float>(bd, tl.w, m, nu, p, d3, f, (double)acc[f][n][e]);
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

// ----------------------------------------------------- contract, 8 waves ---
// The same contraction with eight waves per workgroup, two per SIMD: waves w
// and w + 4 share the 32 complex rows of row group w and split its column
// fragments (waves 0-3 take the first ceil(NB / 2)), so that one wave's
// vector work and waits run while the other's MFMAs issue.  The D/W tiles,
// the staging and the W copies are shared by all eight waves; each lane
// builds the diquark of two sites instead of four.  Every accumulator sees
// the same MFMAs in the same order as in the four-wave kernel, so the two
// kernels give bitwise identical results.
constexpr int THREADS8 = 512;

template <int NB, int B2, bool C64>
__global__ void __launch_bounds__(THREADS8, 1) contract8(GemmArgs a)
{
    using Lt = CLayout<NB, B2>;
    using Wi = WImg<NB>;
    using IT = typename fast::InT<C64>::T;
    constexpr int ESZ = sizeof(IT);
    constexpr int B1 = Lt::B1;
    constexpr int NBA = (NB + 1) / 2;  // column fragments of waves 0-3 (waves 4-7: NB - NBA)
    constexpr int J1 = (Lt::E1 + THREADS8 - 1) / THREADS8, J2 = (Lt::E2 + THREADS8 - 1) / THREADS8;
    constexpr int JL = J1 + J2;
    constexpr int NW = (Wi::DW + 2047) / 2048;  // W copy rounds of 8 KiB (eight waves x 1 KiB)
    __shared__ __align__(16) uint32_t w_a[Wi::DW];
    __shared__ __align__(16) uint32_t w_b[Wi::DW];
    __shared__ __align__(16) uint32_t dtile[2][2 * Lt::DPL];
    __shared__ __align__(16) float2 stg[2][Lt::SG + Lt::SINK];
    __shared__ int s_tile;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int swave = __builtin_amdgcn_readfirstlane(wave);
    const int g = lane >> 5, r = lane & 31;
    const int V = a.V;

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
        const int d1_0 = (tl.y / bd.n_mt2) * B1, d2_0 = (tl.y % bd.n_mt2) * B2;
        const int p0 = (tl.z / bd.n_nt3) * bd.bp, d3_0 = (tl.z % bd.n_nt3) * bd.b3;
        const int xs = tl.w * bd.sps;
        const int xe = min(V, xs + bd.sps);
        const int n_chunks = (xe - xs + CHUNK_SITES - 1) / CHUNK_SITES;
        const uint32_t *img = reinterpret_cast<const uint32_t *>(bd.wimg) +
                              ((size_t)(tl.w - bd.img_s0) * bd.n_nt + tl.z) * bd.cps * (size_t)Wi::DW;

        const __amdgpu_buffer_rsrc_t rs1 = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(reinterpret_cast<const IT *>(bd.q1) + (size_t)xs * 3 * bd.n1), (short)0,
            (xe - xs) * 3 * bd.n1 * ESZ, 0x00020000);
        const __amdgpu_buffer_rsrc_t rs2 = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(reinterpret_cast<const IT *>(bd.q2) + (size_t)xs * 3 * bd.n2), (short)0,
            (xe - xs) * 3 * bd.n2 * ESZ, 0x00020000);
        const uint32_t cstep1 = 24u * bd.n1 * ESZ, cstep2 = 24u * bd.n2 * ESZ;

        // Staging slots: element e = tid + 512 j of array k is (colour c,
        // site x, index i) with e = i + B_k (x + 8c).
        uint32_t voff[JL];
        int sdst[JL];
        auto plan_slot = [&](int q, int j, int n_k, int d0_k, int B_k, int E_k, int sofs_k) {
            const int e = tid + THREADS8 * j;
            const int i = e % B_k, x = (e / B_k) % 8, c = e / (8 * B_k);
            const bool live = e < E_k;
            const bool ok = live && (d0_k + i < n_k);
            voff[q] = ok ? (uint32_t)(((x * 3 + c) * n_k + d0_k + i) * ESZ) : 0x80000000u;
            sdst[q] = live ? sofs_k + e : Lt::SG + lane;
        };
#pragma unroll
        for (int j = 0; j < J1; ++j) plan_slot(j, j, bd.n1, d1_0, B1, Lt::E1, 0);
#pragma unroll
        for (int j = 0; j < J2; ++j) plan_slot(J1 + j, j, bd.n2, d2_0, B2, Lt::E2, Lt::E1);

        IT rv[JL];
        auto qload = [&](int q, int ci) {
            const bool first = q < J1;
            const uint32_t off = voff[q] + (uint32_t)ci * (first ? cstep1 : cstep2);
            if constexpr (C64)
                rv[q] = __builtin_bit_cast(IT, __builtin_amdgcn_raw_buffer_load_b64(first ? rs1 : rs2, off, 0, 0));
            else
                rv[q] = __builtin_bit_cast(IT, __builtin_amdgcn_raw_buffer_load_b128(first ? rs1 : rs2, off, 0, 0));
        };
        auto qstore = [&](int q, float2 *s) { lds_put(s + sdst[q], (float)rv[q].x, (float)rv[q].y); };
        // Direct-to-LDS copy of round k of image ci: wave w copies the 1 KiB
        // slice 8k + w; slices past the image (the second half of the last
        // round when the image holds an odd number of KiB) are skipped.
        const uint32_t lane_off = (uint32_t)lane * 16u;
        auto wcopy = [&](uint32_t *wbuf, int k, int ci) {
            const int ro = (k * 8 + swave) * 256;
            if (ro < Wi::DW) {
                const __amdgpu_buffer_rsrc_t rsi = __builtin_amdgcn_make_buffer_rsrc(
                    (void *)(img + (size_t)ci * Wi::DW), (short)0, Wi::DW * 4, 0x00020000);
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rsi, (lvoid)(wbuf + ro), 16, lane_off, (uint32_t)ro * 4u, 0, 0);
            }
        };

        // Diquark generation: thread -> (i1, i2, site pair xq).
        const int i2 = tid % B2, xq = (tid / B2) & 3, i1 = tid / (4 * B2);
        const int doff = drow(i1 * B2 + i2) + 2 * xq;
        const int wr = swave & 3;
        const int aoff = drow(wr * 32 + r) + 4 * g;
        const int boff = wrow(r) + 4 * g;

        auto body = [&](auto nbw_, auto n0_) {
            constexpr int NBW = decltype(nbw_)::value, N0 = decltype(n0_)::value;
            constexpr int FR = 3 * NBW;  // B fragments of this wave per chunk

            f16_t acc[2][NBW];
#pragma unroll
            for (int f = 0; f < 2; ++f)
#pragma unroll
                for (int n = 0; n < NBW; ++n)
#pragma unroll
                    for (int e = 0; e < 16; ++e) acc[f][n][e] = 0.f;

            bf8_t A[4], An[4];
            uint4 ra[2];
            uint4 bh[2], bl[2];
            auto load_a = [&](const uint32_t *dbuf, int c) {
                ra[0] = *reinterpret_cast<const uint4 *>(dbuf + aoff + 8 * c);
                ra[1] = *reinterpret_cast<const uint4 *>(dbuf + Lt::DPL + aoff + 8 * c);
            };
            auto load_b = [&](const uint32_t *wbuf, int c, int n, int slot) {
                bh[slot] = *reinterpret_cast<const uint4 *>(wbuf + boff + 8 * c + (N0 + n) * wrow(32));
                bl[slot] = *reinterpret_cast<const uint4 *>(wbuf + Wi::WPL + boff + 8 * c + (N0 + n) * wrow(32));
            };
            auto embed_step = [&](int s) {
                if (s == 0) An[0] = __builtin_bit_cast(bf8_t, ra[0]);
                if (s == 1) An[1] = __builtin_bit_cast(bf8_t, ra[1]);
                if (s == 2) An[2] = im_rows(ra[0]);
                if (s == 3) An[3] = im_rows(ra[1]);
            };

            // Diquark generation of one chunk in 26 sub-steps: the reads of
            // the two sites, then per site 12 arithmetic steps (3 colours x 4).
            float2 u[2][3], v[2][3], t1[3];
            uint32_t dh[3][2], dl[3][2];
            auto dgen = [&](auto ss, const float2 *sd, uint32_t *dn) {
                constexpr int st = ss;
                const float2 *S1 = sd, *S2 = sd + Lt::E1;
                if constexpr (st < 2) {
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        u[st][q] = lds_get(S1 + (q * 8 + 2 * xq + st) * B1 + i1);
                        v[st][q] = lds_get(S2 + (q * 8 + 2 * xq + st) * B2 + i2);
                    }
                } else {
                    constexpr int s2 = st - 2, x = s2 / 12, w = s2 % 12;
                    constexpr int c = w / 4, part = w % 4;
                    constexpr int a_ = (c + 1) % 3, b_ = (c + 2) % 3;  // eps_{a b c} = +1
                    const float2 *uu = u[x], *vv = v[x];
                    if constexpr (part == 0) {
                        t1[c].x = fast::diq_re(uu[a_], uu[b_], vv[a_], vv[b_]);
                        pin(t1[c].x);
                    } else if constexpr (part == 1) {
                        t1[c].y = fast::diq_im(uu[a_], uu[b_], vv[a_], vv[b_]);
                        pin(t1[c].y);
                    } else if constexpr (part == 2) {
                        dh[c][x] = pack_bf16(t1[c].x, t1[c].y);
                        pin(dh[c][x]);
                    } else {
                        dl[c][x] = split_lo(t1[c].x, t1[c].y, dh[c][x]);
                        if constexpr (x == 1) {
                            *reinterpret_cast<uint2 *>(dn + doff + 8 * c) = make_uint2(dh[c][0], dh[c][1]);
                            *reinterpret_cast<uint2 *>(dn + Lt::DPL + doff + 8 * c) = make_uint2(dl[c][0], dl[c][1]);
                        }
                    }
                }
            };
            constexpr int NDGEN = 2 + 2 * 12;

            // ---- prologue (as in the four-wave kernel)
#pragma unroll
            for (int q = 0; q < JL; ++q) qload(q, 0);
#pragma unroll
            for (int k = 0; k < NW; ++k) wcopy(w_a, k, 0);
            __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0)
#pragma unroll
            for (int q = 0; q < JL; ++q) qstore(q, stg[0]);
#pragma unroll
            for (int q = 0; q < JL; ++q) qload(q, 1);
            __syncthreads();
            static_for<0, NDGEN>([&](auto ss) { dgen(ss, stg[0], dtile[0]); });
            __builtin_amdgcn_s_waitcnt(0x0f70);
#pragma unroll
            for (int q = 0; q < JL; ++q) qstore(q, stg[1]);
#pragma unroll
            for (int q = 0; q < JL; ++q) qload(q, 2);
            __syncthreads();
            load_a(dtile[0], 0);
            load_b(w_a, 0, 0, 0);
#pragma unroll
            for (int s = 0; s < 4; ++s) embed_step(s);
#pragma unroll
            for (int s = 0; s < 4; ++s) A[s] = An[s];

            // ---- steady state: the schedule of the four-wave kernel over
            // this wave's 6 FR MFMA slots.
            constexpr int NSLOT = 6 * FR - 6;
            constexpr int NQ = JL;
            constexpr int W_STAGE = 0, W_COPY = NQ, W_LOAD = NQ + NW, W_DGEN = 2 * NQ + NW;
            constexpr int NFIRST = NQ + NW;
            constexpr int NWORK = W_DGEN + NDGEN;
            static_assert(NFIRST < NSLOT, "too few MFMA slots for the per-chunk work");
            auto chunk = [&](auto par, int i) {
                constexpr int P = decltype(par)::value;
                uint32_t *Wc = P ? w_b : w_a;
                uint32_t *Wn = P ? w_a : w_b;
                const uint32_t *Dc = dtile[P];
                uint32_t *Dn = dtile[P ^ 1];
                const float2 *Sd = stg[P ^ 1];
                float2 *Ss = stg[P];
                const int cnext = min(i + 1, n_chunks - 1);
                auto work = [&](auto ww) {
                    constexpr int w = ww;
                    if constexpr (w < W_COPY)
                        qstore(w - W_STAGE, Ss);
                    else if constexpr (w < W_LOAD)
                        wcopy(Wn, w - W_COPY, cnext);
                    else if constexpr (w < W_DGEN)
                        qload(w - W_LOAD, i + 3);
                    else
                        dgen(std::integral_constant<int, w - W_DGEN>{}, Sd, Dn);
                };
                static_for<0, 3>([&](auto cc) {
                    constexpr int c = cc;
                    static_for<0, NBW>([&](auto nn) {
                        constexpr int n = nn;
                        constexpr int fr = c * NBW + n;
                        constexpr int slot_b = (P * FR + fr) & 1;
                        if constexpr (fr == FR - 1) {
                            __builtin_amdgcn_sched_barrier(0);
                            __syncthreads();
                            __builtin_amdgcn_sched_barrier(0);
                        }
                        if constexpr (fr + 1 < FR)
                            load_b(Wc, (fr + 1) / NBW, (fr + 1) % NBW, slot_b ^ 1);
                        static_for<0, 6>([&](auto kk) {
                            constexpr int k = kk, f = k & 1, prod = k >> 1;
                            const bf8_t Av = A[2 * f + (prod == 0 ? 1 : 0)];
                            const bf8_t Bv = __builtin_bit_cast(bf8_t, prod == 1 ? bl[slot_b] : bh[slot_b]);
                            acc[f][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Av, Bv, acc[f][n], 0, 0, 0);
                            __builtin_amdgcn_sched_barrier(0);
                            constexpr int s = fr * 6 + k;
                            if constexpr (fr < FR - 1) {
                                if constexpr (s < NFIRST) {
                                    work(std::integral_constant<int, s>{});
                                } else {
                                    constexpr int s2 = s - NFIRST, NS2 = NSLOT - NFIRST, NW2 = NWORK - NFIRST;
                                    static_for<NFIRST + (s2 * NW2 + NS2 - 1) / NS2, NFIRST + ((s2 + 1) * NW2 + NS2 - 1) / NS2>(work);
                                }
                                constexpr int cs = s - c * 6 * NBW;
                                if constexpr (c < 2) {
                                    if constexpr (cs == 3 * NBW) load_a(Dc, c + 1);
                                    if constexpr (cs >= 6 * NBW - 4) embed_step(cs - (6 * NBW - 4));
                                }
                            } else {
                                if constexpr (k == 0) {
                                    load_a(Dn, 0);
                                    load_b(Wn, 0, 0, slot_b ^ 1);
                                }
                                if constexpr (k >= 2) embed_step(k - 2);
                            }
                            __builtin_amdgcn_sched_barrier(0);
                        });
                        if constexpr (n == NBW - 1) {
#pragma unroll
                            for (int s = 0; s < 4; ++s) A[s] = An[s];
                        }
                    });
                });
            };
            int i = 0;
            for (; i + 2 <= n_chunks; i += 2) {
                chunk(std::integral_constant<int, 0>{}, i);
                chunk(std::integral_constant<int, 1>{}, i + 1);
            }
            if (i < n_chunks) chunk(std::integral_constant<int, 0>{}, i);

            // Epilogue: fragment f = Re (0) / Im (1) part of complex row
            // 32 wr + row; column -> (p, d3).
            with_put_mode(bd, tl.w, [&](auto mode) {
                const int B3 = bd.b3;
#pragma unroll
                for (int n = 0; n < NBW; ++n) {
                    const int nl = (N0 + n) * 32 + r;
                    const int ip = nl / B3, d3 = d3_0 + nl % B3, p = p0 + ip;
                    if (ip >= bd.bp || p >= a.n_mom || d3 >= bd.n3) continue;
                    const int nu = p * bd.n3 + d3;
#pragma unroll
                    for (int f = 0; f < 2; ++f)
#pragma unroll
                        for (int e = 0; e < 16; ++e) {
                            const int row = 8 * (e >> 2) + 4 * g + (e & 3);
                            const int ml = wr * 32 + row;
                            const int d1 = d1_0 + ml / B2, d2 = d2_0 + ml % B2;
                            if (d1 >= bd.n1 || d2 >= bd.n2) continue;
                            const int m = d1 * bd.n2 + d2;
                            put_result<decltype(mode)::value, float>(bd, tl.w, m, nu, p, d3, f, (double)acc[f][n][e]);
                        }
                }
            });
        };
        if (swave < 4)
            body(std::integral_constant<int, NBA>{}, std::integral_constant<int, 0>{});
        else
            body(std::integral_constant<int, NB - NBA>{}, std::integral_constant<int, NBA>{});
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

template <int NB, int B2, bool C64>
hipError_t run_contract8(const GemmArgs &a, int grid, hipStream_t st)
{
    contract8<NB, B2, C64><<<dim3(grid), dim3(THREADS8), 0, st>>>(a);
    return hipGetLastError();
}

template <int NB, int B2, bool C64>
hipError_t run_contract(const GemmArgs &a, int grid, hipStream_t st)
{
    contract<NB, B2, C64><<<dim3(grid), dim3(THREADS), 0, st>>>(a);
    return hipGetLastError();
}

template <int NB, bool C64>
hipError_t run_image(const WImageArgs &a, int cps_max, hipStream_t st)
{
    w_image<NB, C64><<<dim3(cps_max, a.n_entries), dim3(THREADS), 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace w3

// Instantiations: NB = 4..7 column fragments (128..224 columns), B2 = 8, 16
// or 32 d2 values per m-tile (d1 blocks of 16, 8 or 4).
#define BBW_FOR_EACH(X) \
    X(7, 32) X(7, 16) X(7, 8) X(6, 32) X(6, 16) X(6, 8) X(5, 32) X(5, 16) X(5, 8) X(4, 32) X(4, 16) X(4, 8)

int w3_lds_bytes(int nb, int b2)
{
#define BBW_LDS(NB_, B2_) \
    if (nb == NB_ && b2 == B2_) return (int)w3::CLayout<NB_, B2_>::lds_bytes();
    BBW_FOR_EACH(BBW_LDS)
#undef BBW_LDS
    return -1;
}

size_t w3_image_bytes(int nb)
{
    switch (nb) {
    case 7: return (size_t)w3::WImg<7>::DW * 4;
    case 6: return (size_t)w3::WImg<6>::DW * 4;
    case 5: return (size_t)w3::WImg<5>::DW * 4;
    case 4: return (size_t)w3::WImg<4>::DW * 4;
    default: return 0;
    }
}

hipError_t launch_w3_image(int nb, int c64, const WImageArgs &a, int cps_max, hipStream_t st)
{
    if (a.n_entries < 1 || a.n_entries > 65535 || cps_max < 1) return hipErrorInvalidValue;
    switch (nb) {
    case 7: return c64 ? w3::run_image<7, true>(a, cps_max, st) : w3::run_image<7, false>(a, cps_max, st);
    case 6: return c64 ? w3::run_image<6, true>(a, cps_max, st) : w3::run_image<6, false>(a, cps_max, st);
    case 5: return c64 ? w3::run_image<5, true>(a, cps_max, st) : w3::run_image<5, false>(a, cps_max, st);
    case 4: return c64 ? w3::run_image<4, true>(a, cps_max, st) : w3::run_image<4, false>(a, cps_max, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_w3(int nb, int b2, int waves, int c64, const GemmArgs &a, int grid, hipStream_t st)
{
    if (waves != 4 && waves != 8) return hipErrorInvalidValue;
#define BBW_CASE(NB_, B2_) \
    if (nb == NB_ && b2 == B2_) { \
        if (waves == 8) \
            return c64 ? w3::run_contract8<NB_, B2_, true>(a, grid, st) : w3::run_contract8<NB_, B2_, false>(a, grid, st); \
        return c64 ? w3::run_contract<NB_, B2_, true>(a, grid, st) : w3::run_contract<NB_, B2_, false>(a, grid, st); \
    }
    BBW_FOR_EACH(BBW_CASE)
#undef BBW_CASE
    return hipErrorInvalidValue;
}
#undef BBW_FOR_EACH

}  // namespace bb
