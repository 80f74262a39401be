// FP64 contraction kernel of libbblock.so (gfx950, plan kernel 5).
//
// The block of the paper (Sec. 2, eq. (3)) as one complex GEMM per block,
//   C[(d1,d2), (p,d3)] = sum_{kappa=(c,x)} D[kappa, (d1,d2)] W[kappa, (p,d3)],
// with the diquark D_c = eps_abc q1_a q2_b of Algorithm 1 as the row operand
// and the phase-weighted third quark W_c = q3_c exp(-i p.x) as the column
// operand, in complex double throughout (the paper's arithmetic, Sec. 4).
//
// Complex products with three real products (Gauss): for D = Dr + i Di and
// W = Wr + i Wi,
//   P1 = (Dr + Di)(Wr + Wi),  P2 = Dr Wr,  P3 = Di Wi,
//   Re(D W) = P2 - P3,        Im(D W) = P1 - P2 - P3,
// so the matrix cores run three real GEMMs of M x N x K instead of the four
// of the usual real embedding: 6 real flops per complex multiply-add on
// v_mfma_f64_16x16x4_f64 instead of 8.
//
// On gfx950 no vector instruction issues on a SIMD while an FP64 MFMA
// occupies it (the counters show zero MFMA/VALU co-execution), so every
// vector instruction costs matrix time.  The kernel keeps them few:
//   * quark loads go through buffer resources whose base and range advance
//     per chunk in scalar registers: no vector address arithmetic, and loads
//     past the split, of rows past M or of columns past N are out of range
//     and return zero (no masks);
//   * the diquark and the phase product are written as fused multiply-adds;
//   * the column sum Wr + Wi is formed once per element when W is built and
//     stored as a third plane, not once per row fragment before each MFMA.
//
// Workgroup: eight wave64, two per SIMD, all doing the same work (while one
// wave of a SIMD waits on LDS or a barrier, the other's MFMAs run).  Tile: 128
// complex rows x 16 CF columns x one site split.  Wave w owns rows 16 w to
// 16 w + 15 and all columns: 3 x CF accumulator fragments of 16 x 16 doubles
// (one per product P1, P2, P3).  Per chunk of 4 sites (12 kappa) a wave runs 3
// k-steps x CF fragments x 3 MFMAs from LDS buffer i & 1, reading the operands
// of fragment f + 1 during fragment f.  Between its last 11 MFMA groups (fenced
// by scheduling barriers) it builds its share of chunk i + 1 into the other
// buffer from registers loaded a chunk earlier: each thread one diquark item
// (row tid % 128 at site tid / 128, three colours) and, in the waves that hold
// one, one W item (column tid % NT at site tid / NT); then it issues the loads
// of chunk i + 2.  The latencies of those loads and of the LDS stores then run
// under the MFMAs, and only the issue slots of the vector instructions cost
// matrix time.  One barrier per chunk.  Tiles are stored k-major
// ([plane][kappa][row]) with row strides of 16 mod 32 doubles, so the two
// k-groups of a half-wave read disjoint LDS banks.
#include <algorithm>

#include "bb_fast.h"
#include "bb_internal.h"

namespace bb {
namespace f64 {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int WG = 512;        // eight waves
constexpr int MT = 128;        // complex rows per tile (16 per wave)
constexpr int SITES = 4;       // sites per chunk (divides CHUNK_SITES, the split granularity)
constexpr int KC = 3 * SITES;  // kappa per chunk
constexpr int DS = MT + 16;    // kappa stride of the D planes (doubles)
static_assert(DS % 32 == 16 && MT * SITES == WG, "D stride off the banks; one D item per thread");
constexpr uint32_t OOB = 0x80000000u;  // a buffer offset past any range: loads return zero

template <int CF>
struct Shape {
    static constexpr int NT = 16 * CF;                          // complex columns per tile
    static constexpr int WS = (NT % 32 == 0) ? NT + 16 : NT;   // kappa stride of the W planes
    static constexpr int DPL = KC * DS, WPL = KC * WS;          // doubles per plane
    static constexpr int BUF = 2 * DPL + 3 * WPL;               // D: Re, Im; W: Re, Im, Re + Im
    static constexpr size_t lds = (size_t)2 * BUF * 8 + (size_t)MAX_L * 16;
    static_assert(WS % 32 == 16, "k-groups must fall on disjoint banks");
    static_assert((NT * SITES) % 64 == 0 && NT * SITES <= WG, "W items end on a wave boundary, one per thread");
};

template <bool C64>
struct In {
    typedef double __attribute__((ext_vector_type(2))) T;
    static constexpr int ESZ = 16;
};
template <>
struct In<true> {
    typedef float __attribute__((ext_vector_type(2))) T;
    static constexpr int ESZ = 8;
};

template <bool C64>
__device__ __forceinline__ double2 ldq(__amdgpu_buffer_rsrc_t rs, uint32_t off)
{
    if constexpr (C64) {
        const float2 v = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
        return make_double2(v.x, v.y);
    } else {
        return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
    }
}

// Resource over sites [x0, x0 + SITES) of a field [V][3][n] (bytes in range:
// the sites below xe only; none when x0 >= xe).
template <bool C64>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t chunk_rsrc(const void *q, int n, int x0, int xe)
{
    constexpr int ESZ = In<C64>::ESZ;
    const int ns = min(max(xe - x0, 0), SITES);
    const unsigned char *base = static_cast<const unsigned char *>(q) + (size_t)x0 * 3 * n * ESZ;
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, ns * 3 * n * ESZ, 0x00020000);
}

template <int CF, bool C64>
__global__ void __launch_bounds__(WG, 1) contract(GemmArgs a)
{
    using Sh = Shape<CF>;
    constexpr int NT = Sh::NT, WS = Sh::WS, DPL = Sh::DPL, WPL = Sh::WPL, BUF = Sh::BUF;
    constexpr int ESZ = In<C64>::ESZ;
    constexpr int NW = NT * SITES;  // W items per chunk (one per thread, waves past it have none)
    __shared__ __align__(16) double lds[2 * BUF];
    __shared__ double2 roots[MAX_L];
    __shared__ int s_tile;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int k = tid; k < a.L; k += WG) roots[k] = make_double2(a.roots[2 * k], a.roots[2 * k + 1]);

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
        const int m0 = tl.y * MT, nu0 = tl.z * NT;
        const int xs = tl.w * bd.sps;
        const int xe = min(a.V, xs + bd.sps);
        const int n_chunks = (xe - xs + SITES - 1) / SITES;

        // ---- generation items of this thread (tile invariant) ----
        // D item: row r = tid % 128 at site s = tid / 128 of each chunk.
        const int r = tid & (MT - 1), s = tid >> 7;
        const int m = m0 + r;
        const bool mok = m < bd.M;
        const int d1 = mok ? m / bd.n2 : 0, d2 = mok ? m - (m / bd.n2) * bd.n2 : 0;
        uint32_t o1[3], o2[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            o1[c] = mok ? (uint32_t)(((s * 3 + c) * bd.n1 + d1) * ESZ) : OOB;
            o2[c] = mok ? (uint32_t)(((s * 3 + c) * bd.n2 + d2) * ESZ) : OOB;
        }
        // W item: column j = tid % NT at site tid / NT (threads past NW: none).
        const bool has_w = wave * 64 < NW;  // wave-uniform: NW is a multiple of 64
        const int wj = tid % NT, wsite = tid / NT;
        const int nu = nu0 + wj;
        const bool wok = tid < NW && nu < bd.N;
        const int p = wok ? nu / bd.n3 : 0, d3 = wok ? nu - (nu / bd.n3) * bd.n3 : 0;
        uint32_t o3[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) o3[c] = wok ? (uint32_t)(((wsite * 3 + c) * bd.n3 + d3) * ESZ) : OOB;
        const uint32_t ok = (uint32_t)(p * a.kstride + wsite);
        const int krec = a.n_mom * a.kstride;

        double2 u[3], v[3], w[3];
        uint32_t kk = 0;
        auto issue = [&](int ci) {
            const int x0 = xs + ci * SITES;
            const __amdgpu_buffer_rsrc_t rs1 = chunk_rsrc<C64>(bd.q1, bd.n1, x0, xe);
            const __amdgpu_buffer_rsrc_t rs2 = chunk_rsrc<C64>(bd.q2, bd.n2, x0, xe);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                u[c] = ldq<C64>(rs1, o1[c]);
                v[c] = ldq<C64>(rs2, o2[c]);
            }
            if (has_w) {
                const __amdgpu_buffer_rsrc_t rs3 = chunk_rsrc<C64>(bd.q3, bd.n3, x0, xe);
                const __amdgpu_buffer_rsrc_t rsk = __builtin_amdgcn_make_buffer_rsrc(
                    (void *)(a.kidx + min(x0, krec)), (short)0, max(krec - x0, 0), 0x00020000);
#pragma unroll
                for (int c = 0; c < 3; ++c) w[c] = ldq<C64>(rs3, o3[c]);
                kk = __builtin_amdgcn_raw_buffer_load_b8(rsk, ok, 0, 0);
            }
        };
        // Diquark u_a v_b - u_b v_a (eps_{a b c} = +1) and W_c = q3_c
        // exp(-i p.x) of the loaded chunk into buffer b.
        auto build = [&](int b) {
            // The buffer offset stays a register value: folded into every
            // store it would exceed the 16-bit LDS offset field and cost one
            // address register per store.
            asm volatile("" : "+s"(b));
            double *Dr = lds + b * BUF, *Di = Dr + DPL, *Wr = Di + DPL, *Wi = Wr + WPL, *Wsum = Wi + WPL;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double2 ua = u[(c + 1) % 3], ub = u[(c + 2) % 3];
                const double2 va = v[(c + 1) % 3], vb = v[(c + 2) % 3];
                const double re = __builtin_fma(ua.x, vb.x, __builtin_fma(-ua.y, vb.y, __builtin_fma(-ub.x, va.x, ub.y * va.y)));
                const double im = __builtin_fma(ua.x, vb.y, __builtin_fma(ua.y, vb.x, __builtin_fma(-ub.x, va.y, -(ub.y * va.x))));
                Dr[(c * SITES + s) * DS + r] = re;
                Di[(c * SITES + s) * DS + r] = im;
            }
            if (has_w) {
                const double2 e = roots[kk];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double wr = __builtin_fma(w[c].x, e.x, -(w[c].y * e.y));
                    const double wi = __builtin_fma(w[c].x, e.y, w[c].y * e.x);
                    const int o = (c * SITES + wsite) * WS + wj;
                    Wr[o] = wr;
                    Wi[o] = wi;
                    Wsum[o] = wr + wi;
                }
            }
        };

        d4_t acc[3][CF];
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int n = 0; n < CF; ++n) acc[q][n] = d4_t{0.0, 0.0, 0.0, 0.0};
        // A[i][k] from lane i + 16 k, B[k][j] from lane j + 16 k.
        const int li = lane & 15, kg = lane >> 4;
        const int arow = wave * 16 + li;

        // One chunk: the MFMAs of the chunk in buffer b, in 3 CF groups of
        // one column fragment's three products, each group followed (in
        // program order, fenced) by a slice of the next chunk's generation
        // into buffer b ^ 1 and, once the registers are consumed, the loads
        // of the chunk after it.  A vector instruction cannot issue while an
        // FP64 MFMA occupies the SIMD, so the slices cost their issue time,
        // but their latencies and the LDS and memory latencies run under
        // the MFMAs.  Operands of fragment f + 1 are read during fragment f.
        auto chunk = [&](int b, int ci_next) {
            asm volatile("" : "+s"(b));  // one base register per buffer, immediate offsets from it
            const double *Dr = lds + b * BUF, *Di = Dr + DPL, *Wr = Di + DPL, *Wi = Wr + WPL, *Wsum = Wi + WPL;
            double *nDr = lds + (b ^ 1) * BUF, *nDi = nDr + DPL, *nWr = nDi + DPL, *nWi = nWr + WPL;
            double *nWs = nWi + WPL;
            constexpr int NG = 3 * CF;  // groups per chunk
            double a_r = Dr[kg * DS + arow], a_i = Di[kg * DS + arow];
            double n_r = 0.0, n_i = 0.0;
            double b_r[2], b_i[2], b_s[2];
            b_r[0] = Wr[kg * WS + li];
            b_i[0] = Wi[kg * WS + li];
            b_s[0] = Wsum[kg * WS + li];
            double a_s = a_r + a_i;
            double dre[3], dim[3];
            double2 e = make_double2(0.0, 0.0);
            auto step = [&](auto ss) {
                constexpr int st = ss;
                if constexpr (st < 6) {
                    // Diquark colour c = st / 2 of this thread's (row, site).
                    constexpr int c = st / 2;
                    const double2 ua = u[(c + 1) % 3], ub = u[(c + 2) % 3];
                    const double2 va = v[(c + 1) % 3], vb = v[(c + 2) % 3];
                    if constexpr (st % 2 == 0) {
                        dre[c] = __builtin_fma(ua.x, vb.x, __builtin_fma(-ua.y, vb.y, __builtin_fma(-ub.x, va.x, ub.y * va.y)));
                        fast::pin(dre[c]);
                    } else {
                        dim[c] = __builtin_fma(ua.x, vb.y, __builtin_fma(ua.y, vb.x, __builtin_fma(-ub.x, va.y, -(ub.y * va.x))));
                        nDr[(c * SITES + s) * DS + r] = dre[c];
                        nDi[(c * SITES + s) * DS + r] = dim[c];
                    }
                } else if constexpr (st == 6) {
                    if (has_w) e = roots[kk];
                } else if constexpr (st < 10) {
                    // Phase-weighted q3, colour c.
                    constexpr int c = st - 7;
                    if (has_w) {
                        const double wr = __builtin_fma(w[c].x, e.x, -(w[c].y * e.y));
                        const double wi = __builtin_fma(w[c].x, e.y, w[c].y * e.x);
                        const int o = (c * SITES + wsite) * WS + wj;
                        nWr[o] = wr;
                        nWi[o] = wi;
                        nWs[o] = wr + wi;
                    }
                } else if constexpr (st == 10) {
                    issue(ci_next);  // the registers of this chunk are consumed
                }
            };
            fast::static_for<0, NG>([&](auto gg) {
                constexpr int g = gg, ks = g / CF, n = g % CF, f = g;
                // Operands of the next fragment (and of the next k-step's rows).
                if constexpr (n + 1 < CF) {
                    const int o = (4 * ks + kg) * WS + (n + 1) * 16 + li;
                    b_r[(f + 1) & 1] = Wr[o];
                    b_i[(f + 1) & 1] = Wi[o];
                    b_s[(f + 1) & 1] = Wsum[o];
                } else if constexpr (ks + 1 < KC / 4) {
                    const int kap = 4 * (ks + 1) + kg;
                    n_r = Dr[kap * DS + arow];
                    n_i = Di[kap * DS + arow];
                    b_r[(f + 1) & 1] = Wr[kap * WS + li];
                    b_i[(f + 1) & 1] = Wi[kap * WS + li];
                    b_s[(f + 1) & 1] = Wsum[kap * WS + li];
                }
                acc[0][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_s, b_s[f & 1], acc[0][n], 0, 0, 0);
                acc[1][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_r, b_r[f & 1], acc[1][n], 0, 0, 0);
                acc[2][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_i, b_i[f & 1], acc[2][n], 0, 0, 0);
                // The generation slices run in the last groups of the chunk,
                // so the loads they end with have a whole chunk to land
                // before the next chunk's slices read them.
                constexpr int G0 = NG > 11 ? NG - 11 : 0;
                if constexpr (g >= G0) fast::slot_steps<g - G0, NG - G0, 11>(step);
                if constexpr (n + 1 == CF && ks + 1 < KC / 4) {
                    a_r = n_r;
                    a_i = n_i;
                    a_s = a_r + a_i;
                }
                __builtin_amdgcn_sched_barrier(0);
            });
        };

        // Prologue: chunk 0 into buffer 0, chunk 1 in registers.
        issue(0);
        build(0);
        issue(1);
        __syncthreads();
        for (int i = 0; i < n_chunks; ++i) {
            chunk(i & 1, i + 2);  // past the split the loads are out of range (zeros)
            __syncthreads();
        }

        // Epilogue: Re = P2 - P3, Im = P1 - P2 - P3.  Accumulator register
        // e of a 16x16 f64 fragment holds row 4 e + lane / 16, column lane % 16.
        with_put_mode(bd, tl.w, [&](auto mode) {
#pragma unroll
            for (int n = 0; n < CF; ++n) {
                const int nuo = nu0 + n * 16 + li;
                if (nuo >= bd.N) continue;
                const int po = nuo / bd.n3, d3o = nuo - (nuo / bd.n3) * bd.n3;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int mo = m0 + wave * 16 + 4 * e + kg;
                    if (mo >= bd.M) continue;
                    const double p1 = acc[0][n][e], p2 = acc[1][n][e], p3 = acc[2][n][e];
                    const double re = p2 - p3, im = (p1 - p2) - p3;
                    put_result<decltype(mode)::value, double>(bd, tl.w, mo, nuo, po, d3o, 0, re);
                    put_result<decltype(mode)::value, double>(bd, tl.w, mo, nuo, po, d3o, 1, im);
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

template <int CF, bool C64>
hipError_t run(const GemmArgs &a, int grid, hipStream_t st)
{
    contract<CF, C64><<<dim3(grid), dim3(WG), 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace f64

int f64_lds_bytes(int cf)
{
    switch (cf) {
    case 2: return (int)f64::Shape<2>::lds;
    case 4: return (int)f64::Shape<4>::lds;
    case 7: return (int)f64::Shape<7>::lds;
    default: return -1;
    }
}

hipError_t launch_f64(int cf, int c64, const GemmArgs &a, int grid, hipStream_t st)
{
#define BBD_CASE(CF_) \
    if (cf == CF_) return c64 ? f64::run<CF_, true>(a, grid, st) : f64::run<CF_, false>(a, grid, st);
    BBD_CASE(2) BBD_CASE(4) BBD_CASE(7)
#undef BBD_CASE
    return hipErrorInvalidValue;
}

}  // namespace bb
