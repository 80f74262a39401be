// FP64 paper-order contraction kernels of libbblock.so (gfx950, plan kernels
// 6 and 8: momentum fragments of 16 and of 4).
//
// The block of the paper (Sec. 2, eq. (3)) in the order of Algorithm 1: per
// site the singlet
//   S[x; (d1,d2), d3] = sum_c D_c[x; d1,d2] q3_c[x; d3],  D_c = eps_abc q1_a q2_b,
// then its projection on the momenta, a complex GEMM with rows (d1,d2,d3),
// columns p and contraction index x:
//   B[p][(d1,d2)][d3] = sum_x S[x; (d1,d2), d3] exp(-i p.x),
// in complex double throughout.  Per (site, row) the matrix cores do one
// complex multiply-add per momentum instead of the fused form's three (one
// per colour), and the vector unit forms the singlet (12 FMAs); on gfx950
// FP64 vector and matrix work run at the same rate and do not overlap, so
// this order is the cheaper one once the momenta outnumber the colours'
// share of the padding.
//
// Complex products with three real products (Gauss), as in kernel 5:
//   P1 = (Sr + Si)(er + ei),  P2 = Sr er,  P3 = Si ei,
//   Re = P2 - P3,  Im = P1 - P2 - P3,  e = exp(-i p.x).
//
// Workgroup: eight wave64, two per SIMD.  Tile: 128 RS rows = NPAIR (d1,d2)
// pairs x a block of B3 d3 values, W CF momenta, one site split.  Wave w
// owns RS row sets of 16 rows (the same 16 d3 values of RS pairs) and all
// momenta: 3 x CF accumulator fragments per row set, of
// v_mfma_f64_16x16x4_f64 (W = 16) or v_mfma_f64_4x4x4_f64 (W = 4: its four
// blocks take the 16 rows four at a time against the same 4 momenta).  The
// A operand of a k-step (4 sites) is the singlet itself: lane l forms S of
// row l % 16 of each row set at site l / 16 from the diquark and q3 tiles in
// LDS, in registers, and feeds it to the MFMAs (both MFMA forms take A[i][k]
// from lane i + 16 k).  Where the registers allow (W = 4, or one fragment
// of 16) the singlets run one k-step ahead: a k-step's MFMAs take the
// singlets formed in the previous one, and the next singlets form after
// them, so the vector chain's latency is not in front of the MFMAs that
// wait for it.  Per chunk of 32 sites (16 where two
// buffers of 32 would not fit the LDS) the
// workgroup builds the next chunk's tiles (the diquark of its pairs, q3 of
// its d3 block, the phases of its momenta with their Re + Im plane) into the
// other LDS buffer from registers loaded a chunk earlier, and issues the
// loads of the chunk after it.  Quark and phase-index loads go through
// per-chunk buffer resources: loads past the split, of pairs past M, of d3
// past n3 or momenta past n_mom return zero (no masks).
//
// Zero momentum (instantiation Z, a.p_skip >= 0): its phase is 1 at every
// site, so its projection is the plain site sum of the singlet.  Each lane
// adds its singlets into two registers, the four k-groups are summed across
// lanes at the end, and the tiles of column block 0 write it; the columns
// hold the other momenta, so a set of 16 k + 1 momenta takes k fragments.
#include <algorithm>

#include "bb_fast.h"
#include "bb_internal.h"

namespace bb {
namespace f64p {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int WG = 512;     // eight waves
constexpr int MT = 128;     // rows (pair, d3) per tile and row set, 16 per wave
constexpr uint32_t OOB = 0x80000000u;  // a buffer offset past any range: loads return zero
constexpr size_t LDS_LIMIT = 160 * 1024;

// Doubles of one LDS buffer for chunks of s sites: D [3][s][dst] (dst: the
// site stride, pairs + 1) and q3 [3][s][b3] as (re, im) pairs, then the
// phase planes Re, Im, Re + Im [s][ps].
constexpr int buffer_doubles(int s, int dst, int b3, int ps) { return 2 * 3 * s * dst + 2 * 3 * s * b3 + 3 * s * ps; }

// Column fragments of W momenta: W = 16 on v_mfma_f64_16x16x4_f64 (plan
// kernel 6), W = 4 on v_mfma_f64_4x4x4_f64 with its four blocks taking the
// wave's 16 rows four at a time against one shared set of 4 columns (plan
// kernel 8: few momenta pad to a multiple of 4, not of 16).  RS row sets of
// 16 rows per wave: with RS = 2 (d3 blocks of 16) a wave holds the same 16
// d3 values of two pairs, reads q3 once for both singlets and has two
// independent singlet chains per k-step.
template <int CF, int B3, int W = 16, int RS = 1>
struct Shape {
    static constexpr int NPAIR = RS * MT / B3;                // (d1,d2) pairs per tile
    // Site stride of the diquark tile (double2): one past the pairs, so
    // that the four k-groups' broadcast reads of one pair sit in different
    // banks (at a multiple of 256 bytes they conflict four ways).
    static constexpr int DST = NPAIR + 1;
    static constexpr int NC = W * CF;                         // momenta per tile
    // Site stride of the phase planes (doubles): the two k-groups of a
    // half-wave read disjoint banks.
    static constexpr int PS = (W == 4) ? NC : (NC % 32 == 0) ? NC + 16 : NC;
    // Sites per chunk: 32 where two buffers of that size fit the LDS (one
    // barrier and one tile build per 32 sites), else 16.
    static constexpr int SITES =
        2 * (size_t)buffer_doubles(32, DST, B3, PS) * 8 + (size_t)MAX_L * 16 <= LDS_LIMIT ? 32 : 16;
    static constexpr int KS = SITES / 4;                      // k-steps per chunk
    static constexpr int ND = NPAIR * SITES;                  // diquark items per chunk
    static constexpr int NQ = SITES * 3 * B3;                 // q3 values per chunk
    static constexpr int NP = SITES * NC;                     // phases per chunk
    static constexpr int JQ = (NQ + WG - 1) / WG, JP = (NP + WG - 1) / WG;
    static constexpr int DOFF = 0, QOFF = 2 * 3 * SITES * DST, POFF = QOFF + 2 * 3 * SITES * B3;
    static constexpr int BUF = POFF + 3 * SITES * PS;  // doubles
    static constexpr size_t lds = (size_t)2 * BUF * 8 + (size_t)MAX_L * 16;
    static_assert(BUF == buffer_doubles(SITES, DST, B3, PS) && lds <= LDS_LIMIT, "two buffers fit the LDS");
    static_assert(W == 4 || PS % 32 == 16, "the two k-groups of a half-wave must read disjoint banks");
    static_assert(W == 16 || W == 4, "16- or 4-wide column fragments");
    static_assert(B3 % 16 == 0 && MT % B3 == 0, "a wave's 16 rows are d3 values of one pair");
    static_assert(RS == 1 || (RS == 2 && B3 == 16), "two row sets: the same d3 block of two pairs");
    static_assert(ND % 64 == 0 && ND <= WG, "diquark items end on a wave boundary, one per thread");
    static_assert(NQ % 64 == 0 && NP % 64 == 0, "q3 and phase items end on a wave boundary");
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
__device__ __forceinline__ std::conditional_t<C64, float2, double2> ldq(__amdgpu_buffer_rsrc_t rs, uint32_t off)
{
    // As loaded: a complex64 value is widened where it is used (to_f64), so
    // that the load is waited for there, a chunk after its issue, and stays
    // in two registers meanwhile.
    if constexpr (C64)
        return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
    else
        return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
}

__device__ __forceinline__ double2 to_f64(double2 v) { return v; }
__device__ __forceinline__ double2 to_f64(float2 v) { return make_double2(v.x, v.y); }

// Resource over sites [x0, x0 + SITES) of a field [V][3][n] (bytes in range:
// the sites below xe only; none when x0 >= xe).
template <int SITES, bool C64>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t chunk_rsrc(const void *q, int n, int x0, int xe)
{
    constexpr int ESZ = In<C64>::ESZ;
    const int ns = __builtin_amdgcn_readfirstlane(min(max(xe - x0, 0), SITES));  // wave-uniform: no waterfall
    const unsigned char *base = static_cast<const unsigned char *>(q) + (size_t)x0 * 3 * n * ESZ;
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, ns * 3 * n * ESZ, 0x00020000);
}

template <int CF, int B3, bool C64, bool Z, int W, int RS>
__global__ void __launch_bounds__(WG, 1) contract(GemmArgs a)
{
    static_assert(!(Z && W == 4), "the zero momentum on the vector unit saves a fragment of 16");
    using Sh = Shape<CF, B3, W, RS>;
    using AccT = std::conditional_t<W == 16, d4_t, double>;
    constexpr int NPAIR = Sh::NPAIR, NC = Sh::NC, PS = Sh::PS, BUF = Sh::BUF, SITES = Sh::SITES, KS = Sh::KS;
    constexpr int ESZ = In<C64>::ESZ;
    // Singlets one k-step ahead of the MFMAs that take them (the vector
    // chain's latency then runs behind the previous k-step's MFMAs) where
    // the extra singlet registers fit: fragments of 4, or one of 16; wider
    // tiles of 16 would spill.
    constexpr bool SKEW = W == 4 || CF == 1;
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

        std::conditional_t<C64, float2, double2> u[3], v[3], w[Sh::JQ];
        uint32_t kk[Sh::JP];
        auto issue = [&](int ci) {
            const int x0 = __builtin_amdgcn_readfirstlane(xs + ci * SITES);
            if (has_d) {
                const __amdgpu_buffer_rsrc_t rs1 = chunk_rsrc<SITES, C64>(bd.q1, bd.n1, x0, xe);
                const __amdgpu_buffer_rsrc_t rs2 = chunk_rsrc<SITES, C64>(bd.q2, bd.n2, x0, xe);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    u[c] = ldq<C64>(rs1, o1[c]);
                    v[c] = ldq<C64>(rs2, o2[c]);
                }
            }
            const __amdgpu_buffer_rsrc_t rs3 = chunk_rsrc<SITES, C64>(bd.q3, bd.n3, x0, xe);
#pragma unroll
            for (int j = 0; j < Sh::JQ; ++j) w[j] = ldq<C64>(rs3, o3[j]);
            const __amdgpu_buffer_rsrc_t rsk = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(a.kidx + min(x0, krec)), (short)0, max(krec - x0, 0), 0x00020000);
#pragma unroll
            for (int j = 0; j < Sh::JP; ++j) kk[j] = __builtin_amdgcn_raw_buffer_load_b8(rsk, ok[j], 0, 0);
        };
        // The loaded chunk into buffer b: diquark u_a v_b - u_b v_a
        // (eps_{a b c} = +1) per colour, q3 as loaded, the phases
        // roots[k] = exp(-2 pi i k / L) with their Re + Im plane.
        auto build = [&](int b) {
            asm volatile("" : "+s"(b));  // one base register per buffer, immediate offsets from it
            double *base = lds + b * BUF;
            double2 *Dt = reinterpret_cast<double2 *>(base + Sh::DOFF);
            double2 *Qt = reinterpret_cast<double2 *>(base + Sh::QOFF);
            double *Pr = base + Sh::POFF, *Pi = Pr + SITES * PS, *Ps = Pi + SITES * PS;
            if (has_d) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double2 ua = to_f64(u[(c + 1) % 3]), ub = to_f64(u[(c + 2) % 3]);
                    const double2 va = to_f64(v[(c + 1) % 3]), vb = to_f64(v[(c + 2) % 3]);
                    const double re = __builtin_fma(ua.x, vb.x, __builtin_fma(-ua.y, vb.y, __builtin_fma(-ub.x, va.x, ub.y * va.y)));
                    const double im = __builtin_fma(ua.x, vb.y, __builtin_fma(ua.y, vb.x, __builtin_fma(-ub.x, va.y, -(ub.y * va.x))));
                    Dt[(c * SITES + ds) * Sh::DST + dp] = make_double2(re, im);
                }
            }
#pragma unroll
            for (int j = 0; j < Sh::JQ; ++j) {
                const int q = tid + WG * j;
                if (q < Sh::NQ) {
                    const int d = q % B3, sc = q / B3, s = sc / 3, c = sc - 3 * s;
                    Qt[(c * SITES + s) * B3 + d] = to_f64(w[j]);
                }
            }
#pragma unroll
            for (int j = 0; j < Sh::JP; ++j) {
                const int q = tid + WG * j;
                if (q < Sh::NP) {
                    const int jc = q % NC, s = q / NC;
                    const double2 e = roots[kk[j]];
                    Pr[s * PS + jc] = e.x;
                    Pi[s * PS + jc] = e.y;
                    Ps[s * PS + jc] = e.x + e.y;
                }
            }
        };

        AccT acc[RS][3][CF];
#pragma unroll
        for (int r = 0; r < RS; ++r)
#pragma unroll
            for (int q = 0; q < 3; ++q)
#pragma unroll
                for (int n = 0; n < CF; ++n) acc[r][q][n] = AccT{};
        // A[i][k] from lane i + 16 k: row 16 (RS wave + r) + i of row set r
        // at site k of the k-step (row sets r of a wave: the same d3 values).
        const int li = lane & 15, kg = lane >> 4;
        const int rw = wave * RS * 16 + li;
        const int pair_l = rw / B3, d3_l = rw % B3;  // row set r: pair pair_l + r

        // One chunk from buffer b: per k-step the singlets of this lane's
        // (row, site) from LDS, then 3 CF MFMAs; after the first k-step the
        // next chunk's tiles go into buffer b ^ 1 and the loads of the chunk
        // after it are issued.
        double zr[RS] = {}, zi[RS] = {};  // this lane's (row, site) singlets summed: the zero momentum
        auto chunk = [&](int b, int ci_next) {
            asm volatile("" : "+s"(b));
            // Per-lane bases (one address each; the k-step, colour, plane and
            // fragment offsets are immediates).
            const double *base = lds + b * BUF;
            const double2 *Dl = reinterpret_cast<const double2 *>(base + Sh::DOFF) + kg * Sh::DST + pair_l;
            const double2 *Ql = reinterpret_cast<const double2 *>(base + Sh::QOFF) + kg * B3 + d3_l;
            // B[k][j]: lane j + 16 k (W = 16); lane j + 4 b + 16 k for every
            // block b (W = 4: the blocks share the columns).
            const double *Pl = base + Sh::POFF + kg * PS + (W == 16 ? li : (li & 3));
            double2 dv[2][RS][3], qv[2][3];
            double br[2][CF], bi[2][CF], bs[2][CF];
            // Operands of k-step ks into register set slot: the diquark and
            // q3 of this lane's (row, site), the phases of its columns.
            auto read_s = [&](int ks, int slot) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
#pragma unroll
                    for (int r = 0; r < RS; ++r) dv[slot][r][c] = Dl[(c * SITES + 4 * ks) * Sh::DST + r];
                    qv[slot][c] = Ql[(c * SITES + 4 * ks) * B3];
                }
#pragma unroll
                for (int n = 0; n < CF; ++n) {
                    br[slot][n] = Pl[4 * ks * PS + n * W];
                    bi[slot][n] = Pl[(SITES + 4 * ks) * PS + n * W];
                    bs[slot][n] = Pl[(2 * SITES + 4 * ks) * PS + n * W];
                }
            };
            double sr[RS], si[RS], ss[RS];
            // Singlet S = sum_c D_c q3_c (complex) of each row set from
            // register set slot, its Re + Im.
            auto singlet = [&](int slot) {
#pragma unroll
                for (int r = 0; r < RS; ++r) {
                    const double2 *dr = dv[slot][r];
                    sr[r] = __builtin_fma(dr[0].x, qv[slot][0].x, -(dr[0].y * qv[slot][0].y));
                    si[r] = __builtin_fma(dr[0].x, qv[slot][0].y, dr[0].y * qv[slot][0].x);
#pragma unroll
                    for (int c = 1; c < 3; ++c) {
                        sr[r] = __builtin_fma(dr[c].x, qv[slot][c].x, sr[r]);
                        sr[r] = __builtin_fma(-dr[c].y, qv[slot][c].y, sr[r]);
                        si[r] = __builtin_fma(dr[c].x, qv[slot][c].y, si[r]);
                        si[r] = __builtin_fma(dr[c].y, qv[slot][c].x, si[r]);
                    }
                    ss[r] = sr[r] + si[r];
                }
                if constexpr (Z) {
#pragma unroll
                    for (int r = 0; r < RS; ++r) {
                        zr[r] += sr[r];
                        zi[r] += si[r];
                    }
                }
            };
            // The momentum projection of the current singlets, phases from register set slot.
            auto project = [&](int slot) {
#pragma unroll
                for (int r = 0; r < RS; ++r)
#pragma unroll
                    for (int n = 0; n < CF; ++n) {
                        if constexpr (W == 16) {
                            acc[r][0][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(ss[r], bs[slot][n], acc[r][0][n], 0, 0, 0);
                            acc[r][1][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(sr[r], br[slot][n], acc[r][1][n], 0, 0, 0);
                            acc[r][2][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(si[r], bi[slot][n], acc[r][2][n], 0, 0, 0);
                        } else {
                            acc[r][0][n] = __builtin_amdgcn_mfma_f64_4x4x4f64(ss[r], bs[slot][n], acc[r][0][n], 0, 0, 0);
                            acc[r][1][n] = __builtin_amdgcn_mfma_f64_4x4x4f64(sr[r], br[slot][n], acc[r][1][n], 0, 0, 0);
                            acc[r][2][n] = __builtin_amdgcn_mfma_f64_4x4x4f64(si[r], bi[slot][n], acc[r][2][n], 0, 0, 0);
                        }
                    }
            };
            read_s(0, 0);
            if constexpr (SKEW) {
                if constexpr (KS > 1) read_s(1, 1);
                singlet(0);
            }
            fast::static_for<0, KS>([&](auto kk_) {
                constexpr int ks = kk_, slot = ks & 1;
                if constexpr (SKEW) {
                    // This k-step's MFMAs on the singlets formed in the last
                    // one; the k-step after next loads into this one's
                    // registers and the next singlet forms after the MFMAs.
                    project(slot);
                    if constexpr (ks + 2 < KS) read_s(ks + 2, slot);
                    if constexpr (ks + 1 < KS) singlet(slot ^ 1);
                } else {
                    singlet(slot);
                    // The next k-step's operands load under this one's MFMAs.
                    if constexpr (ks + 1 < KS) read_s(ks + 1, slot ^ 1);
                    project(slot);
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
#pragma unroll
            for (int r = 0; r < RS; ++r) {
                zr[r] += __shfl_xor(zr[r], 16);
                zi[r] += __shfl_xor(zi[r], 16);
                zr[r] += __shfl_xor(zr[r], 32);
                zi[r] += __shfl_xor(zi[r], 32);
            }
        }

        // Epilogue: Re = P2 - P3, Im = P1 - P2 - P3.  W = 16: accumulator
        // register e of a fragment holds row 4 e + lane / 16, column
        // lane % 16.  W = 4: the lane's one value is block b = (lane / 4) % 4,
        // row i = lane / 16 of it (wave row 4 b + i), column lane % 4.
        with_put_mode(bd, tl.w, [&](auto mode) {
#pragma unroll
            for (int rs = 0; rs < RS; ++rs)
#pragma unroll
                for (int n = 0; n < CF; ++n) {
                    const int col = p0 + n * W + (W == 16 ? li : (lane & 3));
                    if (col >= n_col) continue;
                    const int p = col + (Z && col >= ps ? 1 : 0);
                    constexpr int NE = W == 16 ? 4 : 1;
#pragma unroll
                    for (int e = 0; e < NE; ++e) {
                        const int r = (wave * RS + rs) * 16 + (W == 16 ? 4 * e + kg : 4 * ((lane >> 2) & 3) + kg);
                        const int mo = m12_0 + r / B3, d3 = d3_0 + r % B3;
                        if (mo >= M12 || d3 >= bd.n3) continue;
                        double p1, p2, p3;
                        if constexpr (W == 16) {
                            p1 = acc[rs][0][n][e];
                            p2 = acc[rs][1][n][e];
                            p3 = acc[rs][2][n][e];
                        } else {
                            p1 = acc[rs][0][n];
                            p2 = acc[rs][1][n];
                            p3 = acc[rs][2][n];
                        }
                        const double re = p2 - p3, im = (p1 - p2) - p3;
                        const int nu = p * bd.n3 + d3;
                        put_result<decltype(mode)::value, double>(bd, tl.w, mo, nu, p, d3, 0, re);
                        put_result<decltype(mode)::value, double>(bd, tl.w, mo, nu, p, d3, 1, im);
                    }
                }
            if (Z && zsum && kg == 0) {
#pragma unroll
                for (int r = 0; r < RS; ++r) {
                    const int mo = m12_0 + pair_l + r, d3 = d3_0 + d3_l;
                    if (mo < M12 && d3 < bd.n3) {
                        const int nu = ps * bd.n3 + d3;
                        put_result<decltype(mode)::value, double>(bd, tl.w, mo, nu, ps, d3, 0, zr[r]);
                        put_result<decltype(mode)::value, double>(bd, tl.w, mo, nu, ps, d3, 1, zi[r]);
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

template <int CF, int B3, bool C64, int RS>
hipError_t run(const GemmArgs &a, int grid, hipStream_t st)
{
    if (a.p_skip >= 0)
        contract<CF, B3, C64, true, 16, RS><<<dim3(grid), dim3(WG), 0, st>>>(a);
    else
        contract<CF, B3, C64, false, 16, RS><<<dim3(grid), dim3(WG), 0, st>>>(a);
    return hipGetLastError();
}

template <int CF, int B3, bool C64>
hipError_t run_narrow(const GemmArgs &a, int grid, hipStream_t st)
{
    if (a.p_skip >= 0) return hipErrorInvalidValue;  // a fragment of 4 gains nothing from it
    contract<CF, B3, C64, false, 4, F64N_ROW_SETS><<<dim3(grid), dim3(WG), 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace f64p

int f64p_lds_bytes(int cf, int b3, int w)
{
    if (b3 != 16) return -1;
#define BBQ_SIZE(CF_, W_, RS_) \
    if (cf == CF_ && w == W_) return (int)f64p::Shape<CF_, 16, W_, RS_>::lds;
    BBQ_SIZE(1, 16, f64p_row_sets(1)) BBQ_SIZE(2, 16, f64p_row_sets(2)) BBQ_SIZE(3, 16, f64p_row_sets(3))
    BBQ_SIZE(1, 4, F64N_ROW_SETS) BBQ_SIZE(2, 4, F64N_ROW_SETS) BBQ_SIZE(3, 4, F64N_ROW_SETS)
    BBQ_SIZE(4, 4, F64N_ROW_SETS)
#undef BBQ_SIZE
    return -1;
}

int f64p_pairs(int cf, int b3, int w)
{
    if (b3 != 16) return -1;
    return (w == 4 ? F64N_ROW_SETS : f64p_row_sets(cf)) * f64p::MT / b3;
}

hipError_t launch_f64p(int cf, int b3, int c64, const GemmArgs &a, int grid, hipStream_t st)
{
    if (b3 != 16) return hipErrorInvalidValue;
#define BBQ_CASE(CF_)                                                                \
    if (cf == CF_)                                                                   \
        return c64 ? f64p::run<CF_, 16, true, f64p_row_sets(CF_)>(a, grid, st)      \
                   : f64p::run<CF_, 16, false, f64p_row_sets(CF_)>(a, grid, st);
    BBQ_CASE(1) BBQ_CASE(2) BBQ_CASE(3)
#undef BBQ_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_f64n(int cf, int b3, int c64, const GemmArgs &a, int grid, hipStream_t st)
{
#define BBQ_CASE(CF_, B3_)          \
    if (cf == CF_ && b3 == B3_)     \
        return c64 ? f64p::run_narrow<CF_, B3_, true>(a, grid, st) : f64p::run_narrow<CF_, B3_, false>(a, grid, st);
    BBQ_CASE(1, 16) BBQ_CASE(2, 16) BBQ_CASE(3, 16) BBQ_CASE(4, 16)
#undef BBQ_CASE
    return hipErrorInvalidValue;
}

}  // namespace bb
