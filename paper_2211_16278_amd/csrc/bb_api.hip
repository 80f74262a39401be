// Host side of libbblock.so: the C ABI declared in include/bblock.h.
//
// Responsibilities: argument validation, the phase tables (paper, Sec. 3:
// the phase of the momentum projection is precomputed and reused across
// kernel invocations with the same momentum set), the planner (kernel, tile
// shape, split-K count, workspace), the grouped tile schedule, hipGraph
// capture and replay of grouped launches, and the autotuner (the paper tunes
// its block sizes experimentally per machine, Sec. 4; here the kernel, tile
// shape, split count and scheduling mode are timed on the device).

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bblock.h"
#include "bb_internal.h"

using namespace bb;

// Size of the static device scratch array of the allocation-free entry point.
constexpr size_t SCRATCH_BYTES = BBLOCK_NOALLOC_SCRATCH_BYTES;
static_assert(SCRATCH_BYTES % 4096 == 0, "scratch regions are 4 KiB aligned");
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {

thread_local std::string g_create_error;

constexpr int MAX_NDIL = 4096;
constexpr int ACCURACY_MAX_SITES = 4096;  // FP32-accumulating paths: sites per split at most
constexpr int K_GENERIC = 0, K_PIPELINED = 1, K_W3 = 2, K_PORD = 3, K_W3W8 = 4, K_F64 = 5, K_F64P = 6, K_F32P = 7,
              K_F64N = 8, K_F32N = 9;
// FP64 defaults by momentum count (at 32^3, N_dil 32, ms per block): kernel
// 5 up to F64N_MIN_MOM (4 momenta: 1.28 against kernel 8's 1.41), kernel 8
// (fragments of 4) up to F64P_MIN_MOM (5 to 8 momenta: 1.67-1.70 against
// kernel 5's 2.02-2.52 and kernel 6's 2.26; 12: 2.05 against 2.26), kernel
// 6 above (16: 2.26 against kernel 8's 2.50; 27: 3.75 against kernel 5's 8.5).
constexpr int F64N_MIN_MOM = 4;
constexpr int F64P_MIN_MOM = 12;
// FP32 momenta above which the paper-order kernels are the default (at
// 32^3, N_dil 32, ms per block: kernel 1 0.93-0.94 against 1.34 up to 4
// momenta, 1.50-1.51 against 1.35 from 5 to 7; kernel 7 1.35-1.36 from 1 to
// 16 momenta, 2.5 at 27 against kernel 1's 5.9), kernel 9 (fragments of 4)
// up to F32N_MAX_MOM (5 to 8 momenta: 1.27-1.29 against kernel 7's
// 1.32; 9 to 12: 1.86 against 1.32-1.34).
constexpr int F32P_MIN_MOM = 4;
constexpr int F32N_MAX_MOM = 8;
// Kernel 2 and its eight-wave form 4 share geometry, images and workspace.
inline bool is_w3(int kernel) { return kernel == K_W3 || kernel == K_W3W8; }

struct Plan {
    int kernel = K_GENERIC, nb = 0, splits = 0, persistent = 0, grid = 0;
    // A forced plan whose split count the planner fills in: recomputed at
    // run time from the geometry of the batch's momentum set.
    bool auto_splits = false;
};

using ShapeKey = std::array<int, 4>;  // n1, n2, n3, n_mom

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
int cdiv(int a, int b) { return (a + b - 1) / b; }

// Tile geometry of one block shape under one (kernel, nb).
struct Geometry {
    int kernel = K_GENERIC, nb = 0;
    int m_tile = 0, n_tile = 0;  // complex rows / columns per tile
    int b1 = 0, b2 = 0, b3 = 0, bp = 0, n_mt2 = 1, n_nt3 = 1;  // pipelined rectangles
    int n_mt = 0, n_nt = 0;
    int lds = -1;
};

struct SubBatch {
    int first, count;       // blocks [first, first+count)
    int tile_off, n_tiles;  // into the tile table
    int list_off, n_list;   // into the reduce list
    int kernel, nb, b2, b3;
    int persistent, grid;
    int max_mn;
    int went_off, n_went;   // W-image entries (precomputed-W kernel)
    int cps_max;            // chunks per split, largest of the sub-batch
    int cg_off, n_cg;       // spin projection: output groups completed by this sub-batch
    int cgs_off;            // their start indices (n_cg + 1 entries)
};

// Device table regions of a batch.
enum TableRegion { T_BLOCKS, T_TILES, T_LIST, T_MOM, T_WENT, T_CMEM, T_CCOEF, T_CGS, T_CACC, T_COUNT };

// Device scratch of the allocation-free entry point (bblock_compute_noalloc):
// tables, phase-index table and split-K workspace of one call, laid out
//   [0, SCRATCH_TABLE)                      descriptor, tile and reduce tables
//   [SCRATCH_TABLE, + kidx bytes)           phase-index table (4 KiB aligned)
//   [then, SCRATCH_BYTES)                   split partials and W images
// Host code never uses the array's name as an address: each device's copy
// is found with hipGetSymbolAddress once, at create, with that device
// current.
constexpr size_t SCRATCH_TABLE = (size_t)1 << 20;
constexpr int SCRATCH_MAX_DEVICES = 64;

std::mutex g_scratch_mu;
unsigned char *g_scratch_addr[SCRATCH_MAX_DEVICES] = {};

// Address of the scratch array on device dev (current), looked up once.
hipError_t scratch_address(int dev, unsigned char **out)
{
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[dev] = static_cast<unsigned char *>(ptr);
    }
    *out = g_scratch_addr[dev];
    return hipSuccess;
}

// Device memory one batch runs in: the handle's allocations, or regions of
// the static scratch array.
struct Mem {
    unsigned char *table;
    void *ws;
    unsigned char *kidx;
};

}  // namespace

struct bblock_s {
    int device = 0;
    int L = 0, V = 0;
    int prec = 0, in_dtype = 0, max_ndil = 0;
    size_t ws_cap = 0;
    size_t ws_eff = 0;                // workspace cap of the batch being planned
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    int num_cu = 256;
    int n_xcd = 8, cu_per_xcd = 32;  // gfx950: 32 CUs per XCD
    int lds_max = 160 * 1024;

    double *d_roots = nullptr;  // [L] complex128
    int *d_counter = nullptr;   // [2]
    unsigned char *d_table = nullptr;  // blocks | tiles | list | momenta
    size_t table_cap = 0;
    unsigned char *h_staging = nullptr;  // pinned mirror of d_table
    hipEvent_t staging_free = nullptr;
    void *d_ws = nullptr;
    size_t ws_size = 0;
    unsigned char *d_kidx = nullptr;  // [n_mom][V] phase index of the cached momentum set
    size_t kidx_cap = 0;
    std::vector<int> kidx_mom;        // momentum set (reduced mod L) the table holds
    // Allocation-free entry point: this device's static scratch array (its
    // device address, looked up at create) and a pinned staging buffer for
    // its tables, allocated at create.
    unsigned char *scratch = nullptr;
    unsigned char *h_static = nullptr;
    hipEvent_t static_free = nullptr;

    int graph_mode = 2;               // 0: eager, 1: capture and replay, 2: replay schedules of 4+ launches
    int walk_mode = 2;                // walking tiles: 0 never, 1 every unprojected batch, 2 when the partials do not fit
    int p_skip = -1;                  // zero momentum the paper-order FP64/FP32 kernels sum on the vector unit (-1: none)
    bool profiling = false;
    int plan_gen = 0;                 // bumped whenever forced or tuned plans change
    // The last batch: when a call repeats it (same descriptors, momenta and
    // plans) the device tables are already in place and only the launch (or
    // graph replay) is issued.
    std::vector<unsigned char> last_key;
    std::vector<SubBatch> last_subs;
    size_t last_offs[T_COUNT] = {};  // device table regions of the last batch
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::array<hipEvent_t, 2>> ev_gemm, ev_reduce, ev_prep;
    std::map<std::vector<long long>, hipGraphExec_t> graphs;
    std::map<ShapeKey, Plan> forced, tuned;
    std::string err;
};

namespace {

bblock_status fail(bblock_t h, bblock_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h)
        h->err = buf;
    else
        g_create_error = buf;
    return st;
}

bblock_status hip_fail(bblock_t h, hipError_t e, const char *what)
{
    return fail(h, BBLOCK_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_OR_FAIL(h, call)                                       \
    do {                                                           \
        hipError_t e_ = (call);                                    \
        if (e_ != hipSuccess) return hip_fail((h), e_, #call);     \
    } while (0)

int part_bytes(int prec) { return prec == FP64 ? 8 : 4; }
int in_bytes(int dtype) { return dtype == BBLOCK_C64 ? 8 : 16; }

void clear_graphs(bblock_t h)
{
    for (auto &kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    h->graphs.clear();
    h->last_key.clear();  // a repeated batch must re-plan (workspace or tables moved)
}

int pipelined_block(int n) { return n >= 32 ? 32 : (n >= 16 ? 16 : 0); }

// d2 block of the pipelined kernels (a template size, 16 or 32): the one that
// pads fewer rows, 32 on a tie; 0 below 16.
int row_block(int n)
{
    if (n < 16) return 0;
    return cdiv(n, 32) * 32 <= cdiv(n, 16) * 16 ? 32 : 16;
}

// d2 block of the precomputed-W kernel (8, 16 or 32): the one that pads
// fewer rows, the larger on a tie; 0 below 8.
int w3_row_block(int n)
{
    if (n < 8) return 0;
    int best = 0;
    for (int b : {32, 16, 8})
        if (best == 0 || cdiv(n, b) * b < cdiv(n, best) * best) best = b;
    return best;
}

// d3 block of the precomputed-W kernel.  Its columns (momentum, d3) are
// packed densely into the n-tile and only the W images and the epilogue read
// the split, so any block in [16, 32] works: the balanced one,
// ceil(n3 / ceil(n3 / 32)), pads no d3 column; 0 below 16.
int w3_col_block(int n)
{
    if (n < 16) return 0;
    return cdiv(n, cdiv(n, 32));
}

// The zero momentum the paper-order FP64/FP32 kernels take off the matrix
// cores: the first momentum that is zero mod L, in a set of 16 k + 1 > 1
// momenta (where dropping one saves a padded column fragment); -1 otherwise.
int zero_momentum_column(const int32_t *mom, int n_mom, int L)
{
    if (n_mom < 2 || n_mom % 16 != 1) return -1;
    for (int i = 0; i < n_mom; ++i)
        if (mom[3 * i] % L == 0 && mom[3 * i + 1] % L == 0 && mom[3 * i + 2] % L == 0) return i;
    return -1;
}

// Kernel 3 sums the zero momentum on the vector unit for 32 k + 1 momenta at
// one fragment (32 of the 33 of the paper's shell: one fragment, not two).
bool pord_skips(bblock_t h, int nb, int n_mom) { return h->p_skip >= 0 && nb == 1 && n_mom % 32 == 1; }

// Geometry of (kernel, nb) for one block shape; lds < 0 when unsupported.
Geometry geometry(bblock_t h, int kernel, int nb, int n1, int n2, int n3, int n_mom)
{
    Geometry g;
    g.kernel = kernel;
    g.nb = nb;
    // Momentum columns of the paper-order FP64/FP32 kernels: all but a zero
    // momentum they sum on the vector unit (kernel 3 too, where that saves
    // its second fragment of 32).
    const int mcols = n_mom - (h->p_skip >= 0 ? 1 : 0);
    const int pcols = pord_skips(h, nb, n_mom) ? n_mom - 1 : n_mom;
    if (kernel == K_PIPELINED || is_w3(kernel)) {
        g.b2 = is_w3(kernel) ? w3_row_block(n2) : row_block(n2);
        g.b3 = is_w3(kernel) ? w3_col_block(n3) : pipelined_block(n3);
        const bool nb_ok = is_w3(kernel) ? (nb >= 4 && nb <= 7) : (nb == 4 || nb == 7);
        if (h->prec == FP64 || g.b2 == 0 || g.b3 == 0 || !nb_ok) return g;
        if (is_w3(kernel) && h->prec != BF16X3) return g;
        g.b1 = 128 / g.b2;
        g.m_tile = 128;
        g.n_tile = 32 * nb;
        g.bp = std::min(n_mom, g.n_tile / g.b3);
        g.n_mt2 = cdiv(n2, g.b2);
        g.n_nt3 = cdiv(n3, g.b3);
        g.n_mt = cdiv(n1, g.b1) * g.n_mt2;
        g.n_nt = cdiv(n_mom, g.bp) * g.n_nt3;
        g.lds = is_w3(kernel) ? w3_lds_bytes(nb, g.b2) : fast_lds_bytes(h->prec, nb, g.b2, g.b3, h->L);
    } else if (kernel == K_F64) {
        // Linear row tiles of 128 (d1,d2) pairs, linear column tiles of 16 nb
        // (p,d3) pairs; FP64 only.
        if (h->prec != FP64) return g;
        const int lds = f64_lds_bytes(nb);
        if (lds <= 0) return g;
        g.m_tile = 128;
        g.n_tile = 16 * nb;
        g.n_mt = cdiv(n1 * n2, g.m_tile);
        g.n_nt = cdiv(n3 * n_mom, g.n_tile);
        g.lds = lds;
    } else if (kernel == K_F64P) {
        // Rows (d1,d2,d3): a block of consecutive (d1,d2) pairs x a d3 block
        // of 16, two row sets per wave up to nb 2 (one wave reads q3 for
        // two pairs: 4-7 % faster at 32^3, N_dil 32, 16 to 33 momenta, than
        // one row set with the d3 block of 32 or 16); columns: 16 nb momenta.
        g.b3 = n3 < 16 ? 0 : 16;
        if (h->prec != FP64 || g.b3 == 0) return g;
        const int pairs = f64p_pairs(nb, g.b3, 16), lds = f64p_lds_bytes(nb, g.b3, 16);
        if (pairs <= 0 || lds <= 0) return g;
        g.m_tile = pairs * g.b3;
        g.n_tile = 16 * nb;
        g.bp = 16 * nb;
        g.n_mt2 = cdiv(n3, g.b3);  // d3 blocks
        g.n_mt = cdiv(n1 * n2, pairs) * g.n_mt2;
        g.n_nt = cdiv(mcols, g.n_tile);
        g.lds = lds;
    } else if (kernel == K_F64N) {
        // Kernel 6 with fragments of 4 momenta (nb 1 to 4), d3 blocks of 16.
        g.b3 = n3 < 16 ? 0 : 16;
        if (h->prec != FP64 || g.b3 == 0) return g;
        const int pairs = f64p_pairs(nb, g.b3, 4), lds = f64p_lds_bytes(nb, g.b3, 4);
        if (pairs <= 0 || lds <= 0) return g;
        g.m_tile = pairs * g.b3;
        g.n_tile = 4 * nb;
        g.bp = 4 * nb;
        g.n_mt2 = cdiv(n3, g.b3);  // d3 blocks
        g.n_mt = cdiv(n1 * n2, pairs) * g.n_mt2;
        g.n_nt = cdiv(n_mom, g.n_tile);
        g.lds = lds;
    } else if (kernel == K_F32N) {
        // Kernel 7 with fragments of 4 momenta (nb 1 to 4), d3 blocks of 16.
        g.b3 = n3 < 16 ? 0 : 16;
        if (h->prec != FP32 || g.b3 == 0) return g;
        const int pairs = f32p_pairs(g.b3), lds = f32p_lds_bytes(nb, g.b3, 4);
        if (pairs <= 0 || lds <= 0) return g;
        g.m_tile = pairs * g.b3;
        g.n_tile = 4 * nb;
        g.bp = 4 * nb;
        g.n_mt2 = cdiv(n3, g.b3);  // d3 blocks
        g.n_mt = cdiv(n1 * n2, pairs) * g.n_mt2;
        g.n_nt = cdiv(n_mom, g.n_tile);
        g.lds = lds;
    } else if (kernel == K_F32P) {
        // As kernel 6, in FP32, 16 nb momenta: d3 blocks of 16 up to two
        // momentum fragments (two workgroups then share a CU), else 32
        // (16 below 32).
        g.b3 = n3 < 16 ? 0 : (nb <= 2 || n3 < 32 ? 16 : 32);
        if (h->prec != FP32 || g.b3 == 0) return g;
        const int pairs = f32p_pairs(g.b3), lds = f32p_lds_bytes(nb, g.b3, 16);
        if (pairs <= 0 || lds <= 0) return g;
        g.m_tile = pairs * g.b3;
        g.n_tile = 16 * nb;
        g.bp = 16 * nb;
        g.n_mt2 = cdiv(n3, g.b3);  // d3 blocks
        g.n_mt = cdiv(n1 * n2, pairs) * g.n_mt2;
        g.n_nt = cdiv(mcols, g.n_tile);
        g.lds = lds;
    } else if (kernel == K_PORD) {
        // Rows (d1,d2,d3): a block of consecutive (d1,d2) pairs x a d3 block;
        // columns: 32 nb momenta.
        g.b3 = pipelined_block(n3);
        if (h->prec != BF16X3 || g.b3 == 0 || (nb != 1 && nb != 2)) return g;
        const int pairs = pord_pairs(nb, g.b3);
        if (pairs <= 0) return g;
        g.m_tile = pairs * g.b3;
        g.n_tile = 32 * nb;
        g.bp = 32 * nb;
        g.n_mt2 = cdiv(n3, g.b3);  // d3 blocks
        g.n_mt = cdiv(n1 * n2, pairs) * g.n_mt2;
        g.n_nt = cdiv(pcols, g.n_tile);
        g.lds = 32768;  // static, well below the limit
    } else {
        const KernelGeom k = kernel_geom(h->prec, nb, n_mom, h->L);
        if (k.lds_bytes <= 0) return g;
        g.m_tile = k.m_tile;
        g.n_tile = nb * k.frag_cols;
        g.n_mt = cdiv(n1 * n2, g.m_tile);
        g.n_nt = cdiv(n3 * n_mom, g.n_tile);
        g.lds = k.lds_bytes;
    }
    if (g.lds > h->lds_max) g.lds = -1;
    return g;
}

// Workgroups of a plan that fit one CU at once: two for the paper-order
// kernel and for the FP64 generic kernel up to 7 column fragments (registers
// and LDS allow it, and one workgroup's D/W generation then runs beside the
// other's MFMAs), one otherwise.
int wg_per_cu(bblock_t h, const Geometry &g)
{
    if (g.kernel == K_PORD) return 2;
    if (g.kernel == K_F32P) return f32p_wgs(g.nb, g.b3, 16);
    if (g.kernel == K_F32N) return f32p_wgs(g.nb, g.b3, 4);
    if (g.kernel == K_GENERIC && h->prec == FP64 && g.nb <= 7 && 2 * g.lds <= h->lds_max) return 2;
    return 1;
}

// Splits that fill the device with whole waves of workgroups: up to the
// workgroups the CUs hold at once, the most that keep tiles x splits within
// them (rounding up would leave a second, nearly empty wave that doubles the
// time).
int fill_splits(bblock_t h, const Geometry &g)
{
    const long slots = (long)h->num_cu * wg_per_cu(h, g);
    const long tiles = std::max(1L, (long)g.n_mt * g.n_nt);
    if (tiles <= slots) return (int)(slots / tiles);
    // More tiles than the CUs hold at once: a last, partly filled wave is
    // unavoidable, so take the split count (up to 8) whose waves leave the
    // fewest slots idle, one point of efficiency charged per extra split
    // for its partials (at 32^3, N_dil 40, 7 momenta, FP64: 300 tiles, one
    // split fills 59 % of two waves, five fill 98 % of six).
    int best = 1;
    double best_score = -1.0;
    for (int s = 1; s <= 8; ++s) {
        const long work = tiles * s, waves = (work + slots - 1) / slots;
        const double score = (double)work / (double)(waves * slots) - 0.01 * (s - 1);
        if (score > best_score + 1e-9) {
            best_score = score;
            best = s;
        }
    }
    return best;
}

// Default plan of one block shape: the pipelined kernel where it applies
// (fewest padded columns, then the wider tile), else the generic kernel with
// the N tile covering the columns in as few tiles as possible; the split
// count fills the device for a single block.
Plan default_plan(bblock_t h, int n1, int n2, int n3, int n_mom)
{
    Plan p;
    Geometry best;
    // BF16X3 with many momenta: the paper-order kernel (its MFMA work per
    // (site, row) is 32 momenta per column fragment, the fused GEMM's is 24
    // flops per momentum; measured at 32^3, N_dil 32 it is the cheaper one
    // from 17 momenta on).
    if (h->prec == BF16X3 && n_mom > 16) {
        const int cols = n_mom - (h->p_skip >= 0 && n_mom % 32 == 1 ? 1 : 0);
        const Geometry g = geometry(h, K_PORD, cols > 32 ? 2 : 1, n1, n2, n3, n_mom);
        if (g.lds > 0) {
            p.kernel = K_PORD;
            p.nb = g.nb;
            p.splits = fill_splits(h, g);
            return p;
        }
    }
    if (h->prec == FP32 && n_mom > F32P_MIN_MOM && n_mom <= F32N_MAX_MOM) {
        // FP32 with a few momenta: kernel 9, fragments of 4.
        const Geometry g = geometry(h, K_F32N, cdiv(n_mom, 4), n1, n2, n3, n_mom);
        if (g.lds > 0) {
            p.kernel = K_F32N;
            p.nb = g.nb;
            p.splits = fill_splits(h, g);
            return p;
        }
    }
    if (h->prec == FP32 && n_mom > F32P_MIN_MOM) {
        // FP32 with many momenta: the paper-order kernel 7, with the column
        // width that pads fewest momenta (the wider on a tie).
        for (int nb : {4, 3, 2, 1}) {
            const Geometry g = geometry(h, K_F32P, nb, n1, n2, n3, n_mom);
            if (g.lds < 0) continue;
            if (best.lds < 0 || (long)g.n_nt * g.n_tile < (long)best.n_nt * best.n_tile) best = g;
        }
        if (best.lds >= 0) {
            p.kernel = best.kernel;
            p.nb = best.nb;
            p.splits = fill_splits(h, best);
            return p;
        }
    }
    if (h->prec == FP64 && n_mom > F64N_MIN_MOM && n_mom <= F64P_MIN_MOM) {
        // FP64 with a few momenta: the paper-order kernel 8, fragments of 4.
        const Geometry g = geometry(h, K_F64N, cdiv(n_mom, 4), n1, n2, n3, n_mom);
        if (g.lds > 0) {
            p.kernel = K_F64N;
            p.nb = g.nb;
            p.splits = fill_splits(h, g);
            return p;
        }
    }
    if (h->prec == FP64 && n_mom > F64P_MIN_MOM) {
        // FP64 with many momenta: the paper-order kernel 6, with the column
        // width that pads fewest momenta (the wider on a tie).
        for (int nb : {3, 2, 1}) {
            const Geometry g = geometry(h, K_F64P, nb, n1, n2, n3, n_mom);
            if (g.lds < 0) continue;
            if (best.lds < 0 || (long)g.n_nt * g.n_tile < (long)best.n_nt * best.n_tile) best = g;
        }
        if (best.lds >= 0) {
            p.kernel = best.kernel;
            p.nb = best.nb;
            p.splits = fill_splits(h, best);
            return p;
        }
    }
    if (h->prec == FP64) {
        // FP64 kernel 5: the column width that pads fewest columns (the
        // wider on a tie).
        for (int nb : {7, 4, 2}) {
            const Geometry g = geometry(h, K_F64, nb, n1, n2, n3, n_mom);
            if (g.lds < 0) continue;
            if (best.lds < 0 || (long)g.n_nt * g.n_tile < (long)best.n_nt * best.n_tile) best = g;
        }
        if (best.lds >= 0) {
            p.kernel = best.kernel;
            p.nb = best.nb;
            p.splits = fill_splits(h, best);
            return p;
        }
    }
    const int tiled = h->prec == BF16X3 ? K_W3W8 : K_PIPELINED;
    for (int nb : {7, 6, 5, 4}) {
        const Geometry g = geometry(h, tiled, nb, n1, n2, n3, n_mom);
        if (g.lds < 0) continue;
        if (best.lds < 0 || (long)g.n_nt * g.n_tile < (long)best.n_nt * best.n_tile) best = g;
    }
    if (best.lds < 0) {
        const int *opts;
        const int n_opts = nb_options(h->prec, &opts);
        const int frag = kernel_geom(h->prec, opts[0], n_mom, h->L).frag_cols;
        // FP64: at most 7 fragments, so that two workgroups share a CU.
        const int N = n3 * n_mom, max_nb = h->prec == FP64 ? std::min(7, opts[n_opts - 1]) : opts[n_opts - 1];
        const int n_nt = cdiv(N, max_nb * frag);
        const int want_nb = cdiv(N, n_nt * frag);
        for (int i = n_opts - 1; i >= 0; --i) {
            const Geometry g = geometry(h, K_GENERIC, opts[i], n1, n2, n3, n_mom);
            if (g.lds < 0) continue;
            if (best.lds < 0 || opts[i] >= want_nb) best = g;
        }
    }
    p.kernel = best.kernel;
    p.nb = best.nb;
    p.splits = fill_splits(h, best);
    return p;
}

Plan plan_for(bblock_t h, int n1, int n2, int n3, int n_mom)
{
    const ShapeKey k{n1, n2, n3, n_mom};
    auto f = h->forced.find(k);
    if (f != h->forced.end()) return f->second;
    auto t = h->tuned.find(k);
    if (t != h->tuned.end()) return t->second;
    return default_plan(h, n1, n2, n3, n_mom);
}

int min_splits(bblock_t h)
{
    if (h->prec == FP64) return 1;
    return (h->V + ACCURACY_MAX_SITES - 1) / ACCURACY_MAX_SITES;
}

// Split count of a single block from its plan's count: at least s_min, and
// raised in whole multiples of the plan's count, which fills one wave of
// workgroups (rounding up to s_min alone can leave a second wave with a few
// workgroups: 36 tiles x 8 splits = 288 workgroups on 256 CUs take the time
// of two full waves at N_dil = 48).
int single_splits(int plan_splits, int s_min)
{
    if (plan_splits >= s_min) return plan_splits;
    return cdiv(s_min, plan_splits) * plan_splits;
}

struct BlockPlan {
    BlockDesc d;
    Plan plan;
    Geometry g;
    size_t part_bytes;  // split-K partials
    size_t ws_bytes;    // partials, then (precomputed-W kernel) the W images of one round
    int rounds = 1;     // precomputed-W kernel: rounds of spr splits each
    int spr = 0;
    bool need_part = false;  // partials even for one split (spin projection)
    bool walk = false;       // the tile's workgroup runs all splits in order (no partials)
};

// Sites per split for S splits: a multiple of CHUNK_SITES; the split count
// actually used is ceil(V / sps).
// Tile-decoding fields of a block's descriptor from its plan's geometry
// (again whenever the plan falls back to another kernel).
void take_geometry(BlockPlan &bp)
{
    bp.d.n_mt2 = bp.g.n_mt2;
    bp.d.n_nt3 = bp.g.n_nt3;
    bp.d.bp = bp.g.bp;
    bp.d.b3 = bp.g.b3;
}

void set_splits(bblock_t h, BlockPlan &bp, int S)
{
    S = std::max(1, std::min(S, (h->V + CHUNK_SITES - 1) / CHUNK_SITES));
    const int sps = (int)align_up((size_t)((h->V + S - 1) / S), CHUNK_SITES);
    bp.d.sps = sps;
    bp.d.S = (h->V + sps - 1) / sps;
    bp.d.cps = sps / CHUNK_SITES;
    bp.d.n_nt = bp.g.n_nt;
    const bool parts = (bp.d.S > 1 || bp.need_part) && !bp.walk;
    bp.part_bytes = parts ? (size_t)bp.d.S * 2 * bp.d.M * bp.d.N * part_bytes(h->prec) : 0;
    bp.d.direct = !parts && bp.d.S == 1;
    bp.d.walk = !parts && bp.d.S > 1;
    bp.ws_bytes = bp.part_bytes;
    bp.rounds = 1;
    bp.spr = bp.d.S;
    if (is_w3(bp.plan.kernel)) {
        // W images of all splits if they fit beside the partials, else rounds
        // of as many splits as fit (at least one; 0 = does not fit).
        const size_t per_split = (size_t)bp.g.n_nt * bp.d.cps * w3_image_bytes(bp.plan.nb);
        const size_t part = align_up(bp.part_bytes, 4096);
        const size_t room = h->ws_eff > part ? h->ws_eff - part : 0;
        bp.spr = (int)std::min<size_t>(bp.d.S, room / per_split);
        bp.rounds = bp.spr > 0 ? (bp.d.S + bp.spr - 1) / bp.spr : 1;
        bp.ws_bytes = part + (size_t)std::max(bp.spr, 1) * per_split;
    }
}

// The precomputed-W kernel addresses one split of q1/q2 with 32-bit byte
// offsets (plus three chunks of read-ahead).
bool w3_offsets_fit(bblock_t h, const BlockPlan &bp)
{
    const size_t per_site = (size_t)3 * std::max({bp.d.n1, bp.d.n2, bp.d.n3}) * in_bytes(h->in_dtype);
    return (size_t)(bp.d.sps + 4 * CHUNK_SITES) * per_site < ((size_t)1 << 31);
}

bblock_status validate_desc(bblock_t h, const bblock_desc &d, int i)
{
    if (!d.q1 || !d.q2 || !d.q3 || !d.out) return fail(h, BBLOCK_EINVAL, "desc %d: null pointer", i);
    const uintptr_t al = (uintptr_t)d.q1 | (uintptr_t)d.q2 | (uintptr_t)d.q3 | (uintptr_t)d.out;
    if (al % 16) return fail(h, BBLOCK_EINVAL, "desc %d: buffers must be 16-byte aligned", i);
    if (d.n1 < 1 || d.n2 < 1 || d.n3 < 1 || d.n1 > h->max_ndil || d.n2 > h->max_ndil || d.n3 > h->max_ndil)
        return fail(h, BBLOCK_EINVAL, "desc %d: dilution sizes (%d,%d,%d) outside [1,%d]", i, d.n1, d.n2, d.n3,
                    h->max_ndil);
    return BBLOCK_OK;
}

bblock_status ensure_table(bblock_t h, size_t bytes)
{
    if (bytes <= h->table_cap) return BBLOCK_OK;
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    clear_graphs(h);  // captured kernels point into the old table
    h->last_key.clear();
    if (h->d_table) (void)hipFree(h->d_table);
    if (h->h_staging) (void)hipHostFree(h->h_staging);
    h->d_table = nullptr;
    h->h_staging = nullptr;
    h->table_cap = 0;
    const size_t cap = align_up(bytes + bytes / 2, 1 << 16);
    if (hipMalloc(&h->d_table, cap) != hipSuccess) return fail(h, BBLOCK_ENOMEM, "table allocation of %zu bytes", cap);
    if (hipHostMalloc(&h->h_staging, cap, hipHostMallocDefault) != hipSuccess)
        return fail(h, BBLOCK_ENOMEM, "pinned staging allocation of %zu bytes", cap);
    h->table_cap = cap;
    return BBLOCK_OK;
}

bblock_status ensure_ws(bblock_t h, size_t bytes)
{
    if (bytes <= h->ws_size) return BBLOCK_OK;
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    clear_graphs(h);
    if (h->d_ws) (void)hipFree(h->d_ws);
    h->d_ws = nullptr;
    h->ws_size = 0;
    if (hipMalloc(&h->d_ws, bytes) != hipSuccess) return fail(h, BBLOCK_ENOMEM, "workspace allocation of %zu bytes", bytes);
    h->ws_size = bytes;
    return BBLOCK_OK;
}

int kstride_of(bblock_t h) { return (h->V + 3) & ~3; }

// Phase-index table kidx[p][x] = (n_p . x) mod L of one momentum set, built on
// the device when the set changes (reused across calls, paper Sec. 3).
// d_mom: the reduced momenta already uploaded to the device.
bblock_status ensure_kidx(bblock_t h, const std::vector<int> &mom_red, const int *d_mom)
{
    if (mom_red == h->kidx_mom && h->d_kidx) return BBLOCK_OK;
    const int n_mom = (int)mom_red.size() / 3;
    const size_t bytes = (size_t)n_mom * kstride_of(h);
    if (bytes > h->kidx_cap) {
        HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
        clear_graphs(h);
        if (h->d_kidx) (void)hipFree(h->d_kidx);
        h->d_kidx = nullptr;
        h->kidx_cap = 0;
        if (hipMalloc(&h->d_kidx, bytes) != hipSuccess)
            return fail(h, BBLOCK_ENOMEM, "phase table allocation of %zu bytes", bytes);
        h->kidx_cap = bytes;
    }
    const hipError_t e = launch_phase_index(d_mom, n_mom, h->L, kstride_of(h), h->d_kidx, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "launch of the phase-index kernel");
    h->kidx_mom = mom_red;
    return BBLOCK_OK;
}

hipEvent_t take_event(bblock_t h)
{
    if (!h->ev_pool.empty()) {
        hipEvent_t e = h->ev_pool.back();
        h->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch the kernels of all sub-batches on stream st; tables already uploaded.
bblock_status enqueue(bblock_t h, const Mem &mem, const std::vector<SubBatch> &subs, const size_t *offs, int n_mom,
                      hipStream_t st)
{
    const size_t off_blocks = offs[T_BLOCKS], off_tiles = offs[T_TILES], off_list = offs[T_LIST];
    const size_t off_mom = offs[T_MOM], off_went = offs[T_WENT];
    for (const SubBatch &sb : subs) {
        GemmArgs ga;
        ga.blocks = reinterpret_cast<const BlockDesc *>(mem.table + off_blocks);
        ga.tiles = reinterpret_cast<const int4 *>(mem.table + off_tiles) + sb.tile_off;
        ga.n_tiles = sb.n_tiles;
        ga.counter = sb.persistent ? h->d_counter : nullptr;
        ga.mom = reinterpret_cast<const int *>(mem.table + off_mom);
        ga.n_mom = n_mom;
        ga.L = h->L;
        ga.V = h->V;
        ga.in_c64 = h->in_dtype == BBLOCK_C64;
        ga.roots = h->d_roots;
        ga.kidx = mem.kidx;
        ga.kstride = kstride_of(h);
        ga.p_skip = sb.kernel == K_F64P || sb.kernel == K_F32P || (sb.kernel == K_PORD && pord_skips(h, sb.nb, n_mom))
                        ? h->p_skip
                        : -1;
        const int grid = sb.persistent ? std::min(sb.grid, sb.n_tiles) : sb.n_tiles;
        std::array<hipEvent_t, 2> ev{nullptr, nullptr};
        if (is_w3(sb.kernel)) {
            WImageArgs wa;
            wa.blocks = ga.blocks;
            wa.entries = reinterpret_cast<const int4 *>(mem.table + off_went) + sb.went_off;
            wa.n_entries = sb.n_went;
            wa.mom = ga.mom;
            wa.n_mom = n_mom;
            wa.L = h->L;
            wa.V = h->V;
            wa.roots = h->d_roots;
            if (h->profiling) {
                ev = {take_event(h), take_event(h)};
                if (!ev[0] || !ev[1]) return fail(h, BBLOCK_EHIP, "profiling event creation failed");
                HIP_OR_FAIL(h, hipEventRecord(ev[0], st));
            }
            hipError_t e = launch_w3_image(sb.nb, ga.in_c64, wa, sb.cps_max, st);
            if (e != hipSuccess) return hip_fail(h, e, "launch of the W-image kernel");
            if (h->profiling) {
                HIP_OR_FAIL(h, hipEventRecord(ev[1], st));
                h->ev_prep.push_back(ev);
            }
        }
        if (h->profiling) {
            ev = {take_event(h), take_event(h)};
            if (!ev[0] || !ev[1]) return fail(h, BBLOCK_EHIP, "profiling event creation failed");
            HIP_OR_FAIL(h, hipEventRecord(ev[0], st));
        }
        hipError_t e = sb.kernel == K_PIPELINED ? launch_fast(h->prec, sb.nb, sb.b2, sb.b3, ga.in_c64, ga, grid, st)
                       : is_w3(sb.kernel)       ? launch_w3(sb.nb, sb.b2, sb.kernel == K_W3W8 ? 8 : 4, ga.in_c64, ga,
                                                            grid, st)
                       : sb.kernel == K_PORD    ? launch_pord(sb.nb, sb.b3, ga.in_c64, ga, grid, st)
                       : sb.kernel == K_F64     ? launch_f64(sb.nb, ga.in_c64, ga, grid, st)
                       : sb.kernel == K_F64P    ? launch_f64p(sb.nb, sb.b3, ga.in_c64, ga, grid, st)
                       : sb.kernel == K_F64N    ? launch_f64n(sb.nb, sb.b3, ga.in_c64, ga, grid, st)
                       : sb.kernel == K_F32P    ? launch_f32p(sb.nb, sb.b3, ga.in_c64, ga, grid, st)
                       : sb.kernel == K_F32N    ? launch_f32n(sb.nb, ga.in_c64, ga, grid, st)
                                                : launch_gemm(h->prec, sb.nb, ga, grid, st);
        if (e != hipSuccess) return hip_fail(h, e, "launch of the contraction kernel");
        if (h->profiling) {
            HIP_OR_FAIL(h, hipEventRecord(ev[1], st));
            h->ev_gemm.push_back(ev);
        }
        if (sb.n_cg > 0) {
            CombineArgs ca;
            ca.blocks = ga.blocks;
            ca.list = reinterpret_cast<const int *>(mem.table + offs[T_CMEM]);
            ca.coef = reinterpret_cast<const double *>(mem.table + offs[T_CCOEF]);
            ca.gstart = reinterpret_cast<const int *>(mem.table + offs[T_CGS]) + sb.cgs_off;
            ca.accumulate = reinterpret_cast<const int *>(mem.table + offs[T_CACC]) + sb.cg_off;
            ca.n_groups = sb.n_cg;
            if (h->profiling) {
                ev = {take_event(h), take_event(h)};
                if (!ev[0] || !ev[1]) return fail(h, BBLOCK_EHIP, "profiling event creation failed");
                HIP_OR_FAIL(h, hipEventRecord(ev[0], st));
            }
            e = launch_combine(h->prec, ca, sb.max_mn, st);
            if (e != hipSuccess) return hip_fail(h, e, "launch of the spin-projection combination");
            if (h->profiling) {
                HIP_OR_FAIL(h, hipEventRecord(ev[1], st));
                h->ev_reduce.push_back(ev);
            }
        }
        if (sb.n_list > 0) {
            ReduceArgs ra;
            ra.blocks = ga.blocks;
            ra.list = reinterpret_cast<const int *>(mem.table + off_list) + sb.list_off;
            ra.n_list = sb.n_list;
            if (h->profiling) {
                ev = {take_event(h), take_event(h)};
                if (!ev[0] || !ev[1]) return fail(h, BBLOCK_EHIP, "profiling event creation failed");
                HIP_OR_FAIL(h, hipEventRecord(ev[0], st));
            }
            e = launch_reduce(h->prec, ra, sb.max_mn, st);
            if (e != hipSuccess) return hip_fail(h, e, "launch of the split-K reduction");
            if (h->profiling) {
                HIP_OR_FAIL(h, hipEventRecord(ev[1], st));
                h->ev_reduce.push_back(ev);
            }
        }
    }
    return BBLOCK_OK;
}

// Launch a planned batch whose tables are on the device: eagerly, or by
// replaying (capturing on first use) the graph of this batch structure.
bblock_status launch_planned(bblock_t h, const Mem &mem, const std::vector<SubBatch> &subs, const size_t *offs,
                             int n_mom, bool eager)
{
    if (eager || h->graph_mode == 0 || h->profiling) return enqueue(h, mem, subs, offs, n_mom, h->stream);
    if (h->graph_mode == 2) {
        // A replayed graph separates its kernels by more idle time than eager
        // launches on one stream (≈1 % of a single-block call); it pays only
        // when it saves many launches.
        int launches = 0;
        for (const SubBatch &sb : subs)
            launches += 1 + is_w3(sb.kernel) + (sb.n_cg > 0) + (sb.n_list > 0);
        if (launches < 4) return enqueue(h, mem, subs, offs, n_mom, h->stream);
    }
    // Graph signature: everything baked into kernel arguments.
    std::vector<long long> sig;
    sig.push_back(n_mom);
    sig.push_back((long long)(uintptr_t)h->d_table);
    sig.push_back((long long)(uintptr_t)h->d_kidx);
    sig.push_back((long long)(uintptr_t)h->d_ws);
    for (int k = 0; k < T_COUNT; ++k) sig.push_back((long long)offs[k]);
    sig.push_back(h->p_skip);
    for (const SubBatch &sb : subs)
        sig.insert(sig.end(), {sb.first, sb.count, sb.tile_off, sb.n_tiles, sb.list_off, sb.n_list, sb.kernel, sb.nb,
                               sb.b2, sb.b3, sb.persistent, sb.grid, sb.max_mn, sb.went_off, sb.n_went, sb.cps_max,
                               sb.cg_off, sb.n_cg, sb.cgs_off});
    auto it = h->graphs.find(sig);
    if (it == h->graphs.end()) {
        HIP_OR_FAIL(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
        bblock_status st = enqueue(h, mem, subs, offs, n_mom, h->cap_stream);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(h->cap_stream, &graph);
        if (st != BBLOCK_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return hip_fail(h, e, "hipStreamEndCapture");
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(h, e, "hipGraphInstantiate");
        if (h->graphs.size() > 64) clear_graphs(h);
        it = h->graphs.emplace(sig, exec).first;
    }
    HIP_OR_FAIL(h, hipGraphLaunch(it->second, h->stream));
    return BBLOCK_OK;
}

// coef == nullptr: every descriptor's block is written to its out.  Else
// (spin projection) descriptors sharing an out pointer form one output group
// and out = sum of coef_i * B_i over the group.
//
// noalloc: the allocation-free form.  Tables, phase-index table and
// workspace live in the device's static scratch array instead of the
// handle's allocations, the tables go up through the pinned buffer
// allocated at create, launches are eager (a graph instantiation
// allocates), and nothing is cached across calls (the scratch array is
// shared by every call on the device).
bblock_status run_batch(bblock_t h, const bblock_desc *desc, int n_desc, const int32_t *mom, int n_mom,
                        const double *coef = nullptr, bool noalloc = false)
{
    if (!h) return fail(h, BBLOCK_EINVAL, "null handle");
    if (!desc || n_desc < 1) return fail(h, BBLOCK_EINVAL, "empty batch");
    if (n_desc > 65535) return fail(h, BBLOCK_EINVAL, "at most 65535 blocks per batch");
    if (!mom || n_mom < 1 || n_mom > MAX_MOM) return fail(h, BBLOCK_EINVAL, "n_mom must be in [1,%d]", MAX_MOM);
    for (int i = 0; i < n_desc; ++i) {
        bblock_status st = validate_desc(h, desc[i], i);
        if (st != BBLOCK_OK) return st;
    }

    // A set of 16 k + 1 momenta that holds the zero momentum: the paper-order
    // FP64/FP32 kernels project on the other 16 k in k momentum fragments and
    // sum the sites for the zero momentum (phase 1) on the vector unit.
    h->p_skip = zero_momentum_column(mom, n_mom, h->L);

    // Spin projection: output groups by out pointer, in order of first use.
    std::vector<int> group_of(n_desc, -1);
    int n_groups = 0;
    if (coef) {
        std::map<void *, int> gid;    // out pointer -> group
        std::vector<int> first;       // group -> its first descriptor
        for (int i = 0; i < n_desc; ++i) {
            auto it = gid.find(desc[i].out);
            if (it == gid.end()) {
                gid.emplace(desc[i].out, n_groups);
                first.push_back(i);
                group_of[i] = n_groups++;
            } else {
                const bblock_desc &f = desc[first[it->second]];
                if (f.n1 != desc[i].n1 || f.n2 != desc[i].n2 || f.n3 != desc[i].n3)
                    return fail(h, BBLOCK_EINVAL, "desc %d: blocks summed into one output must have one shape", i);
                group_of[i] = it->second;
            }
            if (!std::isfinite(coef[2 * i]) || !std::isfinite(coef[2 * i + 1]))
                return fail(h, BBLOCK_EINVAL, "desc %d: coefficient is not finite", i);
        }
    }
    // A repeat of the previous batch reuses its device tables and schedule.
    const size_t coef_bytes = coef ? sizeof(double) * 2 * n_desc : 0;
    std::vector<unsigned char> key(sizeof(bblock_desc) * n_desc + sizeof(int32_t) * 3 * n_mom + coef_bytes +
                                   4 * sizeof(int));
    {
        unsigned char *kp = key.data();
        std::memcpy(kp, desc, sizeof(bblock_desc) * n_desc);
        kp += sizeof(bblock_desc) * n_desc;
        std::memcpy(kp, mom, sizeof(int32_t) * 3 * n_mom);
        kp += sizeof(int32_t) * 3 * n_mom;
        if (coef) std::memcpy(kp, coef, coef_bytes);
        kp += coef_bytes;
        const int tail[4] = {h->plan_gen, n_mom, n_desc, coef ? 1 : 0};
        std::memcpy(kp, tail, sizeof tail);
    }
    // The allocation-free form: the phase-index table after the tables, the
    // workspace in the rest of the scratch array.
    size_t s_kidx_off = 0, s_ws_off = 0;
    if (noalloc) {
        if (!h->scratch || !h->h_static) return fail(h, BBLOCK_EHIP, "no static scratch on this device");
        s_kidx_off = SCRATCH_TABLE;
        s_ws_off = align_up(s_kidx_off + (size_t)n_mom * kstride_of(h), 4096);
        if (s_ws_off >= SCRATCH_BYTES)
            return fail(h, BBLOCK_ENOMEM, "the phase-index table of %d momenta at L=%d (%zu bytes) exceeds the static "
                        "scratch of %zu bytes", n_mom, h->L, (size_t)n_mom * kstride_of(h), SCRATCH_BYTES);
        h->ws_eff = std::min(h->ws_cap, SCRATCH_BYTES - s_ws_off);
    } else {
        if (key == h->last_key && !h->last_subs.empty())
            return launch_planned(h, Mem{h->d_table, h->d_ws, h->d_kidx}, h->last_subs, h->last_offs, n_mom, false);
        h->last_key.clear();
        h->ws_eff = h->ws_cap;
    }

    // Plans, geometry and split counts per block.
    const int s_min = min_splits(h);
    std::vector<BlockPlan> bps(n_desc);
    long total_tiles_s1 = 0;
    for (int i = 0; i < n_desc; ++i) {
        const bblock_desc &d = desc[i];
        BlockPlan &bp = bps[i];
        bp.plan = plan_for(h, d.n1, d.n2, d.n3, n_mom);
        bp.g = geometry(h, bp.plan.kernel, bp.plan.nb, d.n1, d.n2, d.n3, n_mom);
        if (bp.g.lds < 0)
            return fail(h, BBLOCK_EUNSUPPORTED, "no kernel for plan (kernel %d, nb %d) at shape (%d,%d,%d), n_mom %d",
                        bp.plan.kernel, bp.plan.nb, d.n1, d.n2, d.n3, n_mom);
        std::memset(&bp.d, 0, sizeof bp.d);
        bp.d.q1 = d.q1;
        bp.d.q2 = d.q2;
        bp.d.q3 = d.q3;
        bp.d.out = reinterpret_cast<double *>(d.out);
        bp.d.n1 = d.n1;
        bp.d.n2 = d.n2;
        bp.d.n3 = d.n3;
        bp.d.M = d.n1 * d.n2;
        bp.d.N = d.n3 * n_mom;
        take_geometry(bp);
        total_tiles_s1 += (long)bp.g.n_mt * bp.g.n_nt;
    }
    // Walking tiles (the sum over sites of Algorithm 1 kept in one
    // workgroup): the workgroup of a (block, m-tile, n-tile) runs the block's
    // splits (as few as the FP32 accumulation bound allows) in order and sums
    // them into the output in FP64.  No partials, no reduction launch, no
    // workspace beyond W images, so a batch of one kernel instantiation is
    // one launch however many blocks it holds.  They need tiles that fill
    // the device without splitting the sites, and they cost time where the
    // split schedule keeps the concurrent workgroups on one site range (the
    // paper-order kernel: 9-15 % on 48^3 and 64^3 batches), so by default a
    // batch walks only when its split partials would not fit the workspace
    // (the sub-batches that would take) and the paper-order kernel never
    // does.  Spin projection keeps the partials: the combination reads them.
    const bool walk_fill = !coef && h->walk_mode != 0 && (h->walk_mode == 1 || total_tiles_s1 >= 2L * h->num_cu);
    bool walk = false;
    auto walk_of = [&](const BlockPlan &bp) { return walk && (h->walk_mode == 1 || bp.plan.kernel != K_PORD); };
    // Split count: a forced plan fixes it; a single block uses its plan's
    // count; batches fill the device; never below the accuracy bound.
    // trial: plan without failing (the walk decision looks at the result).
    auto split_pass = [&](bool trial) -> bblock_status {
        for (int i = 0; i < n_desc; ++i) {
            BlockPlan &bp = bps[i];
            const ShapeKey k{bp.d.n1, bp.d.n2, bp.d.n3, n_mom};
            const bool fixed = h->forced.count(k) && bp.plan.splits > 0;
            int S;
            if (fixed)
                S = bp.plan.auto_splits ? single_splits(fill_splits(h, bp.g), s_min) : bp.plan.splits;
            else if (walk_of(bp))
                S = s_min;
            else if (n_desc == 1 && bp.plan.splits > 0)
                S = single_splits(bp.plan.splits, s_min);
            else
                S = std::max<int>(s_min, (int)std::max<long>(1, 2L * h->num_cu / std::max(1L, total_tiles_s1)));
            bp.need_part = coef != nullptr;
            bp.walk = walk_of(bp);
            set_splits(h, bp, S);
            if (bp.walk && is_w3(bp.plan.kernel) && bp.rounds > 1) {
                // A walking tile needs the images of all its splits at once.
                bp.walk = false;
                set_splits(h, bp, S);
            }
            if (!fixed && bp.ws_bytes > h->ws_eff) set_splits(h, bp, s_min);
            if (is_w3(bp.plan.kernel) && (bp.ws_bytes > h->ws_eff || !w3_offsets_fit(h, bp))) {
                // Not even one split's W images fit beside the partials (or the
                // split is too long for 32-bit offsets): the pipelined kernel
                // builds W in LDS instead.
                if (h->forced.count(k)) {
                    if (trial) return BBLOCK_EUNSUPPORTED;
                    return fail(h, BBLOCK_EUNSUPPORTED, "block %d: the precomputed-W plan needs %zu workspace bytes "
                                "(cap %zu) and splits of at most 2 GiB of q1/q2", i, bp.ws_bytes, h->ws_eff);
                }
                // Its column fragments: 7 or 4, whichever pads fewer columns.
                bp.plan.kernel = K_PIPELINED;
                bp.g = Geometry{};
                for (int nb : {7, 4}) {
                    const Geometry g = geometry(h, K_PIPELINED, nb, bp.d.n1, bp.d.n2, bp.d.n3, n_mom);
                    if (g.lds >= 0 && (bp.g.lds < 0 || (long)g.n_nt * g.n_tile < (long)bp.g.n_nt * bp.g.n_tile)) bp.g = g;
                }
                bp.plan.nb = bp.g.nb;
                if (bp.g.lds < 0) {
                    if (trial) return BBLOCK_EUNSUPPORTED;
                    return fail(h, BBLOCK_EUNSUPPORTED, "block %d: no kernel for its shape", i);
                }
                take_geometry(bp);
                set_splits(h, bp, S);
                if (bp.ws_bytes > h->ws_eff) set_splits(h, bp, s_min);
            }
            if (bp.plan.kernel == K_PORD && !w3_offsets_fit(h, bp)) {
                if (h->forced.count(k)) {
                    if (trial) return BBLOCK_EUNSUPPORTED;
                    return fail(h, BBLOCK_EUNSUPPORTED, "block %d: the paper-order plan needs splits of at most 2 GiB of "
                                "q1/q2/q3", i);
                }
                bp.plan.kernel = K_GENERIC;
                bp.plan.nb = 4;
                bp.g = geometry(h, K_GENERIC, bp.plan.nb, bp.d.n1, bp.d.n2, bp.d.n3, n_mom);
                if (bp.g.lds < 0) {
                    if (trial) return BBLOCK_EUNSUPPORTED;
                    return fail(h, BBLOCK_EUNSUPPORTED, "block %d: no kernel for its shape", i);
                }
                take_geometry(bp);
                set_splits(h, bp, S);
            }
            if (bp.ws_bytes > h->ws_eff) {
                if (trial) return BBLOCK_ENOMEM;
                return fail(h, BBLOCK_ENOMEM, "block %d needs %zu workspace bytes, cap is %zu%s", i, bp.ws_bytes, h->ws_eff,
                            noalloc ? " (what the static scratch of the allocation-free entry point leaves for it)" : "");
            }
        }
        return BBLOCK_OK;
    };
    if (walk_fill && h->walk_mode == 2) {
        const std::vector<BlockPlan> bps0 = bps;
        size_t need = 0;
        const bblock_status st = split_pass(true);
        for (const BlockPlan &bp : bps) need += align_up(bp.ws_bytes, 256);
        walk = st != BBLOCK_OK || need > h->ws_eff;
        bps = bps0;
    } else {
        walk = walk_fill;
    }
    {
        const bblock_status st = split_pass(false);
        if (st != BBLOCK_OK) return st;
    }

    // Work units: (block, round).  Every block is one unit, except a
    // precomputed-W block whose images need rounds: each round is a unit of
    // its own with its own descriptor (a copy of the block's with img_s0 set).
    struct Unit {
        int b, r, d;  // block, round, descriptor index
    };
    std::vector<Unit> units;
    std::vector<BlockDesc> descs(n_desc);
    // Blocks in order of kernel instantiation (stable), so that each
    // instantiation forms one sub-batch however the caller interleaves the
    // shapes; spin projection keeps descriptor order (its sums run in it).
    std::vector<int> order(n_desc);
    for (int b = 0; b < n_desc; ++b) order[b] = b;
    if (!coef) {
        auto inst = [&](int b) {
            const BlockPlan &x = bps[b];
            return std::array<int, 5>{x.plan.kernel, x.plan.nb, x.g.b2, x.g.b3, x.plan.persistent};
        };
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return inst(x) < inst(y); });
    }
    for (int b : order) {
        for (int r = 0; r < bps[b].rounds; ++r) {
            int d = b;
            if (r > 0) {
                d = (int)descs.size();
                descs.push_back(BlockDesc{});
            }
            units.push_back({b, r, d});
        }
    }
    if (descs.size() > 65535) return fail(h, BBLOCK_EUNSUPPORTED, "more than 65535 block rounds in one batch");

    // Sub-batches: consecutive units with one kernel instantiation and
    // workspace within the cap (a unit of a block in rounds stays alone).
    // Sub-batches run one after the other on the stream, so each one reuses
    // the workspace from offset 0; a block in rounds keeps its partials at
    // offset 0 through all its rounds and is reduced after the last.
    std::vector<SubBatch> subs;
    std::vector<int4> tiles, went;
    std::vector<int> list;
    std::vector<int> cmem, cgs, cacc;    // spin projection: members, group starts, accumulate flags
    std::vector<double> ccoef;
    std::vector<char> group_started(n_groups, 0);
    std::vector<size_t> ws_off(descs.size(), 0);
    std::vector<size_t> img_off(descs.size(), 0);  // workspace offset of each unit's W images
    size_t ws_need = 0;
    bool any_pipelined = false;
    auto same_kernel = [&](const BlockPlan &x, const SubBatch &sb) {
        return x.plan.kernel == sb.kernel && x.plan.nb == sb.nb && x.g.b2 == sb.b2 && x.g.b3 == sb.b3 &&
               x.plan.persistent == sb.persistent;
    };
    for (size_t u = 0; u < units.size();) {
        const BlockPlan &b0 = bps[units[u].b];
        SubBatch sb{};
        sb.first = (int)u;
        sb.kernel = b0.plan.kernel;
        sb.nb = b0.plan.nb;
        sb.b2 = b0.g.b2;
        sb.b3 = b0.g.b3;
        sb.persistent = b0.plan.persistent;
        sb.grid = b0.plan.grid > 0 ? b0.plan.grid : h->num_cu;
        any_pipelined |= sb.kernel == K_PIPELINED || sb.kernel == K_PORD || sb.kernel == K_F64 || sb.kernel == K_F64P ||
                         sb.kernel == K_F32P || sb.kernel == K_F64N || sb.kernel == K_F32N;
        size_t used = 0;
        long n_went = 0;
        const size_t u0 = u;
        // W images depend on q3, its d3/momentum blocking and the split
        // structure only: blocks of the sub-batch that share them (the spin
        // triples of one noise triple use each q3 several times) share one
        // set, produced once.
        std::map<std::array<long long, 8>, size_t> img_of;
        std::vector<char> makes_img(units.size(), 0);
        while (u < units.size()) {
            const BlockPlan &bp = bps[units[u].b];
            if (u > u0 && (bp.rounds > 1 || b0.rounds > 1)) break;
            if (!same_kernel(bp, sb)) break;
            const std::array<long long, 8> ikey{(long long)(uintptr_t)bp.d.q3, bp.d.n3, bp.plan.nb, bp.g.b3, bp.g.bp,
                                                bp.g.n_nt, bp.d.S, bp.d.sps};
            const bool shared = is_w3(sb.kernel) && bp.rounds == 1 && img_of.count(ikey);
            const size_t need = shared ? align_up(bp.part_bytes, 4096) : bp.ws_bytes;
            if (used + need > h->ws_eff) break;
            if (is_w3(sb.kernel) && !shared) {  // image entries form the y dimension of one launch
                const long e = (long)bp.g.n_nt * bp.spr;
                if (u > u0 && n_went + e > 65535) break;
                n_went += e;
            }
            ws_off[units[u].d] = used;
            if (shared) {
                img_off[units[u].d] = img_of[ikey];
            } else {
                img_off[units[u].d] = used + align_up(bp.part_bytes, 4096);
                makes_img[u] = 1;
                if (is_w3(sb.kernel) && bp.rounds == 1) img_of[ikey] = img_off[units[u].d];
            }
            used += align_up(need, 256);
            ++u;
        }
        sb.count = (int)(u - u0);
        ws_need = std::max(ws_need, used);
        // Tiles, longest first (cost ~ rows x columns x sites); ties keep
        // (block, split, n-tile, m-tile) order so neighbours share inputs.
        struct Item {
            long cost;
            size_t group;  // workspace offset of the W images the tile reads (tiles sharing them stay together)
            int4 t;
        };
        std::vector<Item> items;
        sb.list_off = (int)list.size();
        sb.went_off = (int)went.size();
        for (size_t v = u0; v < u; ++v) {
            const Unit &un = units[v];
            const BlockPlan &bp = bps[un.b];
            const int s_lo = un.r * bp.spr, s_hi = std::min(bp.d.S, s_lo + bp.spr);
            // A walking tile is one entry (split 0) that runs all splits.
            for (int s = s_lo; s < (bp.d.walk ? s_lo + 1 : s_hi); ++s) {
                const long sites = bp.d.walk ? h->V : std::min(bp.d.sps, h->V - s * bp.d.sps);
                const long cost = (long)bp.g.m_tile * bp.g.n_tile * sites;
                for (int nt = 0; nt < bp.g.n_nt; ++nt)
                    for (int mt = 0; mt < bp.g.n_mt; ++mt)
                        items.push_back({cost, img_off[un.d] + (size_t)nt, make_int4(un.d, mt, nt, s)});
            }
            if (is_w3(sb.kernel) && makes_img[v]) {
                sb.cps_max = std::max(sb.cps_max, bp.d.cps);
                for (int s = s_lo; s < s_hi; ++s)
                    for (int nt = 0; nt < bp.g.n_nt; ++nt) went.push_back(make_int4(un.d, nt, s, 0));
            }
            if (!coef && bp.d.S > 1 && !bp.d.walk && un.r == bp.rounds - 1) {
                list.push_back(un.d);
                sb.max_mn = std::max(sb.max_mn, bp.d.M * bp.d.N);
            }
        }
        sb.n_list = (int)list.size() - sb.list_off;
        if (coef) {
            // Blocks completed in this sub-batch, grouped by output (groups
            // in order of first use, members in descriptor order).
            std::map<int, std::vector<int>> members;  // group -> descriptor indices of last rounds
            for (size_t v = u0; v < u; ++v) {
                const Unit &un = units[v];
                if (un.r == bps[un.b].rounds - 1) members[group_of[un.b]].push_back(v);
            }
            sb.cg_off = (int)cacc.size();
            sb.cgs_off = (int)cgs.size();
            for (auto &kv : members) {
                cgs.push_back((int)cmem.size());
                cacc.push_back(group_started[kv.first] ? 1 : 0);
                group_started[kv.first] = 1;
                for (int v : kv.second) {
                    const Unit &un = units[v];
                    cmem.push_back(un.d);
                    ccoef.push_back(coef[2 * un.b]);
                    ccoef.push_back(coef[2 * un.b + 1]);
                    sb.max_mn = std::max(sb.max_mn, bps[un.b].d.M * bps[un.b].d.N);
                }
            }
            cgs.push_back((int)cmem.size());
            sb.n_cg = (int)members.size();
            if (sb.n_cg > 65535) return fail(h, BBLOCK_EUNSUPPORTED, "more than 65535 outputs in one sub-batch");
        }
        if (went.size() - sb.went_off > 65535)
            return fail(h, BBLOCK_EUNSUPPORTED, "block %d has more than 65535 (n-tile, split) pairs", units[u0].b);
        sb.n_went = (int)went.size() - sb.went_off;
        std::stable_sort(items.begin(), items.end(), [&](const Item &x, const Item &y) {
            if (x.cost != y.cost) return x.cost > y.cost;
            return is_w3(sb.kernel) && x.group < y.group;  // tiles reading one image set side by side
        });
        sb.tile_off = (int)tiles.size();
        sb.n_tiles = (int)items.size();
        // One workgroup per tile launches n_tiles x block-size work-items,
        // and a launch holds fewer than 2^32 of them: past 2^20 tiles the
        // sub-batch runs persistent workgroups that take tiles from the
        // counter (uneven-32 in FP32 with the paper-order kernel: 12.7
        // million tiles of 512 threads).
        if (!sb.persistent && sb.n_tiles > (1 << 20)) {
            sb.persistent = 1;
            sb.grid = h->num_cu * wg_per_cu(h, b0.g);
        }
        // XCD-aware order.  The dispatcher hands workgroup g to XCD g mod
        // n_xcd, and each XCD has its own L2.  The tiles of one (block,
        // split) read the same q2/q3 site range, so they are dealt to one
        // XCD: in each round of n_xcd * k table entries, XCD x receives k
        // consecutive entries of the cost-sorted list (k = tiles per split).
        // A persistent launch takes tiles from a counter instead, where the
        // order only sets the cost ordering.
        {
            const int n_xcd = sb.persistent ? 1 : h->n_xcd;
            long per = (long)b0.g.n_mt * b0.g.n_nt;  // tiles per split, or per shared image set
            if (is_w3(sb.kernel) && !items.empty()) {
                long same = 0;
                while (same < (long)items.size() && items[same].group == items[0].group) ++same;
                per = std::max(per, same);
            }
            const int k = (int)std::min<long>(std::max<long>(1, per), h->cu_per_xcd);
            const int n = (int)items.size();
            for (int base = 0; base < n; base += n_xcd * k) {
                const int m = std::min(n_xcd * k, n - base);
                const int q = m / n_xcd, r = m % n_xcd;
                for (int j = 0; j < m; ++j) {
                    const int x = j % n_xcd, local = j / n_xcd;
                    tiles.push_back(items[base + x * q + std::min(x, r) + local].t);
                }
            }
        }
        subs.push_back(sb);
    }
    if (!noalloc) {
        bblock_status st = ensure_ws(h, ws_need);
        if (st != BBLOCK_OK) return st;
    }
    void *ws_base = noalloc ? static_cast<void *>(h->scratch + s_ws_off) : h->d_ws;
    for (const Unit &un : units) {
        BlockPlan &bp = bps[un.b];
        BlockDesc d = bp.d;
        unsigned char *base = static_cast<unsigned char *>(ws_base) + ws_off[un.d];
        d.ws = bp.part_bytes ? base : nullptr;
        d.wimg = is_w3(bp.plan.kernel) ? static_cast<unsigned char *>(ws_base) + img_off[un.d] : nullptr;
        d.img_s0 = un.r * bp.spr;
        descs[un.d] = d;
    }

    // Device tables: blocks | tiles | reduce list | momenta (reduced mod L).
    std::vector<int> mom_red(3 * n_mom);
    for (int i = 0; i < 3 * n_mom; ++i) mom_red[i] = ((mom[i] % h->L) + h->L) % h->L;
    const size_t off_blocks = 0;
    const size_t off_tiles = align_up(off_blocks + sizeof(BlockDesc) * descs.size(), 256);
    const size_t off_list = align_up(off_tiles + sizeof(int4) * tiles.size(), 256);
    const size_t off_mom = align_up(off_list + sizeof(int) * std::max<size_t>(1, list.size()), 256);
    const size_t off_went = align_up(off_mom + sizeof(int) * 3 * n_mom, 256);
    const size_t off_cmem = align_up(off_went + sizeof(int4) * std::max<size_t>(1, went.size()), 256);
    const size_t off_ccoef = align_up(off_cmem + sizeof(int) * std::max<size_t>(1, cmem.size()), 256);
    const size_t off_cgs = align_up(off_ccoef + sizeof(double) * std::max<size_t>(2, ccoef.size()), 256);
    const size_t off_cacc = align_up(off_cgs + sizeof(int) * std::max<size_t>(1, cgs.size()), 256);
    const size_t bytes = align_up(off_cacc + sizeof(int) * std::max<size_t>(1, cacc.size()), 256);
    if (noalloc) {
        if (bytes > SCRATCH_TABLE)
            return fail(h, BBLOCK_ENOMEM, "the batch's tables (%zu bytes) exceed the %zu bytes the static scratch holds "
                        "for them", bytes, SCRATCH_TABLE);
    } else {
        bblock_status st = ensure_table(h, bytes);
        if (st != BBLOCK_OK) return st;
    }
    const Mem mem = noalloc ? Mem{h->scratch, ws_base, h->scratch + s_kidx_off} : Mem{h->d_table, h->d_ws, nullptr};
    hipEvent_t upload_done = noalloc ? h->static_free : h->staging_free;
    HIP_OR_FAIL(h, hipEventSynchronize(upload_done));  // previous upload has left the staging buffer
    unsigned char *hs = noalloc ? h->h_static : h->h_staging;
    std::memcpy(hs + off_blocks, descs.data(), sizeof(BlockDesc) * descs.size());
    if (!tiles.empty()) std::memcpy(hs + off_tiles, tiles.data(), sizeof(int4) * tiles.size());
    if (!list.empty()) std::memcpy(hs + off_list, list.data(), sizeof(int) * list.size());
    std::memcpy(hs + off_mom, mom_red.data(), sizeof(int) * 3 * n_mom);
    if (!went.empty()) std::memcpy(hs + off_went, went.data(), sizeof(int4) * went.size());
    if (!cmem.empty()) std::memcpy(hs + off_cmem, cmem.data(), sizeof(int) * cmem.size());
    if (!ccoef.empty()) std::memcpy(hs + off_ccoef, ccoef.data(), sizeof(double) * ccoef.size());
    if (!cgs.empty()) std::memcpy(hs + off_cgs, cgs.data(), sizeof(int) * cgs.size());
    if (!cacc.empty()) std::memcpy(hs + off_cacc, cacc.data(), sizeof(int) * cacc.size());
    HIP_OR_FAIL(h, hipMemcpyAsync(mem.table, hs, bytes, hipMemcpyHostToDevice, h->stream));
    HIP_OR_FAIL(h, hipEventRecord(upload_done, h->stream));
    if (noalloc) {
        // Rebuilt on every call: another call may have overwritten it.
        if (any_pipelined) {
            const hipError_t e = launch_phase_index(reinterpret_cast<const int *>(mem.table + off_mom), n_mom, h->L,
                                                    kstride_of(h), mem.kidx, h->stream);
            if (e != hipSuccess) return hip_fail(h, e, "launch of the phase-index kernel");
        }
        size_t offs[T_COUNT] = {off_blocks, off_tiles, off_list, off_mom, off_went, off_cmem, off_ccoef, off_cgs, off_cacc};
        return launch_planned(h, mem, subs, offs, n_mom, true);
    }
    if (any_pipelined) {
        bblock_status st = ensure_kidx(h, mom_red, reinterpret_cast<const int *>(h->d_table + off_mom));
        if (st != BBLOCK_OK) return st;
    }

    h->last_key = std::move(key);
    h->last_subs = subs;
    h->last_offs[T_BLOCKS] = off_blocks;
    h->last_offs[T_TILES] = off_tiles;
    h->last_offs[T_LIST] = off_list;
    h->last_offs[T_MOM] = off_mom;
    h->last_offs[T_WENT] = off_went;
    h->last_offs[T_CMEM] = off_cmem;
    h->last_offs[T_CCOEF] = off_ccoef;
    h->last_offs[T_CGS] = off_cgs;
    h->last_offs[T_CACC] = off_cacc;
    return launch_planned(h, Mem{h->d_table, h->d_ws, h->d_kidx}, subs, h->last_offs, n_mom, false);
}

// ---------------------------------------------------------------- tuner ---
template <class F>
__global__ void fill_uniform(F *p, size_t n, unsigned seed)
{
    // Deterministic pseudo-random fill in [-1, 1), for timing only.
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        unsigned x = (unsigned)(i * 2654435761u) ^ seed;
        x ^= x >> 16;
        x *= 0x7feb352du;
        x ^= x >> 15;
        x *= 0x846ca68bu;
        x ^= x >> 16;
        p[i] = (F)((double)(x >> 8) * (2.0 / 16777216.0) - 1.0);
    }
}

bblock_status shape_ok(bblock_t h, int n1, int n2, int n3, int n_mom)
{
    if (n1 < 1 || n2 < 1 || n3 < 1 || n1 > h->max_ndil || n2 > h->max_ndil || n3 > h->max_ndil || n_mom < 1 ||
        n_mom > MAX_MOM)
        return fail(h, BBLOCK_EINVAL, "bad shape (%d,%d,%d) n_mom %d", n1, n2, n3, n_mom);
    return BBLOCK_OK;
}

}  // namespace

// ================================================================== ABI ===
extern "C" {

const char *bblock_version(void) { return "bblock 0.2 (gfx950)"; }

bblock_status bblock_create(bblock_t *out, int32_t L, int32_t prec, int32_t in_dtype, int32_t max_ndil,
                            size_t workspace_cap, void *hip_stream)
{
    if (!out) return fail(nullptr, BBLOCK_EINVAL, "out is NULL");
    *out = nullptr;
    if (L < 1 || L > MAX_L) return fail(nullptr, BBLOCK_EINVAL, "L=%d outside [1,%d]", L, MAX_L);
    if (prec < BBLOCK_FP64 || prec > BBLOCK_BF16X3) return fail(nullptr, BBLOCK_EINVAL, "unknown precision %d", prec);
    if (in_dtype != BBLOCK_C128 && in_dtype != BBLOCK_C64) return fail(nullptr, BBLOCK_EINVAL, "unknown dtype %d", in_dtype);
    if (max_ndil < 1 || max_ndil > MAX_NDIL) return fail(nullptr, BBLOCK_EINVAL, "max_ndil=%d outside [1,%d]", max_ndil, MAX_NDIL);
    int dev = 0, count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return fail(nullptr, BBLOCK_ENODEV, "no HIP device");
    if (hipGetDevice(&dev) != hipSuccess) return fail(nullptr, BBLOCK_ENODEV, "no current HIP device");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return fail(nullptr, BBLOCK_ENODEV, "device query failed");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, BBLOCK_ENODEV, "device %d is %s, this library is built for gfx950", dev, prop.gcnArchName);

    bblock_t h = new (std::nothrow) bblock_s;
    if (!h) return fail(nullptr, BBLOCK_ENOMEM, "host allocation");
    h->device = dev;
    h->L = L;
    h->V = L * L * L;
    h->prec = prec;
    h->in_dtype = in_dtype;
    h->max_ndil = max_ndil;
    h->ws_cap = workspace_cap ? workspace_cap : (size_t)8 << 30;
    h->stream = reinterpret_cast<hipStream_t>(hip_stream);
    h->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    h->n_xcd = std::max(1, h->num_cu / h->cu_per_xcd);
    h->lds_max = (int)prop.sharedMemPerBlock;

    auto bail = [&](bblock_status st, const char *what) {
        bblock_destroy(h);
        g_create_error = what;
        return st;
    };
    // Best effort: ROCm launches accept dynamic LDS up to the device limit
    // without this attribute; where the call is supported it documents intent.
    if (prepare_kernels(h->lds_max) != hipSuccess) (void)hipGetLastError();
    if (prepare_fast_kernels(h->lds_max) != hipSuccess) (void)hipGetLastError();
    if (hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return bail(BBLOCK_EHIP, "stream creation failed");
    if (hipEventCreateWithFlags(&h->staging_free, hipEventDisableTiming) != hipSuccess)
        return bail(BBLOCK_EHIP, "event creation failed");
    // Phase roots exp(-2 pi i k / L), k = 0..L-1, in FP64 on the host.
    std::vector<double> roots(2 * L);
    for (int k = 0; k < L; ++k) {
        const double ang = 2.0 * M_PI * (double)k / (double)L;
        roots[2 * k] = std::cos(ang);
        roots[2 * k + 1] = -std::sin(ang);
    }
    if (hipMalloc(&h->d_roots, sizeof(double) * 2 * L) != hipSuccess) return bail(BBLOCK_ENOMEM, "roots allocation");
    if (hipMemcpy(h->d_roots, roots.data(), sizeof(double) * 2 * L, hipMemcpyHostToDevice) != hipSuccess)
        return bail(BBLOCK_EHIP, "roots upload");
    if (hipMalloc(&h->d_counter, 2 * sizeof(int)) != hipSuccess) return bail(BBLOCK_ENOMEM, "counter allocation");
    if (hipMemset(h->d_counter, 0, 2 * sizeof(int)) != hipSuccess) return bail(BBLOCK_EHIP, "counter reset");
    // The allocation-free entry point: this device's scratch array (looked up
    // once per device, with the device current) and the pinned buffer its
    // tables go up through.
    if (scratch_address(dev, &h->scratch) != hipSuccess) return bail(BBLOCK_EHIP, "static scratch lookup");
    if (hipHostMalloc(&h->h_static, SCRATCH_TABLE, hipHostMallocDefault) != hipSuccess)
        return bail(BBLOCK_ENOMEM, "pinned staging allocation");
    if (hipEventCreateWithFlags(&h->static_free, hipEventDisableTiming) != hipSuccess)
        return bail(BBLOCK_EHIP, "event creation failed");

    // Walking tiles: BBLOCK_SPLIT_WALK=0 never, 1 every block of every
    // unprojected batch (tests force it on small batches), unset: batches
    // that fill the device and whose partials exceed the workspace.
    if (const char *w = std::getenv("BBLOCK_SPLIT_WALK")) h->walk_mode = std::atoi(w) == 0 ? 0 : (std::atoi(w) == 1 ? 1 : 2);
    // Tuned plans persisted by earlier runs.
    if (const char *path = std::getenv("BBLOCK_TUNE_CACHE")) {
        if (FILE *f = std::fopen(path, "r")) {
            int pr, l, n1, n2, n3, nm, ke, nb, sp, pe, gr;
            char line[256];
            while (std::fgets(line, sizeof line, f))
                if (std::sscanf(line, "%d %d %d %d %d %d %d %d %d %d %d", &pr, &l, &n1, &n2, &n3, &nm, &ke, &nb, &sp,
                                &pe, &gr) == 11 &&
                    pr == prec && l == L && geometry(h, ke, nb, n1, n2, n3, nm).lds > 0)
                    h->tuned[{n1, n2, n3, nm}] = Plan{ke, nb, sp, pe, gr};
            std::fclose(f);
        }
    }
    *out = h;
    return BBLOCK_OK;
}

}  // extern "C"

namespace {

bblock_status compute_range(bblock_t h, const void *Q1, const void *Q2, const void *Q3, int32_t n1, int32_t n2,
                            int32_t n3, const int32_t *mom, int32_t n_mom, int32_t t_begin, int32_t t_end, void *B,
                            bool noalloc)
{
    if (!h) return fail(h, BBLOCK_EINVAL, "null handle");
    if (t_begin < 0 || t_end <= t_begin) return fail(h, BBLOCK_EINVAL, "empty or negative timeslice range [%d,%d)", t_begin, t_end);
    if (!Q1 || !Q2 || !Q3 || !B) return fail(h, BBLOCK_EINVAL, "null buffer");
    if (n1 < 1 || n2 < 1 || n3 < 1 || n1 > h->max_ndil || n2 > h->max_ndil || n3 > h->max_ndil)
        return fail(h, BBLOCK_EINVAL, "dilution sizes (%d,%d,%d) outside [1,%d]", n1, n2, n3, h->max_ndil);
    if (!mom || n_mom < 1 || n_mom > MAX_MOM) return fail(h, BBLOCK_EINVAL, "n_mom must be in [1,%d]", MAX_MOM);
    const int nt = t_end - t_begin;
    const size_t eb = in_bytes(h->in_dtype);
    std::vector<bblock_desc> d(nt);
    for (int i = 0; i < nt; ++i) {
        const size_t t = (size_t)(t_begin + i);
        d[i].q1 = static_cast<const unsigned char *>(Q1) + t * h->V * 3 * n1 * eb;
        d[i].q2 = static_cast<const unsigned char *>(Q2) + t * h->V * 3 * n2 * eb;
        d[i].q3 = static_cast<const unsigned char *>(Q3) + t * h->V * 3 * n3 * eb;
        d[i].n1 = n1;
        d[i].n2 = n2;
        d[i].n3 = n3;
        d[i].reserved = 0;
        d[i].out = static_cast<unsigned char *>(B) + (size_t)i * n_mom * n1 * n2 * n3 * 16;
    }
    return run_batch(h, d.data(), nt, mom, n_mom, nullptr, noalloc);
}

}  // namespace

extern "C" {

bblock_status bblock_compute(bblock_t h, const void *Q1, const void *Q2, const void *Q3, int32_t n1, int32_t n2,
                             int32_t n3, const int32_t *mom, int32_t n_mom, int32_t t_begin, int32_t t_end, void *B)
{
    return compute_range(h, Q1, Q2, Q3, n1, n2, n3, mom, n_mom, t_begin, t_end, B, false);
}

bblock_status bblock_compute_noalloc(bblock_t h, const void *Q1, const void *Q2, const void *Q3, int32_t n1,
                                     int32_t n2, int32_t n3, const int32_t *mom, int32_t n_mom, int32_t t_begin,
                                     int32_t t_end, void *B)
{
    return compute_range(h, Q1, Q2, Q3, n1, n2, n3, mom, n_mom, t_begin, t_end, B, true);
}

bblock_status bblock_compute_batch(bblock_t h, const bblock_desc *desc, int32_t n_desc, const int32_t *mom, int32_t n_mom)
{
    return run_batch(h, desc, n_desc, mom, n_mom);
}

bblock_status bblock_compute_projected(bblock_t h, const bblock_desc *desc, const double *coef, int32_t n_desc,
                                       const int32_t *mom, int32_t n_mom)
{
    if (!coef) return fail(h, BBLOCK_EINVAL, "coef is NULL");
    return run_batch(h, desc, n_desc, mom, n_mom, coef);
}

namespace {

// One complex GEMM launch on the handle's stream, event-timed with the
// contraction kernels when profiling is on.
bblock_status zgemm_timed(bblock_t h, ZgemmArgs za, const char *what)
{
    std::array<hipEvent_t, 2> ev{nullptr, nullptr};
    if (h->profiling) {
        ev = {take_event(h), take_event(h)};
        if (!ev[0] || !ev[1]) return fail(h, BBLOCK_EHIP, "profiling event creation failed");
        HIP_OR_FAIL(h, hipEventRecord(ev[0], h->stream));
    }
    const hipError_t e = launch_zgemm(za, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, what);
    if (h->profiling) {
        HIP_OR_FAIL(h, hipEventRecord(ev[1], h->stream));
        h->ev_gemm.push_back(ev);
    }
    return BBLOCK_OK;
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

}  // namespace

bblock_status bblock_reconstruct(bblock_t h, const void *phi, int32_t n_ev, const void *Q, int32_t n_dil, int32_t n_q,
                                 void *q)
{
    if (!h) return fail(h, BBLOCK_EINVAL, "null handle");
    if (!phi || !Q || !q) return fail(h, BBLOCK_EINVAL, "null buffer");
    if (n_ev < 1 || n_ev > MAX_MODES) return fail(h, BBLOCK_EINVAL, "n_ev must be in [1,%d]", MAX_MODES);
    if (n_dil < 1 || n_q < 1 || (long long)n_dil * n_q > MAX_MODES * 64LL)
        return fail(h, BBLOCK_EINVAL, "n_dil (%d) and n_q (%d) must be >= 1 with n_dil * n_q <= %d", n_dil, n_q,
                    MAX_MODES * 64);
    if (!aligned(phi, 16) || !aligned(Q, 16) || !aligned(q, in_bytes(h->in_dtype)))
        return fail(h, BBLOCK_EINVAL, "misaligned buffer");
    ZgemmArgs za{};
    za.A = static_cast<const double *>(phi);
    za.a_sm = n_ev;
    za.a_sk = 1;
    za.B = static_cast<const double *>(Q);
    za.b_sk = 1;
    za.b_sn = n_ev;
    za.C = q;
    za.c_sm = n_dil;
    za.c_sn = 1;
    za.c_ng = n_dil;
    za.c_sg = 3LL * h->V * n_dil;
    za.c_c64 = h->in_dtype == BBLOCK_C64;
    za.M = 3 * h->V;
    za.N = n_dil * n_q;
    za.K = n_ev;
    za.batch = 1;
    return zgemm_timed(h, za, "launch of the reconstruction GEMM");
}

bblock_status bblock_mode_triplets(bblock_t h, const void *phi, int32_t n_ev, const int32_t *mom, int32_t n_mom,
                                   void *T)
{
    if (!h) return fail(h, BBLOCK_EINVAL, "null handle");
    bblock_desc d{};
    d.q1 = d.q2 = d.q3 = phi;
    d.n1 = d.n2 = d.n3 = n_ev;
    d.out = T;
    return run_batch(h, &d, 1, mom, n_mom);
}

namespace {

// The block from the mode triplets for n_c coefficient triples sharing T and
// shapes (Sec. 2, after eq. (4)), as three batched GEMMs per round of
// momenta: X1[p][c][d1][l2 l3] = sum_l1 Q1[c][d1][l1] T[p][l1][l2 l3] (the
// triples stacked into the rows), X2[p][c][d1][d2][l3] = sum_l2
// Q2[c][d2][l2] X1[p][c][d1][l2][l3], B[c][p][d1 d2][d3] = sum_l3
// X2[p][c][d1 d2][l3] Q3[c][d3][l3].
bblock_status mode_contract(bblock_t h, const void *T, int n_ev, int n_mom, int n_c, const void *Q1, int n1,
                            const void *Q2, int n2, const void *Q3, int n3, void *B)
{
    if (!h) return fail(h, BBLOCK_EINVAL, "null handle");
    if (!T || !Q1 || !Q2 || !Q3 || !B) return fail(h, BBLOCK_EINVAL, "null buffer");
    if (n_ev < 1 || n_ev > MAX_MODES) return fail(h, BBLOCK_EINVAL, "n_ev must be in [1,%d]", MAX_MODES);
    if (n_mom < 1 || n_mom > MAX_MOM) return fail(h, BBLOCK_EINVAL, "n_mom must be in [1,%d]", MAX_MOM);
    if (n_c < 1 || n_c > 65536) return fail(h, BBLOCK_EINVAL, "n_c must be in [1,65536]");
    if (n1 < 1 || n2 < 1 || n3 < 1 || n1 > MAX_MODES || n2 > MAX_MODES || n3 > MAX_MODES)
        return fail(h, BBLOCK_EINVAL, "dilution sizes (%d,%d,%d) outside [1,%d]", n1, n2, n3, MAX_MODES);
    if ((long long)n_c * n1 > 0x7fffffffLL / 2 || (long long)n1 * n2 > 0x7fffffffLL / 2)
        return fail(h, BBLOCK_EINVAL, "n_c * n1 and n1 * n2 must fit the GEMM row count");
    if (!aligned(T, 16) || !aligned(Q1, 16) || !aligned(Q2, 16) || !aligned(Q3, 16) || !aligned(B, 16))
        return fail(h, BBLOCK_EINVAL, "misaligned buffer");
    // Intermediates per momentum; momenta go in rounds that fit the cap.
    const size_t e = (size_t)n_ev;
    const size_t x1 = (size_t)n_c * n1 * e * e * 16, x2 = (size_t)n_c * n1 * n2 * e * 16;
    const size_t per_mom = x1 + x2;
    const int pm = (int)std::min<size_t>((size_t)n_mom, h->ws_cap / per_mom);
    if (pm < 1) return fail(h, BBLOCK_ENOMEM, "one momentum needs %zu bytes of workspace, cap %zu", per_mom, h->ws_cap);
    if ((long long)pm * n_c * n1 > 0x7fffffffLL) return fail(h, BBLOCK_EINVAL, "batch of the second GEMM too large");
    if (bblock_status st = ensure_ws(h, (size_t)pm * per_mom)) return st;
    double *X1 = static_cast<double *>(h->d_ws);
    double *X2 = reinterpret_cast<double *>(static_cast<unsigned char *>(h->d_ws) + (size_t)pm * x1);
    const long long ne = n_ev, ne2 = ne * ne, blk = (long long)n1 * n2 * n3;
    for (int p0 = 0; p0 < n_mom; p0 += pm) {
        const int np = std::min(pm, n_mom - p0);
        ZgemmArgs s1{};  // batch p; rows (c, d1)
        s1.A = static_cast<const double *>(Q1);
        s1.a_sm = ne;
        s1.a_sk = 1;
        s1.B = static_cast<const double *>(T) + 2 * p0 * ne2 * ne;
        s1.b_sk = ne2;
        s1.b_sn = 1;
        s1.b_b = batch_uniform(ne2 * ne);
        s1.C = X1;
        s1.c_sm = ne2;
        s1.c_sn = 1;
        s1.c_ng = (int)ne2;
        s1.c_b = batch_uniform((long long)n_c * n1 * ne2);
        s1.M = n_c * n1;
        s1.N = (int)ne2;
        s1.K = n_ev;
        s1.batch = np;
        if (bblock_status st = zgemm_timed(h, s1, "launch of the first mode contraction")) return st;
        ZgemmArgs s2{};  // batch b = (p n_c + c) n1 + d1
        s2.A = static_cast<const double *>(Q2);
        s2.a_sm = ne;
        s2.a_sk = 1;
        s2.a_b.s0 = (long long)n2 * ne;  // Q2[c], c = (b / n1) % n_c
        s2.a_b.d0 = n1;
        s2.a_b.m0 = n_c;
        s2.B = X1;
        s2.b_sk = ne;
        s2.b_sn = 1;
        s2.b_b = batch_uniform(ne2);
        s2.C = X2;
        s2.c_sm = ne;
        s2.c_sn = 1;
        s2.c_ng = n_ev;
        s2.c_b = batch_uniform((long long)n2 * ne);
        s2.M = n2;
        s2.N = n_ev;
        s2.K = n_ev;
        s2.batch = np * n_c * n1;
        if (bblock_status st = zgemm_timed(h, s2, "launch of the second mode contraction")) return st;
        ZgemmArgs s3{};  // batch b = p n_c + c
        s3.A = X2;
        s3.a_sm = ne;
        s3.a_sk = 1;
        s3.a_b = batch_uniform((long long)n1 * n2 * ne);
        s3.B = static_cast<const double *>(Q3);
        s3.b_sk = 1;
        s3.b_sn = ne;
        s3.b_b.s0 = (long long)n3 * ne;  // Q3[c], c = b % n_c
        s3.b_b.m0 = n_c;
        s3.C = static_cast<unsigned char *>(B) + (size_t)p0 * blk * 16;
        s3.c_sm = n3;
        s3.c_sn = 1;
        s3.c_ng = n3;
        s3.c_b.s0 = (long long)n_mom * blk;  // B[c][p0 + p]: c = b % n_c, p = b / n_c
        s3.c_b.m0 = n_c;
        s3.c_b.s1 = blk;
        s3.c_b.d1 = n_c;
        s3.c_b.m1 = 0x7fffffff;
        s3.M = n1 * n2;
        s3.N = n3;
        s3.K = n_ev;
        s3.batch = np * n_c;
        if (bblock_status st = zgemm_timed(h, s3, "launch of the third mode contraction")) return st;
    }
    return BBLOCK_OK;
}

}  // namespace

bblock_status bblock_mode_contract(bblock_t h, const void *T, int32_t n_ev, int32_t n_mom, const void *Q1, int32_t n1,
                                   const void *Q2, int32_t n2, const void *Q3, int32_t n3, void *B)
{
    return mode_contract(h, T, n_ev, n_mom, 1, Q1, n1, Q2, n2, Q3, n3, B);
}

bblock_status bblock_mode_contract_batch(bblock_t h, const void *T, int32_t n_ev, int32_t n_mom, int32_t n_c,
                                         const void *Q1, int32_t n1, const void *Q2, int32_t n2, const void *Q3,
                                         int32_t n3, void *B)
{
    return mode_contract(h, T, n_ev, n_mom, n_c, Q1, n1, Q2, n2, Q3, n3, B);
}

bblock_status bblock_set_graph(bblock_t h, int32_t enable)
{
    if (!h) return fail(h, BBLOCK_EINVAL, "null handle");
    if (enable < 0 || enable > 2) return fail(h, BBLOCK_EINVAL, "graph mode must be 0, 1 or 2");
    h->graph_mode = enable;
    return BBLOCK_OK;
}

bblock_status bblock_set_plan(bblock_t h, int32_t n1, int32_t n2, int32_t n3, int32_t n_mom, const bblock_plan *plan)
{
    if (!h) return fail(h, BBLOCK_EINVAL, "null handle");
    if (bblock_status st = shape_ok(h, n1, n2, n3, n_mom)) return st;
    const ShapeKey k{n1, n2, n3, n_mom};
    ++h->plan_gen;
    if (!plan) {
        h->forced.erase(k);
        return BBLOCK_OK;
    }
    if (plan->kernel != K_GENERIC && plan->kernel != K_PIPELINED && !is_w3(plan->kernel) && plan->kernel != K_PORD &&
        plan->kernel != K_F64 && plan->kernel != K_F64P && plan->kernel != K_F32P && plan->kernel != K_F64N &&
        plan->kernel != K_F32N)
        return fail(h, BBLOCK_EINVAL, "unknown kernel %d", plan->kernel);
    if (plan->splits < 0 || plan->grid < 0 || (plan->persistent != 0 && plan->persistent != 1))
        return fail(h, BBLOCK_EINVAL, "bad plan fields");
    if (geometry(h, plan->kernel, plan->nb, n1, n2, n3, n_mom).lds <= 0)
        return fail(h, BBLOCK_EINVAL, "kernel %d with nb=%d is not available for this precision and shape", plan->kernel,
                    plan->nb);
    // FP32-accumulating paths hold at most ACCURACY_MAX_SITES sites per split:
    // an explicit count below that floor is refused, and the planner's own
    // count (splits = 0) is raised to it in whole multiples of the
    // wave-filling count, as for an unforced single block.
    const int s_min = min_splits(h);
    if (plan->splits > 0 && plan->splits < s_min)
        return fail(h, BBLOCK_EINVAL, "splits=%d is below the accuracy floor of %d splits (at most %d sites per "
                    "split in FP32 accumulation)", plan->splits, s_min, ACCURACY_MAX_SITES);
    Plan p{plan->kernel, plan->nb, plan->splits, plan->persistent, plan->grid};
    p.auto_splits = p.splits == 0;
    if (p.splits == 0) p.splits = single_splits(fill_splits(h, geometry(h, p.kernel, p.nb, n1, n2, n3, n_mom)), s_min);
    h->forced[k] = p;
    return BBLOCK_OK;
}

bblock_status bblock_get_plan(bblock_t h, int32_t n1, int32_t n2, int32_t n3, int32_t n_mom, bblock_plan *plan)
{
    if (!h || !plan) return fail(h, BBLOCK_EINVAL, "null argument");
    if (bblock_status st = shape_ok(h, n1, n2, n3, n_mom)) return st;
    // The plan of a momentum set that holds the zero momentum (it differs
    // from one without only at 16 k + 1 momenta).
    const int saved_skip = h->p_skip;
    h->p_skip = n_mom > 1 && n_mom % 16 == 1 ? 0 : -1;
    Plan p = plan_for(h, n1, n2, n3, n_mom);
    if (p.auto_splits)
        p.splits = single_splits(fill_splits(h, geometry(h, p.kernel, p.nb, n1, n2, n3, n_mom)), min_splits(h));
    h->p_skip = saved_skip;
    plan->nb = p.nb;
    plan->splits = h->forced.count(ShapeKey{n1, n2, n3, n_mom}) ? p.splits : single_splits(p.splits, min_splits(h));
    plan->persistent = p.persistent;
    plan->grid = p.grid;
    plan->kernel = p.kernel;
    return BBLOCK_OK;
}

bblock_status bblock_tune(bblock_t h, int32_t n1, int32_t n2, int32_t n3, int32_t n_mom)
{
    if (!h) return fail(h, BBLOCK_EINVAL, "null handle");
    if (bblock_status st = shape_ok(h, n1, n2, n3, n_mom)) return st;
    const ShapeKey key{n1, n2, n3, n_mom};
    const size_t eb = in_bytes(h->in_dtype);
    const size_t qn[3] = {(size_t)h->V * 3 * n1, (size_t)h->V * 3 * n2, (size_t)h->V * 3 * n3};
    const size_t out_elems = (size_t)n_mom * n1 * n2 * n3;
    void *q[3] = {nullptr, nullptr, nullptr};
    double *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bblock_status st = BBLOCK_OK;
    std::vector<int32_t> mom(3 * n_mom);
    for (int i = 0; i < n_mom; ++i) {  // a spread of momenta; timing does not depend on them
        mom[3 * i] = i % 3 == 0 ? i / 3 : 0;
        mom[3 * i + 1] = i % 3 == 1 ? i / 3 : 0;
        mom[3 * i + 2] = i % 3 == 2 ? i / 3 : 0;
    }
    const int saved_graph = h->graph_mode;
    const bool saved_prof = h->profiling;
    const bool had_forced = h->forced.count(key) != 0;
    const Plan saved_forced = had_forced ? h->forced[key] : Plan{};
    Plan best{};
    bool have_best = false;
    float best_ms = 1e30f;
    std::vector<double> hout(2 * out_elems), href(2 * out_elems);

    auto cleanup = [&]() {
        ++h->plan_gen;
        for (void *p : q)
            if (p) (void)hipFree(p);
        if (out) (void)hipFree(out);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        h->graph_mode = saved_graph;
        h->profiling = saved_prof;
        if (had_forced)
            h->forced[key] = saved_forced;
        else
            h->forced.erase(key);
    };
    for (int i = 0; i < 3 && st == BBLOCK_OK; ++i) {
        if (hipMalloc(&q[i], qn[i] * eb) != hipSuccess)
            st = fail(h, BBLOCK_ENOMEM, "tune inputs");
        else if (h->in_dtype == BBLOCK_C128)
            hipLaunchKernelGGL(fill_uniform<double>, dim3(512), dim3(256), 0, h->stream, (double *)q[i], qn[i] * 2, 17u * (i + 1));
        else
            hipLaunchKernelGGL(fill_uniform<float>, dim3(512), dim3(256), 0, h->stream, (float *)q[i], qn[i] * 2, 17u * (i + 1));
    }
    if (st == BBLOCK_OK && hipMalloc(&out, out_elems * 16) != hipSuccess) st = fail(h, BBLOCK_ENOMEM, "tune outputs");
    if (st == BBLOCK_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        st = fail(h, BBLOCK_EHIP, "tune events");
    if (st != BBLOCK_OK) {
        cleanup();
        return st;
    }
    h->graph_mode = 0;
    h->profiling = false;

    // Candidates: kernel x column fragments x split count x scheduling.
    std::vector<Plan> cands;
    {
        const int *opts;
        const int n_opts = nb_options(h->prec, &opts);
        std::vector<std::pair<int, int>> kn;
        for (int nb : {1, 2}) kn.push_back({K_PORD, nb});
        for (int nb : {7, 6, 5, 4}) kn.push_back({K_W3W8, nb});
        for (int nb : {7, 6, 5, 4}) kn.push_back({K_W3, nb});
        for (int nb : {7, 4}) kn.push_back({K_PIPELINED, nb});
        for (int nb : {7, 4, 2}) kn.push_back({K_F64, nb});
        for (int nb : {3, 2, 1}) kn.push_back({K_F64P, nb});
        for (int nb : {4, 3, 2, 1}) kn.push_back({K_F64N, nb});
        for (int nb : {4, 3, 2, 1}) kn.push_back({K_F32P, nb});
        for (int nb : {4, 3, 2, 1}) kn.push_back({K_F32N, nb});
        for (int i = 0; i < n_opts; ++i) kn.push_back({K_GENERIC, opts[i]});
        const int N = n3 * n_mom;
        for (auto [kernel, nb] : kn) {
            const Geometry g = geometry(h, kernel, nb, n1, n2, n3, n_mom);
            if (g.lds <= 0) continue;
            const long padded = (long)g.n_nt * g.n_tile;  // columns, or momenta for the paper-order kernel
            const bool by_mom = kernel == K_PORD || kernel == K_F64P || kernel == K_F32P || kernel == K_F64N ||
                                kernel == K_F32N;
            if (padded > 2L * std::max(by_mom ? n_mom : N, 32)) continue;  // mostly padding
            // Split counts as a tuned plan will run them (at least the
            // accuracy floor, in whole multiples of the wave-filling count).
            const int s_base = fill_splits(h, g), s_min = min_splits(h);
            int last = -1;
            for (int sf : {1, 2, 4}) {
                const int S = single_splits(std::max(s_base * sf / 2, 1), s_min);
                if (S == last) continue;
                last = S;
                for (int pers = 0; pers < 2; ++pers) cands.push_back(Plan{kernel, nb, S, pers, pers ? h->num_cu : 0});
            }
        }
    }
    // Reference: the default plan (the tested one).  A candidate must agree
    // with it to within the error contract of the precision (FP64 1e-10 of
    // the block's largest entry, the FP32-accumulating paths 1e-5) with
    // room for the spread between two correct plans: 1e-11 and 2e-5.
    const double tol = h->prec == FP64 ? 1e-11 : 2e-5;
    const bool verbose = std::getenv("BBLOCK_TUNE_VERBOSE") != nullptr;
    {
        h->forced.erase(key);
        ++h->plan_gen;
        const bblock_desc d{q[0], q[1], q[2], n1, n2, n3, 0, out};
        st = run_batch(h, &d, 1, mom.data(), n_mom);
        if (st == BBLOCK_OK && hipStreamSynchronize(h->stream) != hipSuccess)
            st = fail(h, BBLOCK_EHIP, "tune reference failed");
        if (st == BBLOCK_OK && hipMemcpy(href.data(), out, out_elems * 16, hipMemcpyDeviceToHost) != hipSuccess)
            st = fail(h, BBLOCK_EHIP, "tune reference copy failed");
        if (st != BBLOCK_OK) {
            cleanup();
            return st;
        }
    }
    for (const Plan &cand : cands) {
        h->forced[key] = cand;
        ++h->plan_gen;  // else run_batch would replay the previous candidate's cached schedule
        const bblock_desc d{q[0], q[1], q[2], n1, n2, n3, 0, out};
        st = run_batch(h, &d, 1, mom.data(), n_mom);
        if (st == BBLOCK_EUNSUPPORTED || st == BBLOCK_ENOMEM) {  // candidate does not fit this shape
            st = BBLOCK_OK;
            continue;
        }
        if (st != BBLOCK_OK) break;
        if (hipStreamSynchronize(h->stream) != hipSuccess) {
            st = fail(h, BBLOCK_EHIP, "tune candidate failed");
            break;
        }
        // Consistency against the default plan's result.
        if (hipMemcpy(hout.data(), out, out_elems * 16, hipMemcpyDeviceToHost) != hipSuccess) {
            st = fail(h, BBLOCK_EHIP, "tune candidate copy failed");
            break;
        }
        {
            double dmax = 0, rmax = 0;
            for (size_t i = 0; i < hout.size(); ++i) {
                dmax = std::max(dmax, std::fabs(hout[i] - href[i]));
                rmax = std::max(rmax, std::fabs(href[i]));
            }
            if (!(dmax <= tol * std::max(rmax, 1e-300))) {  // rejected candidate
                if (verbose)
                    std::fprintf(stderr, "bblock_tune: kernel %d nb %d splits %d persistent %d grid %d: rejected "
                                 "(max difference %.3g of %.3g)\n", cand.kernel, cand.nb, cand.splits, cand.persistent,
                                 cand.grid, dmax, rmax);
                continue;
            }
        }
        float best_of = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            (void)hipEventRecord(e0, h->stream);
            st = run_batch(h, &d, 1, mom.data(), n_mom);
            (void)hipEventRecord(e1, h->stream);
            if (st != BBLOCK_OK || hipEventSynchronize(e1) != hipSuccess) break;
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            best_of = std::min(best_of, ms);
        }
        if (st != BBLOCK_OK) break;
        if (verbose)
            std::fprintf(stderr, "bblock_tune: kernel %d nb %d splits %d persistent %d grid %d: %.4f ms\n", cand.kernel,
                         cand.nb, cand.splits, cand.persistent, cand.grid, best_of);
        if (best_of < best_ms) {
            best_ms = best_of;
            best = cand;
            have_best = true;
        }
    }
    cleanup();
    if (st != BBLOCK_OK) return st;
    if (!have_best) return fail(h, BBLOCK_EHIP, "no tuning candidate passed");
    h->tuned[key] = best;
    ++h->plan_gen;
    if (const char *path = std::getenv("BBLOCK_TUNE_CACHE")) {
        if (FILE *f = std::fopen(path, "a")) {
            std::fprintf(f, "%d %d %d %d %d %d %d %d %d %d %d\n", h->prec, h->L, n1, n2, n3, n_mom, best.kernel, best.nb,
                         best.splits, best.persistent, best.grid);
            std::fclose(f);
        }
    }
    return BBLOCK_OK;
}

bblock_status bblock_profile(bblock_t h, int32_t enable)
{
    if (!h) return fail(h, BBLOCK_EINVAL, "null handle");
    h->profiling = enable != 0;
    return BBLOCK_OK;
}

bblock_status bblock_profile_read(bblock_t h, double *gemm_ms, double *reduce_ms, double *prep_ms,
                                  int32_t *gemm_launches)
{
    if (!h) return fail(h, BBLOCK_EINVAL, "null handle");
    double sums[3] = {0.0, 0.0, 0.0};
    const int n_gemm = (int)h->ev_gemm.size();
    bblock_status st = BBLOCK_OK;
    std::vector<std::array<hipEvent_t, 2>> *lists[3] = {&h->ev_gemm, &h->ev_reduce, &h->ev_prep};
    for (int k = 0; k < 3; ++k) {
        for (auto &ev : *lists[k]) {
            float ms = 0.0f;
            hipError_t e = hipEventSynchronize(ev[1]);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
            if (e != hipSuccess && st == BBLOCK_OK) st = hip_fail(h, e, "reading profiling events");
            sums[k] += ms;
            h->ev_pool.push_back(ev[0]);
            h->ev_pool.push_back(ev[1]);
        }
        lists[k]->clear();
    }
    if (gemm_ms) *gemm_ms = sums[0];
    if (reduce_ms) *reduce_ms = sums[1];
    if (prep_ms) *prep_ms = sums[2];
    if (gemm_launches) *gemm_launches = n_gemm;
    return st;
}

bblock_status bblock_sync(bblock_t h)
{
    if (!h) return fail(h, BBLOCK_EINVAL, "null handle");
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
    HIP_OR_FAIL(h, hipGetLastError());
    return BBLOCK_OK;
}

bblock_status bblock_destroy(bblock_t h)
{
    if (!h) return BBLOCK_OK;
    if (h->d_table || h->d_roots || h->h_static) (void)hipStreamSynchronize(h->stream);
    clear_graphs(h);
    if (h->d_ws) (void)hipFree(h->d_ws);
    if (h->d_table) (void)hipFree(h->d_table);
    if (h->d_kidx) (void)hipFree(h->d_kidx);
    if (h->h_staging) (void)hipHostFree(h->h_staging);
    if (h->d_roots) (void)hipFree(h->d_roots);
    if (h->d_counter) (void)hipFree(h->d_counter);
    if (h->staging_free) (void)hipEventDestroy(h->staging_free);
    if (h->h_static) (void)hipHostFree(h->h_static);
    if (h->static_free) (void)hipEventDestroy(h->static_free);
    for (auto &ev : h->ev_gemm) h->ev_pool.insert(h->ev_pool.end(), ev.begin(), ev.end());
    for (auto &ev : h->ev_reduce) h->ev_pool.insert(h->ev_pool.end(), ev.begin(), ev.end());
    for (auto &ev : h->ev_prep) h->ev_pool.insert(h->ev_pool.end(), ev.begin(), ev.end());
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    delete h;
    return BBLOCK_OK;
}

const char *bblock_last_error(bblock_t h)
{
    if (!h) return g_create_error.c_str();
    return h->err.c_str();
}

}  // extern "C"
