// Host side of libbblock.so: the C ABI declared in include/bblock.h.
//
// Responsibilities: argument validation, the phase-root table (paper, Sec. 3:
// the phase of the momentum projection is precomputed and reused across
// kernel invocations with the same momentum set), the planner (tile shape,
// split-K count, workspace), the grouped tile schedule, hipGraph capture and
// replay of grouped launches, and the autotuner (the paper tunes its block
// sizes experimentally per machine, Sec. 4; here the tile shape and split
// count are timed on the device).

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/bblock.h"
#include "bb_internal.h"

using namespace bb;

namespace {

thread_local std::string g_create_error;

constexpr int MAX_NDIL = 4096;
constexpr int ACCURACY_MAX_SITES = 4096;  // FP32-accumulating paths: sites per split at most

struct Plan {
    int nb = 0, splits = 0, persistent = 0, grid = 0;
};

using ShapeKey = std::array<int, 4>;  // n1, n2, n3, n_mom

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

struct bblock_s {
    int device = 0;
    int L = 0, V = 0;
    int prec = 0, in_dtype = 0, max_ndil = 0;
    size_t ws_cap = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    int num_cu = 256;
    int lds_max = 160 * 1024;

    double *d_roots = nullptr;  // [L] complex128
    int *d_counter = nullptr;   // [2]
    unsigned char *d_table = nullptr;  // blocks | tiles | list | momenta
    size_t table_cap = 0;
    unsigned char *h_staging = nullptr;  // pinned mirror of d_table
    hipEvent_t staging_free = nullptr;
    void *d_ws = nullptr;
    size_t ws_size = 0;

    bool graph_enabled = true;
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::array<hipEvent_t, 2>> ev_gemm, ev_reduce;
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
}

// Default plan of one block shape: the N tile covers the columns (p, d3) in
// as few tiles as possible, the split count fills the device for a single
// block and keeps FP32 accumulation chains bounded.
Plan default_plan(bblock_t h, int n1, int n2, int n3, int n_mom)
{
    const int *opts;
    const int n_opts = nb_options(h->prec, &opts);
    const KernelGeom g0 = kernel_geom(h->prec, opts[0], n_mom, h->L);
    const int N = n3 * n_mom, M = n1 * n2;
    const int max_nb = opts[n_opts - 1];
    const int n_nt = (N + max_nb * g0.frag_cols - 1) / (max_nb * g0.frag_cols);
    const int want_nb = (N + n_nt * g0.frag_cols - 1) / (n_nt * g0.frag_cols);
    Plan p;
    p.nb = max_nb;
    for (int i = 0; i < n_opts; ++i)
        if (opts[i] >= want_nb) {
            p.nb = opts[i];
            break;
        }
    const KernelGeom g = kernel_geom(h->prec, p.nb, n_mom, h->L);
    const long tiles = (long)((M + g.m_tile - 1) / g.m_tile) * ((N + p.nb * g.frag_cols - 1) / (p.nb * g.frag_cols));
    long s = (h->num_cu + tiles - 1) / tiles;
    p.splits = (int)std::max<long>(1, s);
    p.persistent = 0;
    p.grid = 0;
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

struct BlockPlan {
    BlockDesc d;
    Plan plan;
    int n_mt, n_nt;
    size_t ws_bytes;
};

// Sites per split for S splits: a multiple of CHUNK_SITES; the split count
// actually used is ceil(V / sps).
void set_splits(bblock_t h, BlockPlan &bp, int S)
{
    S = std::max(1, std::min(S, (h->V + CHUNK_SITES - 1) / CHUNK_SITES));
    int sps = (int)align_up((size_t)((h->V + S - 1) / S), CHUNK_SITES);
    bp.d.sps = sps;
    bp.d.S = (h->V + sps - 1) / sps;
    bp.ws_bytes = bp.d.S > 1 ? (size_t)bp.d.S * 2 * bp.d.M * bp.d.N * part_bytes(h->prec) : 0;
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
    if (h->d_table) (void)hipFree(h->d_table);
    if (h->h_staging) (void)hipHostFree(h->h_staging);
    h->d_table = nullptr;
    h->h_staging = nullptr;
    h->table_cap = 0;
    const size_t cap = align_up(std::max(bytes, bytes + bytes / 2), 1 << 16);
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
    if (h->d_ws) (void)hipFree(h->d_ws);
    h->d_ws = nullptr;
    h->ws_size = 0;
    if (hipMalloc(&h->d_ws, bytes) != hipSuccess) return fail(h, BBLOCK_ENOMEM, "workspace allocation of %zu bytes", bytes);
    h->ws_size = bytes;
    return BBLOCK_OK;
}

struct SubBatch {
    int first, count;       // blocks [first, first+count)
    int tile_off, n_tiles;  // into the tile table
    int list_off, n_list;   // into the reduce list
    int nb;                 // kernel instantiation
    int persistent, grid;
    int max_mn;
};

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
bblock_status enqueue(bblock_t h, const std::vector<SubBatch> &subs, size_t off_blocks, size_t off_tiles,
                      size_t off_list, size_t off_mom, int n_mom, hipStream_t st)
{
    for (const SubBatch &sb : subs) {
        GemmArgs ga;
        ga.blocks = reinterpret_cast<const BlockDesc *>(h->d_table + off_blocks);
        ga.tiles = reinterpret_cast<const int4 *>(h->d_table + off_tiles) + sb.tile_off;
        ga.n_tiles = sb.n_tiles;
        ga.counter = sb.persistent ? h->d_counter : nullptr;
        ga.mom = reinterpret_cast<const int *>(h->d_table + off_mom);
        ga.n_mom = n_mom;
        ga.L = h->L;
        ga.V = h->V;
        ga.in_c64 = h->in_dtype == BBLOCK_C64;
        ga.roots = h->d_roots;
        const int grid = sb.persistent ? std::min(sb.grid, sb.n_tiles) : sb.n_tiles;
        std::array<hipEvent_t, 2> ev{nullptr, nullptr};
        if (h->profiling) {
            ev = {take_event(h), take_event(h)};
            if (!ev[0] || !ev[1]) return fail(h, BBLOCK_EHIP, "profiling event creation failed");
            HIP_OR_FAIL(h, hipEventRecord(ev[0], st));
        }
        hipError_t e = launch_gemm(h->prec, sb.nb, ga, grid, st);
        if (e != hipSuccess) return hip_fail(h, e, "launch of the contraction kernel");
        if (h->profiling) {
            HIP_OR_FAIL(h, hipEventRecord(ev[1], st));
            h->ev_gemm.push_back(ev);
        }
        if (sb.n_list > 0) {
            ReduceArgs ra;
            ra.blocks = ga.blocks;
            ra.list = reinterpret_cast<const int *>(h->d_table + off_list) + sb.list_off;
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

bblock_status run_batch(bblock_t h, const bblock_desc *desc, int n_desc, const int32_t *mom, int n_mom)
{
    if (!h) return fail(h, BBLOCK_EINVAL, "null handle");
    if (!desc || n_desc < 1) return fail(h, BBLOCK_EINVAL, "empty batch");
    if (!mom || n_mom < 1 || n_mom > MAX_MOM) return fail(h, BBLOCK_EINVAL, "n_mom must be in [1,%d]", MAX_MOM);
    for (int i = 0; i < n_desc; ++i) {
        bblock_status st = validate_desc(h, desc[i], i);
        if (st != BBLOCK_OK) return st;
    }
    // Plans and workspace per block.
    const int s_min = min_splits(h);
    std::vector<BlockPlan> bps(n_desc);
    long total_tiles_s1 = 0;
    for (int i = 0; i < n_desc; ++i) {
        const bblock_desc &d = desc[i];
        BlockPlan &bp = bps[i];
        bp.plan = plan_for(h, d.n1, d.n2, d.n3, n_mom);
        const KernelGeom g = kernel_geom(h->prec, bp.plan.nb, n_mom, h->L);
        if (g.lds_bytes < 0 || g.lds_bytes > h->lds_max)
            return fail(h, BBLOCK_EUNSUPPORTED, "no kernel for nb=%d with n_mom=%d, L=%d", bp.plan.nb, n_mom, h->L);
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
        bp.n_mt = (bp.d.M + g.m_tile - 1) / g.m_tile;
        bp.n_nt = (bp.d.N + bp.plan.nb * g.frag_cols - 1) / (bp.plan.nb * g.frag_cols);
        total_tiles_s1 += (long)bp.n_mt * bp.n_nt;
    }
    // Split count: a forced/tuned plan fixes it for single blocks; in batches
    // it follows from the device size, never below the accuracy bound.
    for (int i = 0; i < n_desc; ++i) {
        BlockPlan &bp = bps[i];
        int S;
        const ShapeKey k{bp.d.n1, bp.d.n2, bp.d.n3, n_mom};
        const bool fixed = h->forced.count(k) && bp.plan.splits > 0;
        if (fixed)
            S = bp.plan.splits;
        else if (n_desc == 1 && bp.plan.splits > 0)
            S = std::max(bp.plan.splits, s_min);
        else
            S = std::max<long>(s_min, (2L * h->num_cu + total_tiles_s1 - 1) / total_tiles_s1);
        set_splits(h, bp, S);
        if (!fixed && bp.ws_bytes > h->ws_cap) set_splits(h, bp, s_min);
        if (bp.ws_bytes > h->ws_cap)
            return fail(h, BBLOCK_ENOMEM, "block %d needs %zu workspace bytes, cap is %zu", i, bp.ws_bytes, h->ws_cap);
    }

    // Sub-batches: consecutive blocks with one kernel instantiation and
    // workspace within the cap.  Sub-batches run one after the other on the
    // stream, so each one reuses the workspace from offset 0.
    std::vector<SubBatch> subs;
    std::vector<int4> tiles;
    std::vector<int> list;
    std::vector<size_t> ws_off(n_desc, 0);
    size_t ws_need = 0;
    for (int i = 0; i < n_desc;) {
        SubBatch sb{};
        sb.first = i;
        sb.nb = bps[i].plan.nb;
        sb.persistent = bps[i].plan.persistent;
        sb.grid = bps[i].plan.grid > 0 ? bps[i].plan.grid : h->num_cu;
        size_t used = 0;
        while (i < n_desc && bps[i].plan.nb == sb.nb && bps[i].plan.persistent == sb.persistent &&
               used + bps[i].ws_bytes <= h->ws_cap) {
            ws_off[i] = used;
            used += align_up(bps[i].ws_bytes, 256);
            ++i;
        }
        sb.count = i - sb.first;
        ws_need = std::max(ws_need, used);
        // Tiles, longest first (cost ~ rows x columns x sites); ties keep
        // (block, split, n-tile, m-tile) order so neighbours share inputs.
        struct Item {
            long cost;
            int4 t;
        };
        std::vector<Item> items;
        sb.list_off = (int)list.size();
        for (int b = sb.first; b < i; ++b) {
            const BlockPlan &bp = bps[b];
            const KernelGeom g = kernel_geom(h->prec, bp.plan.nb, n_mom, h->L);
            const int nt_w = bp.plan.nb * g.frag_cols;
            for (int s = 0; s < bp.d.S; ++s) {
                const long sites = std::min(bp.d.sps, h->V - s * bp.d.sps);
                for (int nt = 0; nt < bp.n_nt; ++nt)
                    for (int mt = 0; mt < bp.n_mt; ++mt) {
                        const long rows = std::min(g.m_tile, bp.d.M - mt * g.m_tile);
                        const long cols = std::min(nt_w, bp.d.N - nt * nt_w);
                        items.push_back({rows * cols * sites, make_int4(b, mt, nt, s)});
                    }
            }
            if (bp.d.S > 1) {
                list.push_back(b);
                sb.max_mn = std::max(sb.max_mn, bp.d.M * bp.d.N);
            }
        }
        sb.n_list = (int)list.size() - sb.list_off;
        std::stable_sort(items.begin(), items.end(), [](const Item &x, const Item &y) { return x.cost > y.cost; });
        sb.tile_off = (int)tiles.size();
        sb.n_tiles = (int)items.size();
        for (const Item &it : items) tiles.push_back(it.t);
        subs.push_back(sb);
    }
    {
        bblock_status st = ensure_ws(h, ws_need);
        if (st != BBLOCK_OK) return st;
    }
    for (int i = 0; i < n_desc; ++i)
        bps[i].d.ws = bps[i].ws_bytes ? static_cast<unsigned char *>(h->d_ws) + ws_off[i] : nullptr;

    // Device tables: blocks | tiles | reduce list | momenta (reduced mod L).
    const size_t off_blocks = 0;
    const size_t off_tiles = align_up(off_blocks + sizeof(BlockDesc) * n_desc, 256);
    const size_t off_list = align_up(off_tiles + sizeof(int4) * tiles.size(), 256);
    const size_t off_mom = align_up(off_list + sizeof(int) * std::max<size_t>(1, list.size()), 256);
    const size_t bytes = align_up(off_mom + sizeof(int) * 3 * n_mom, 256);
    {
        bblock_status st = ensure_table(h, bytes);
        if (st != BBLOCK_OK) return st;
    }
    HIP_OR_FAIL(h, hipEventSynchronize(h->staging_free));  // previous upload has left the staging buffer
    unsigned char *hs = h->h_staging;
    for (int i = 0; i < n_desc; ++i) std::memcpy(hs + off_blocks + sizeof(BlockDesc) * i, &bps[i].d, sizeof(BlockDesc));
    if (!tiles.empty()) std::memcpy(hs + off_tiles, tiles.data(), sizeof(int4) * tiles.size());
    if (!list.empty()) std::memcpy(hs + off_list, list.data(), sizeof(int) * list.size());
    int *hm = reinterpret_cast<int *>(hs + off_mom);
    for (int i = 0; i < 3 * n_mom; ++i) hm[i] = ((mom[i] % h->L) + h->L) % h->L;
    HIP_OR_FAIL(h, hipMemcpyAsync(h->d_table, hs, bytes, hipMemcpyHostToDevice, h->stream));
    HIP_OR_FAIL(h, hipEventRecord(h->staging_free, h->stream));

    if (!h->graph_enabled || h->profiling)
        return enqueue(h, subs, off_blocks, off_tiles, off_list, off_mom, n_mom, h->stream);

    // Graph signature: everything baked into kernel arguments.
    std::vector<long long> sig;
    sig.push_back(n_mom);
    sig.push_back((long long)(uintptr_t)h->d_table);
    for (const SubBatch &sb : subs) {
        sig.insert(sig.end(), {sb.first, sb.count, sb.tile_off, sb.n_tiles, sb.list_off, sb.n_list, sb.nb,
                               sb.persistent, sb.grid, sb.max_mn});
    }
    sig.push_back(n_desc);
    sig.push_back((long long)tiles.size());
    auto it = h->graphs.find(sig);
    if (it == h->graphs.end()) {
        HIP_OR_FAIL(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
        bblock_status st = enqueue(h, subs, off_blocks, off_tiles, off_list, off_mom, n_mom, h->cap_stream);
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

}  // namespace

// ================================================================== ABI ===
extern "C" {

const char *bblock_version(void) { return "bblock 0.1 (gfx950)"; }

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

    auto bail = [&](bblock_status st, const char *what) {
        g_create_error = what;
        bblock_destroy(h);
        return st;
    };
    // Best effort: ROCm launches accept dynamic LDS up to the device limit
    // without this attribute; where the call is supported it documents intent.
    if (prepare_kernels((int)prop.sharedMemPerBlock) != hipSuccess) (void)hipGetLastError();
    h->lds_max = (int)prop.sharedMemPerBlock;
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

    // Tuned plans persisted by earlier runs.
    if (const char *path = std::getenv("BBLOCK_TUNE_CACHE")) {
        if (FILE *f = std::fopen(path, "r")) {
            int pr, l, n1, n2, n3, nm, nb, sp, pe, gr;
            char line[256];
            while (std::fgets(line, sizeof line, f))
                if (std::sscanf(line, "%d %d %d %d %d %d %d %d %d %d", &pr, &l, &n1, &n2, &n3, &nm, &nb, &sp, &pe, &gr) == 10 &&
                    pr == prec && l == L && kernel_geom(prec, nb, nm, L).lds_bytes > 0)
                    h->tuned[{n1, n2, n3, nm}] = Plan{nb, sp, pe, gr};
            std::fclose(f);
        }
    }
    *out = h;
    return BBLOCK_OK;
}

bblock_status bblock_compute(bblock_t h, const void *Q1, const void *Q2, const void *Q3, int32_t n1, int32_t n2,
                             int32_t n3, const int32_t *mom, int32_t n_mom, int32_t t_begin, int32_t t_end, void *B)
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
    return run_batch(h, d.data(), nt, mom, n_mom);
}

bblock_status bblock_compute_batch(bblock_t h, const bblock_desc *desc, int32_t n_desc, const int32_t *mom, int32_t n_mom)
{
    return run_batch(h, desc, n_desc, mom, n_mom);
}

bblock_status bblock_set_graph(bblock_t h, int32_t enable)
{
    if (!h) return fail(h, BBLOCK_EINVAL, "null handle");
    h->graph_enabled = enable != 0;
    return BBLOCK_OK;
}

bblock_status bblock_set_plan(bblock_t h, int32_t n1, int32_t n2, int32_t n3, int32_t n_mom, const bblock_plan *plan)
{
    if (!h) return fail(h, BBLOCK_EINVAL, "null handle");
    if (n1 < 1 || n2 < 1 || n3 < 1 || n_mom < 1 || n_mom > MAX_MOM) return fail(h, BBLOCK_EINVAL, "bad shape");
    const ShapeKey k{n1, n2, n3, n_mom};
    if (!plan) {
        h->forced.erase(k);
        return BBLOCK_OK;
    }
    const KernelGeom g = kernel_geom(h->prec, plan->nb, n_mom, h->L);
    if (g.lds_bytes <= 0 || g.lds_bytes > h->lds_max)
        return fail(h, BBLOCK_EINVAL, "nb=%d is not available for this precision/momentum count", plan->nb);
    if (plan->splits < 0 || plan->grid < 0 || (plan->persistent != 0 && plan->persistent != 1))
        return fail(h, BBLOCK_EINVAL, "bad plan fields");
    Plan p{plan->nb, plan->splits, plan->persistent, plan->grid};
    if (p.splits == 0) p.splits = default_plan(h, n1, n2, n3, n_mom).splits;
    h->forced[k] = p;
    return BBLOCK_OK;
}

bblock_status bblock_get_plan(bblock_t h, int32_t n1, int32_t n2, int32_t n3, int32_t n_mom, bblock_plan *plan)
{
    if (!h || !plan) return fail(h, BBLOCK_EINVAL, "null argument");
    if (n1 < 1 || n2 < 1 || n3 < 1 || n_mom < 1 || n_mom > MAX_MOM) return fail(h, BBLOCK_EINVAL, "bad shape");
    const Plan p = plan_for(h, n1, n2, n3, n_mom);
    plan->nb = p.nb;
    plan->splits = std::max(p.splits, min_splits(h));
    plan->persistent = p.persistent;
    plan->grid = p.grid;
    return BBLOCK_OK;
}

bblock_status bblock_tune(bblock_t h, int32_t n1, int32_t n2, int32_t n3, int32_t n_mom)
{
    if (!h) return fail(h, BBLOCK_EINVAL, "null handle");
    if (n1 < 1 || n2 < 1 || n3 < 1 || n1 > h->max_ndil || n2 > h->max_ndil || n3 > h->max_ndil || n_mom < 1 ||
        n_mom > MAX_MOM)
        return fail(h, BBLOCK_EINVAL, "bad shape");
    const ShapeKey key{n1, n2, n3, n_mom};
    const size_t eb = in_bytes(h->in_dtype);
    const size_t qn[3] = {(size_t)h->V * 3 * n1, (size_t)h->V * 3 * n2, (size_t)h->V * 3 * n3};
    const size_t out_elems = (size_t)n_mom * n1 * n2 * n3;
    void *q[3] = {nullptr, nullptr, nullptr};
    double *out = nullptr, *ref = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bblock_status st = BBLOCK_OK;
    std::vector<int32_t> mom(3 * n_mom);
    for (int i = 0; i < n_mom; ++i) {
        mom[3 * i] = i % 3 == 0 ? i / 3 : 0;
        mom[3 * i + 1] = i % 3 == 1 ? i / 3 : 0;
        mom[3 * i + 2] = i % 3 == 2 ? i / 3 : 0;
    }
    const bool saved_graph = h->graph_enabled;
    const bool had_forced = h->forced.count(key) != 0;
    const Plan saved_forced = had_forced ? h->forced[key] : Plan{};
    Plan best{};
    float best_ms = 1e30f;
    std::vector<double> hout(2 * out_elems), href(2 * out_elems);

    auto cleanup = [&]() {
        for (void *p : q)
            if (p) (void)hipFree(p);
        if (out) (void)hipFree(out);
        if (ref) (void)hipFree(ref);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        h->graph_enabled = saved_graph;
        if (had_forced)
            h->forced[key] = saved_forced;
        else
            h->forced.erase(key);
    };
    for (int i = 0; i < 3 && st == BBLOCK_OK; ++i) {
        if (hipMalloc(&q[i], qn[i] * eb) != hipSuccess) st = fail(h, BBLOCK_ENOMEM, "tune inputs");
        else if (h->in_dtype == BBLOCK_C128)
            hipLaunchKernelGGL(fill_uniform<double>, dim3(512), dim3(256), 0, h->stream, (double *)q[i], qn[i] * 2, 17u * (i + 1));
        else
            hipLaunchKernelGGL(fill_uniform<float>, dim3(512), dim3(256), 0, h->stream, (float *)q[i], qn[i] * 2, 17u * (i + 1));
    }
    if (st == BBLOCK_OK && (hipMalloc(&out, out_elems * 16) != hipSuccess || hipMalloc(&ref, out_elems * 16) != hipSuccess))
        st = fail(h, BBLOCK_ENOMEM, "tune outputs");
    if (st == BBLOCK_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        st = fail(h, BBLOCK_EHIP, "tune events");
    if (st != BBLOCK_OK) {
        cleanup();
        return st;
    }
    h->graph_enabled = false;

    const int *opts;
    const int n_opts = nb_options(h->prec, &opts);
    const Plan def = default_plan(h, n1, n2, n3, n_mom);
    const KernelGeom g0 = kernel_geom(h->prec, opts[0], n_mom, h->L);
    const int N = n3 * n_mom;
    const double tol = h->prec == FP64 ? 1e-11 : 1e-4;
    bool have_ref = false;
    for (int oi = 0; oi < n_opts && st == BBLOCK_OK; ++oi) {
        const int nb = opts[oi];
        const KernelGeom g = kernel_geom(h->prec, nb, n_mom, h->L);
        if (g.lds_bytes <= 0 || g.lds_bytes > h->lds_max) continue;
        if (nb * g.frag_cols > 2 * std::max(N, g0.frag_cols) && nb != def.nb) continue;  // mostly padding
        const int n_tiles = ((n1 * n2 + g.m_tile - 1) / g.m_tile) * ((N + nb * g.frag_cols - 1) / (nb * g.frag_cols));
        const int s_base = std::max(1, (h->num_cu + n_tiles - 1) / n_tiles);
        for (int sf : {1, 2, 4}) {
            for (int pers = 0; pers < 2; ++pers) {
                Plan cand{nb, std::max(s_base * sf / 2, 1), pers, pers ? h->num_cu : 0};
                h->forced[key] = cand;
                const bblock_desc d{q[0], q[1], q[2], n1, n2, n3, 0, out};
                st = run_batch(h, &d, 1, mom.data(), n_mom);
                if (st != BBLOCK_OK) break;
                if (hipStreamSynchronize(h->stream) != hipSuccess) {
                    st = fail(h, BBLOCK_EHIP, "tune candidate failed");
                    break;
                }
                // Consistency against the first candidate's result.
                if (!have_ref) {
                    (void)hipMemcpy(ref, out, out_elems * 16, hipMemcpyDeviceToDevice);
                    (void)hipMemcpy(href.data(), ref, out_elems * 16, hipMemcpyDeviceToHost);
                    have_ref = true;
                } else {
                    (void)hipMemcpy(hout.data(), out, out_elems * 16, hipMemcpyDeviceToHost);
                    double dmax = 0, rmax = 0;
                    for (size_t i = 0; i < hout.size(); ++i) {
                        dmax = std::max(dmax, std::fabs(hout[i] - href[i]));
                        rmax = std::max(rmax, std::fabs(href[i]));
                    }
                    if (!(dmax <= tol * std::max(rmax, 1e-300))) continue;  // rejected candidate
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
                if (best_of < best_ms) {
                    best_ms = best_of;
                    best = cand;
                }
            }
            if (st != BBLOCK_OK) break;
        }
    }
    cleanup();
    if (st != BBLOCK_OK) return st;
    if (best.nb == 0) return fail(h, BBLOCK_EHIP, "no tuning candidate passed");
    h->tuned[key] = best;
    if (const char *path = std::getenv("BBLOCK_TUNE_CACHE")) {
        if (FILE *f = std::fopen(path, "a")) {
            std::fprintf(f, "%d %d %d %d %d %d %d %d %d %d\n", h->prec, h->L, n1, n2, n3, n_mom, best.nb, best.splits,
                         best.persistent, best.grid);
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

bblock_status bblock_profile_read(bblock_t h, double *gemm_ms, double *reduce_ms, int32_t *gemm_launches)
{
    if (!h) return fail(h, BBLOCK_EINVAL, "null handle");
    double sums[2] = {0.0, 0.0};
    const int n_gemm = (int)h->ev_gemm.size();
    bblock_status st = BBLOCK_OK;
    std::vector<std::array<hipEvent_t, 2>> *lists[2] = {&h->ev_gemm, &h->ev_reduce};
    for (int k = 0; k < 2; ++k) {
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
    if (h->stream || h->d_table) (void)hipStreamSynchronize(h->stream);
    clear_graphs(h);
    if (h->d_ws) (void)hipFree(h->d_ws);
    if (h->d_table) (void)hipFree(h->d_table);
    if (h->h_staging) (void)hipHostFree(h->h_staging);
    if (h->d_roots) (void)hipFree(h->d_roots);
    if (h->d_counter) (void)hipFree(h->d_counter);
    if (h->staging_free) (void)hipEventDestroy(h->staging_free);
    for (auto &ev : h->ev_gemm) h->ev_pool.insert(h->ev_pool.end(), ev.begin(), ev.end());
    for (auto &ev : h->ev_reduce) h->ev_pool.insert(h->ev_pool.end(), ev.begin(), ev.end());
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
