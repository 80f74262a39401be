/*
 * bblock.h -- C ABI of libbblock.so: baryon blocks of the stochastic LapH
 * method on AMD Instinct MI355X (gfx950).
 *
 * Operation (paper "Performance Optimization of Baryon-block Construction in
 * the Stochastic LapH Method", Sec. 2, eq. (3), written with the
 * reconstructed quark fields of eq. (2)):
 *
 *   B[p][d1][d2][d3] = sum_x exp(-i p.x) eps_abc q1[x][a][d1] q2[x][b][d2] q3[x][c][d3]
 *
 * per timeslice, for a set of integer momenta n with p = 2 pi n / L.  Spin
 * projection and noise bookkeeping stay with the caller (Sec. 2, after
 * eq. (1)); the kernel is called many times with the same momentum set
 * (Sec. 2, after eq. (3); Sec. 3 on reusing the precomputed phase).
 *
 * Conventions
 *   - site index x = ix + L*(iy + L*iz), 0 <= ix,iy,iz < L, V = L^3;
 *   - phase exp(-i p.x) = exp(-2 pi i k / L) with k = (n.x) mod L (exact);
 *   - eps_012 = +1; dilution indices are 0-based.
 *
 * Layouts (row-major, complex interleaved (re, im)):
 *   quark field  q[t][x][colour 0..2][d], complex128 or complex64 (in_dtype)
 *   output       B[t][p][d1][d2][d3], complex128, always OVERWRITTEN
 *   momenta      host int32 [n_mom][3]; components may be any integers
 *                (reduced mod L).
 *
 * Ownership: the caller owns every quark-field and output buffer (device
 * memory, e.g. torch tensors) and keeps it alive until the work enqueued on
 * the handle's stream has completed.  The handle owns its workspace (split-K
 * partials, phase roots, descriptor and tile tables, work counters, captured
 * graphs, tuned plans).
 *
 * Errors: every entry point validates its arguments on the host before it
 * enqueues anything; on failure it returns a non-zero status, enqueues
 * nothing and records a message readable with bblock_last_error().  Nothing
 * is thrown across the ABI.  Work is asynchronous on the handle's stream: a
 * device-side failure is reported as BBLOCK_EHIP by a later call or by
 * bblock_sync().  A handle is not thread-safe; distinct handles are
 * independent.
 */
#ifndef BBLOCK_H
#define BBLOCK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bblock_s *bblock_t;

typedef enum {
    BBLOCK_OK = 0,
    BBLOCK_EINVAL = 1,       /* bad argument (null pointer, size out of range, misalignment) */
    BBLOCK_ENOMEM = 2,       /* device or host allocation failed, or workspace cap too small */
    BBLOCK_EHIP = 3,         /* HIP runtime error (launch failure, device fault) */
    BBLOCK_ENODEV = 4,       /* no usable gfx950 device */
    BBLOCK_EUNSUPPORTED = 5  /* valid request the library does not implement */
} bblock_status;

/* Arithmetic of the contraction.  FP64: complex double end to end (MFMA f64).
 * FP32: products and per-split accumulation on FP32 MFMA.  BF16X3: each FP32
 * operand split into bf16 hi + lo, three bf16 MFMA products (hi*hi, hi*lo,
 * lo*hi) accumulated in FP32.  For FP32 and BF16X3 the cross-split reduction
 * and the final block sum are FP64. */
typedef enum { BBLOCK_FP64 = 0, BBLOCK_FP32 = 1, BBLOCK_BF16X3 = 2 } bblock_prec;

/* Element type of the quark fields. */
typedef enum { BBLOCK_C128 = 0, BBLOCK_C64 = 1 } bblock_dtype;

/* One block of a grouped launch: one timeslice, one spin-component triple,
 * one noise triple (the caller's labels).  q1, q2, q3 point at a single
 * timeslice [V][3][n_i] of in_dtype; out at [n_mom][n1][n2][n3] complex128. */
typedef struct {
    const void *q1, *q2, *q3;
    int32_t n1, n2, n3;
    int32_t reserved;
    void *out;
} bblock_desc;

/* Launch plan of one block shape (see bblock_set_plan). */
typedef struct {
    int32_t nb;          /* MFMA column fragments per wave (N tile = nb * fragment width) */
    int32_t splits;      /* split-K count over sites (>= 1); 0 = planner chooses */
    int32_t persistent;  /* 1: persistent workgroups pull tiles from an atomic counter */
    int32_t grid;        /* persistent grid size; 0 = planner chooses */
    int32_t kernel;      /* 0: generic tiles (any shape, every precision);
                            1: pipelined rectangular tiles (FP32 and BF16X3,
                               n2 >= 16 and n3 >= 16; nb 4 or 7; the FP32
                               default up to 4 momenta);
                            2: as 1 with the phase-weighted q3 precomputed
                               into workspace images by a separate launch
                               (BF16X3 only; n2 >= 8,
                               n3 >= 16; nb 4 to 7).  Needs workspace for
                               one image per (column tile, chunk of 8
                               sites): 28672, 32768, 40960 or 45056 bytes
                               for nb 4, 5, 6, 7; the planner falls back to
                               1 when the cap does not allow it.
                            3: paper order (section 3: diquark, singlet,
                               then the momentum projection): the singlet
                               S[x][d1 d2 d3] is formed in registers and only
                               the momentum sum runs as an MFMA product over
                               sites (BF16X3 only, n3 >= 16; nb 1 or 2 column
                               fragments of 32 momenta; the default for more
                               than 16 momenta).  Needs no image workspace.
                            4: kernel 2 with eight waves per workgroup, two
                               per SIMD, which split the column fragments
                               (same shapes, images and workspace as 2, and
                               bitwise the same results; the BF16X3 default
                               up to 16 momenta).
                            5: complex double on the FP64 matrix cores with
                               three real products per complex product
                               (FP64 only, any shape; nb 2, 4 or 7 column
                               fragments of 16; 128-row tiles, D and W built
                               in LDS; the FP64 default up to 4 momenta).
                            6: paper order in complex double: the singlet on
                               the vector unit, the momentum projection on
                               the FP64 matrix cores with three real
                               products (FP64 only, n3 >= 16; nb 1, 2 or 3
                               fragments of 16 momenta; the FP64 default
                               from 13 momenta).
                            7: kernel 6's order in FP32: the momentum
                               projection on the FP32 matrix cores with
                               three real products up to nb 2, four above
                               (FP32 only, n3 >= 16; nb 1 to 4 fragments of
                               16 momenta; the FP32 default from 9
                               momenta).
                            8: kernel 6 with fragments of 4 momenta on the
                               FP64 matrix cores' 4x4x4 form and two row
                               sets of 16 per wave (FP64 only, n3 >= 16;
                               nb 1 to 4 fragments of 4; the FP64 default
                               from 5 to 12 momenta, kernel 5 up to 4).
                            9: kernel 7 with fragments of 4 momenta on the
                               FP32 matrix cores' 4x4x1 form of 16 blocks
                               (FP32 only, n3 >= 16; nb 1 to 4 fragments
                               of 4; the FP32 default from 5 to 8 momenta,
                               kernel 1 up to 4).
                            Kernels 6 and 7 (not 8 and 9, whose fragments
                            of 4 keep every momentum a column), given
                            16 k + 1 > 1 momenta of
                            which one is zero mod L (the first such), sum
                            that one's sites (phase 1) on the vector unit
                            and project the other 16 k on the matrix cores:
                            the paper's 33 momenta fill 2 fragments, not 3;
                            kernel 3 with nb 1 does the same at 32 k + 1
                            (33 momenta: one fragment of 32, not two). */
} bblock_plan;

/* Create a handle bound to the current HIP device (paper, Sec. 2 after
 * eq. (3): the block kernel is called many times, for different noise and
 * spin combinations, with one momentum set; Sec. 3: the phases are
 * precomputed once and reused.  The handle holds what those calls share:
 * the phase roots, the tables of the last momentum set and batch, the
 * workspace and the launch plans).
 *   L               lattice extent, 1 <= L <= 256 (V = L^3 sites per timeslice)
 *   prec            bblock_prec
 *   in_dtype        bblock_dtype of the quark fields
 *   max_ndil        largest dilution size any call will use, 1..4096
 *   workspace_cap   bytes of split-K workspace the handle may allocate
 *                   (0 = 8 GiB); batches needing more run in sub-batches
 *   hip_stream      hipStream_t to enqueue on (NULL = the null stream)
 * Returns BBLOCK_ENODEV when no gfx950 device is current. */
bblock_status bblock_create(bblock_t *out, int32_t L, int32_t prec, int32_t in_dtype,
                            int32_t max_ndil, size_t workspace_cap, void *hip_stream);

/* Baryon blocks of eq. (3) (paper, Sec. 2), one per timeslice (each
 * timeslice is an independent block, Sec. 2 after eq. (1)).
 * Compute the blocks of timeslices [t_begin, t_end) of Q1, Q2, Q3
 * ([T][V][3][n_i] device buffers) into B ([t_end - t_begin][n_mom][n1][n2][n3]
 * complex128 device buffer).  All timeslices go through one grouped launch.
 * Buffers must be 16-byte aligned.  n_i in 1..max_ndil, 1 <= n_mom <= 128,
 * 0 <= t_begin < t_end. */
bblock_status bblock_compute(bblock_t h, const void *Q1, const void *Q2, const void *Q3,
                             int32_t n1, int32_t n2, int32_t n3,
                             const int32_t *mom, int32_t n_mom,
                             int32_t t_begin, int32_t t_end, void *B);

/* bblock_compute for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, results and plans as bblock_compute, but the call
 * allocates nothing: its tables, phase-index table and split-K workspace
 * live in a static device array of BBLOCK_NOALLOC_SCRATCH_BYTES that the
 * library holds on each device it runs on until the process ends (1 MiB of
 * tables, then n_mom * L^3 bytes of phase indices, then the workspace), and
 * the tables go up through a pinned buffer allocated by bblock_create.  The
 * planner fits the plan into what remains of the array (fewer splits, or the
 * kernel that builds W in LDS instead of workspace images); a batch that
 * still does not fit returns BBLOCK_ENOMEM with the sizes in the message.
 * Launches are eager (no graph), nothing is cached between calls, and the
 * array is shared by every call and handle on the device: calls that overlap
 * on one GPU (other streams, other threads) race and must be serialised by
 * the caller. */
#define BBLOCK_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
bblock_status bblock_compute_noalloc(bblock_t h, const void *Q1, const void *Q2, const void *Q3,
                                     int32_t n1, int32_t n2, int32_t n3,
                                     const int32_t *mom, int32_t n_mom,
                                     int32_t t_begin, int32_t t_end, void *B);

/* Many eq. (3) blocks in one grouped launch (paper, Sec. 2 after eq. (3):
 * the kernel is evaluated for many noise and spin combinations per
 * timeslice with the same momentum set; Sec. 3: independent blocks run in
 * parallel).
 * Grouped launch over n_desc independent blocks (uneven dilution sizes
 * allowed), one momentum set: one contraction launch per kernel
 * instantiation the batch needs (blocks are grouped by it), plus the W-image
 * launches of kernels 2 and 4, whose blocks with the same third field share
 * one set of images.  When the batch's tiles fill the device without
 * splitting the sites and its split partials would not fit the workspace,
 * each tile's workgroup runs all its site splits in order and adds each
 * split's result into B in FP64 (walking tiles: no partials, no reduction
 * launch, no sub-batches; bitwise the result of the split-K reduction; not
 * for kernel 3, which runs faster in sub-batches); the environment variable
 * BBLOCK_SPLIT_WALK=0 turns this off, =1 forces it for every block.  The tile schedule of a batch structure is captured into a
 * hipGraph on first use and replayed when the same structure (count,
 * shapes, momentum count) comes back; only the descriptor table is
 * re-uploaded.  desc is host memory, read before the call returns. */
bblock_status bblock_compute_batch(bblock_t h, const bblock_desc *desc, int32_t n_desc,
                                   const int32_t *mom, int32_t n_mom);

/* Spin-projected blocks (paper, eq. (1): a baryon correlator term is a linear
 * combination over spin triples of eq. (3) blocks).  Descriptors whose out
 * pointers are equal form one output; each output is overwritten with
 *   out = sum_i coef_i * B_i
 * over its descriptors i, coef_i = coef[2i] + i coef[2i+1] (host, complex128,
 * finite).  Blocks summed into one output must have one shape (n1, n2, n3).
 * The sum runs in FP64 in descriptor order (reproducible).  Otherwise as
 * bblock_compute_batch; the B_i themselves are not written. */
bblock_status bblock_compute_projected(bblock_t h, const bblock_desc *desc, const double *coef, int32_t n_desc,
                                       const int32_t *mom, int32_t n_mom);

/* ---- LapH subspace (paper, Sec. 2, eqs. (2) and (4)) ----------------------
 * The quark fields are combinations of the Laplacian eigenvectors phi^{(l)},
 * l = 0..n_ev-1, of one timeslice, with per-field coefficients Q.  Two routes
 * lead to the block of eq. (3): reconstruct the fields (bblock_reconstruct)
 * and run bblock_compute on them, or precompute the mode triplets of eq. (4)
 * once (bblock_mode_triplets) and contract each set of coefficients onto
 * them (bblock_mode_contract).  All three run on the handle's stream and
 * enqueue nothing when they return an error.  n_ev <= 4096. */

/* Quark-field reconstruction, eq. (2):
 *   q[i][x][a][d] = sum_l Q[i][d][l] * phi[x][a][l]
 * for n_q coefficient sets i (spin components, quark lines) in one pass over
 * the eigenvectors.
 *   phi  [V][3][n_ev] complex128 device buffer (V = L^3 of the handle)
 *   Q    [n_q][n_dil][n_ev] complex128 device buffer
 *   q    [n_q][V][3][n_dil] device buffer in the handle's input dtype
 *        (complex128, or complex64 rounded from the FP64 sum), overwritten:
 *        exactly the field layout bblock_compute reads.
 * Arithmetic: FP64 complex multiply-adds on the matrix cores.  Buffers
 * 16-byte aligned (q: 8 for complex64).  n_dil * n_q <= 262144.
 * The GEMMs of this entry point and of bblock_mode_contract pick one of six
 * wave layouts per launch; the environment variable BBLOCK_ZGEMM_LAYOUT=0..5
 * forces one (for tests). */
bblock_status bblock_reconstruct(bblock_t h, const void *phi, int32_t n_ev, const void *Q, int32_t n_dil,
                                 int32_t n_q, void *q);

/* Mode triplets, eq. (4):
 *   T[p][l1][l2][l3] = sum_x exp(-i p.x) eps_abc phi[x][a][l1] phi[x][b][l2] phi[x][c][l3]
 * i.e. the block of eq. (3) with all three fields set to the eigenvectors:
 * phi is a [V][3][n_ev] field in the handle's input dtype, T a
 * [n_mom][n_ev][n_ev][n_ev] complex128 device buffer (overwritten), computed
 * in the handle's precision by the block kernels (n_ev <= max_ndil). */
bblock_status bblock_mode_triplets(bblock_t h, const void *phi, int32_t n_ev, const int32_t *mom, int32_t n_mom,
                                   void *T);

/* The block from the mode triplets (Sec. 2, after eq. (4)):
 *   B[p][d1][d2][d3] = sum_{l1 l2 l3} Q1[d1][l1] Q2[d2][l2] Q3[d3][l3] T[p][l1][l2][l3]
 *   T   [n_mom][n_ev][n_ev][n_ev] complex128 device buffer (bblock_mode_triplets)
 *   Qi  [n_i][n_ev] complex128 device buffers
 *   B   [n_mom][n1][n2][n3] complex128 device buffer, overwritten
 * Three FP64 complex GEMMs on the matrix cores, one per eigenvector index
 * (l1, then l2, then l3), through handle workspace of
 * (n1 n_ev^2 + n1 n2 n_ev) * 16 bytes per momentum; momenta go in rounds
 * when the cap holds fewer (BBLOCK_ENOMEM when it holds not even one).
 * n_i <= 4096, 1 <= n_mom <= 128, buffers 16-byte aligned. */
bblock_status bblock_mode_contract(bblock_t h, const void *T, int32_t n_ev, int32_t n_mom, const void *Q1, int32_t n1,
                                   const void *Q2, int32_t n2, const void *Q3, int32_t n3, void *B);

/* bblock_mode_contract for n_c coefficient triples at once (the paper's many
 * noise and spin combinations per timeslice, Sec. 2 after eq. (3)), sharing
 * T and the shapes: Qi [n_c][n_i][n_ev] complex128, B [n_c][n_mom][n1][n2][n3]
 * complex128 (block c at B + c n_mom n1 n2 n3).  The triples share each GEMM
 * launch (the first stacks them into its rows), so a call costs far less
 * than n_c single ones.  Workspace (n1 n_ev^2 + n1 n2 n_ev) * 16 * n_c bytes
 * per momentum; 1 <= n_c <= 65536; otherwise as bblock_mode_contract. */
bblock_status bblock_mode_contract_batch(bblock_t h, const void *T, int32_t n_ev, int32_t n_mom, int32_t n_c,
                                         const void *Q1, int32_t n1, const void *Q2, int32_t n2, const void *Q3,
                                         int32_t n3, void *B);

/* hipGraph use in bblock_compute_batch, bblock_compute and
 * bblock_compute_projected: 0 = eager launches, 1 = capture each schedule
 * once and replay it, 2 = replay only schedules of 4 or more kernel launches
 * (the default: a replayed graph leaves more idle time between its kernels
 * than eager launches on one stream, so it pays only when it saves many
 * launches).  Other values: BBLOCK_EINVAL. */
bblock_status bblock_set_graph(bblock_t h, int32_t enable);

/* Autotune the launch plan for one block shape (paper, Sec. 4: the block
 * sizes of the CPU kernel are tuned experimentally per machine; here the
 * GPU kernel family, tile width, split count and scheduling mode).  Times
 * the candidate plans (column fragments per wave, split count, persistent
 * or not) on synthetic data with HIP events, checks each candidate's result
 * against the default plan's (relative to the block's largest entry: 1e-11
 * for FP64, 2e-5 for FP32 and BF16X3), keeps the fastest, and appends it to the file named by the
 * BBLOCK_TUNE_CACHE environment variable when that is set; with
 * BBLOCK_TUNE_VERBOSE set it prints each candidate's time (or rejection) to
 * stderr.  Synchronous. */
bblock_status bblock_tune(bblock_t h, int32_t n1, int32_t n2, int32_t n3, int32_t n_mom);

/* Force (or, with plan == NULL, forget) the plan used for one block shape
 * (paper, Sec. 4: tuned block sizes).  For FP32 and BF16X3 a split holds at
 * most 4096 sites (the FP32 accumulation depth the 1e-5 error contract
 * assumes): an explicit split count below ceil(L^3 / 4096) returns
 * BBLOCK_EINVAL, and splits = 0 takes the planner's wave-filling count,
 * raised to that floor in whole multiples of itself. */
bblock_status bblock_set_plan(bblock_t h, int32_t n1, int32_t n2, int32_t n3, int32_t n_mom,
                              const bblock_plan *plan);

/* The plan the handle would use for one block shape (forced, tuned or
 * default).  At 16 k + 1 momenta it is the plan of a set that holds the
 * zero momentum (kernels 6 and 7 then count 16 k momentum columns; the
 * paper's momentum shells hold it). */
bblock_status bblock_get_plan(bblock_t h, int32_t n1, int32_t n2, int32_t n3, int32_t n_mom,
                              bblock_plan *plan);

/* Kernel timing.  While enabled (enable = 1), launches run eagerly (never
 * from a captured graph) and every contraction-kernel, reduction-kernel and
 * W-image launch is bracketed by HIP events recorded on the handle's stream;
 * the complex GEMMs of bblock_reconstruct and bblock_mode_contract count as
 * contraction kernels. */
bblock_status bblock_profile(bblock_t h, int32_t enable);

/* Synchronises on the last recorded event, then returns the summed
 * event-timed milliseconds of the contraction kernels (gemm_ms), of the
 * split-K reduction kernels (reduce_ms) and of the W-image kernels of plan
 * kernels 2 and 4 (prep_ms) recorded since the previous read, and the number of
 * contraction launches among them.  Any output pointer may be NULL. */
bblock_status bblock_profile_read(bblock_t h, double *gemm_ms, double *reduce_ms, double *prep_ms,
                                  int32_t *gemm_launches);

/* Block until the handle's stream has drained; reports device-side errors. */
bblock_status bblock_sync(bblock_t h);

/* Release the handle (synchronises its stream first, then frees the
 * workspace, tables, graphs and events bblock_create and the calls on the
 * handle allocated; the paper's Sec. 2 sequence of calls with one momentum
 * set ends here).  NULL is accepted. */
bblock_status bblock_destroy(bblock_t h);

/* Message of the last failure on h; with h == NULL, of the calling thread's
 * last failed bblock_create.  Never NULL; valid until the next call on h. */
const char *bblock_last_error(bblock_t h);

/* Library version string. */
const char *bblock_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BBLOCK_H */
