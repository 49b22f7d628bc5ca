/*
 * ptap.h -- C ABI of the MI355X (gfx950) library for the sparse triple product
 *
 *     C = P^T A P,   A: n x n,  P: n x m,  C: m x m   (Section 3, Eq. tripleproduct)
 *
 * built with the all-at-once and merged all-at-once algorithms (Section 3, Alg. 7-10):
 * each row R_I = A(I,:) P of the product AP is formed in a hash accumulator and folded at
 * once into C by the outer product P(I,:) (x) R_I (Eq. allatonceoutproduct), so that neither
 * AP nor P^T is ever stored.  The two-step method (Alg. 5-6: AP and P^T stored explicitly,
 * then P^T (AP)) is provided beside it as the memory and speed comparison.
 *
 * Conventions shared by every entry point
 *  - Matrices are CSR: int32 row pointers (n_rows + 1 entries, rowptr[0] = 0), int32 column
 *    indices sorted strictly ascending within each row, double values.  Every matrix
 *    pointer is a DEVICE pointer unless stated otherwise.
 *  - The computation is split as in Section 2: a symbolic phase that fixes the pattern of C
 *    with no floating point, and a numeric phase that can be repeated with new values on
 *    the same patterns (the paper runs one symbolic and eleven numerics, Section 4.1).
 *  - The pattern of C is the structural product: (i, j) is stored whenever some I, J have
 *    P(I,i), A(I,J) and P(J,j) stored, whatever their values.  Rows of C are sorted.
 *  - Every launch is enqueued on the caller's stream.  ptap_plan_create (with validation)
 *    and ptap_symbolic synchronise that stream; ptap_numeric, ptap_backward and the batch
 *    launch never do.
 *  - Every entry point returns a ptap_status; no C++ exception crosses this boundary.
 *    Plans are not thread-safe: calls on one plan must not overlap.
 *  - Device workspace is obtained from the caller's allocator (or hipMalloc when none is
 *    given) and counted in ptap_plan_stats.
 */
#ifndef PTAP_H_
#define PTAP_H_

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ptap_status {
  PTAP_OK = 0,
  PTAP_ERR_INPUT = 1,       /* malformed CSR, shape mismatch, bad option, NULL argument */
  PTAP_ERR_TOO_LARGE = 2,   /* a count would overflow int32 indexing */
  PTAP_ERR_OOM = 3,         /* the allocator returned NULL or host memory ran out; the plan is
                               left unchanged */
  PTAP_ERR_HIP = 4,         /* a HIP runtime call failed; see ptap_last_hip_error */
  PTAP_ERR_STATE = 5,       /* call out of order (e.g. numeric before symbolic) */
  PTAP_ERR_UNSUPPORTED = 6  /* option combination not provided (also any other host library
                               error, which is never let through the interface) */
} ptap_status;

/* Algorithm choice (the paper's "allatonce", "merged" and "two-step", Section 4). */
typedef enum ptap_algo {
  PTAP_ALLATONCE = 0, /* Alg. 7/8: pass 1 over rows with off-block P entries, pass 2 over
                         rows with on-block P entries; R_I is formed again in pass 2 */
  PTAP_MERGED = 1,    /* Alg. 9/10: one pass, R_I formed once and folded into both parts */
  PTAP_TWOSTEP = 2    /* Alg. 5/6: stored AP and P^T, then the row-wise product P^T (AP) */
} ptap_algo;

/* How the outer product P(I,:) (x) R_I is added into C (all-at-once and merged only). */
typedef enum ptap_fold {
  PTAP_FOLD_AUTO = 0,   /* per plan, the fold a cost model estimates faster from the symbolic
                           phase's counts (rows formed by the owner fold against rows needed,
                           products, fold terms), with constants measured on MI355X; the owner
                           fold's tiles are built first and released if the atomic fold wins */
  PTAP_FOLD_ATOMIC = 1, /* fine-row sweep; device-wide FP64 atomic adds into C at the slot of
                           each (i, j), found through C's column list of row i */
  PTAP_FOLD_OWNER = 2   /* coarse-row ownership: a workgroup owns a tile of C rows (grown
                           breadth-first over C's pattern at symbolic time), visits the fine
                           rows I with P(I,i) stored for i in the tile (found through P's column
                           index lists, i.e. Eq. allatoncerow), forms each R_I and accumulates
                           the tile in LDS, written to C once.  A row of C longer than a tile is
                           accumulated in C itself with device atomics.  The wavefronts of a
                           workgroup add into the tile in the order they arrive, so results on
                           non-dyadic values can differ in the last bits between runs (every
                           order is a valid FP64 evaluation of the same sum). */
} ptap_fold;

/* Allocator for device workspace.  alloc returns a device pointer or NULL; release frees a
 * pointer returned by alloc.  ctx is passed through unchanged.  Releases are stream-ordered: the
 * library may call release right after enqueueing, on the plan's stream, the last launch that
 * uses the pointer, so release must not let the memory be reused before the work already
 * enqueued on that stream has finished (stream-ordered allocators and caching allocators that
 * track the stream do this; a plain hipFree waits for the device). */
typedef struct ptap_allocator {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*release)(void* ptr, size_t bytes, void* ctx);
  void* ctx;
} ptap_allocator;

typedef struct ptap_options {
  int32_t algo;          /* ptap_algo */
  int32_t fold;          /* ptap_fold; ignored by PTAP_TWOSTEP */
  int32_t nblocks;       /* K >= 1: virtual ownership blocks.  Fine rows and coarse columns are
                            split into K contiguous ranges as in the 1D row partition of
                            Section 2 (Eq. partition); P(I,i) is "diagonal" (P_d) when I and i
                            fall in the same block and "off-diagonal" (P_o) otherwise.  K = 1
                            makes P_o empty, so all-at-once and merged coincide. */
  int32_t tile_entries;  /* owner fold: maximum C entries per tile held on chip (0: default) */
  int32_t hash_slots;    /* 0: automatic.  Otherwise the largest on-chip hash table, in slots
                            (power of two >= 64); longer rows use tables in device memory.
                            Setting it low forces the spill path (used by tests). */
  int32_t validate;      /* 1 (default): check both CSR inputs at plan creation and again at
                            the start of ptap_symbolic (the caller's arrays may have changed in
                            between); 2: at plan creation only, for callers that run the
                            symbolic phase right after creating the plan; 0: never.  Each
                            check is one pass over both patterns and one sync. */
  int32_t xcd_remap;     /* nonzero: map workgroups to tiles so that consecutive tiles run on
                            the same XCD (shared L2 for their common fine rows) */
  int32_t backward;      /* nonzero: also prepare the adjoint (ptap_backward) at symbolic time */
  int32_t owner_waves;   /* owner fold: wavefronts per workgroup, 4, 8 or 16 (0: default 16) */
  int32_t tile_lds;      /* owner fold: LDS bytes per workgroup the tiles are sized for
                            (0: default 80 KiB, two workgroups per CU; capped by the device) */
  int32_t cache;         /* nonzero: cache intermediate data between numerics (Section 4.2,
                            Table 8: repeated products keep what symbolic derived, for more
                            memory).  Here: for every entry A(I,J) the extent of row J of P,
                            start and length packed in 32 bits (4 * nnz(A) bytes, built at
                            symbolic time), read by the owner fold's short-row kernel instead of
                            looking the row pointers of P up again in every numeric.  Built only
                            when the owner fold uses that kernel and nnz(P) < 2^26; the bytes
                            held are reported in ptap_stats.cache_bytes. */
  int32_t owner_kernel;  /* owner fold, merged form (and all-at-once with K = 1): 0 = the
                            short-row and general owner kernels (default); 1 = staged tiles where
                            they fit: the tile's workgroup first copies the rows P(J,:) that its
                            fine rows read (the halo: the columns of A(I,:) over the tile's fine
                            rows I, and the rows I) into LDS, then forms each R_I from there
                            (Eq. allatoncerow).  The halo lists cost 4 bytes per halo row per
                            tile, held by the plan (ptap_stats.workspace_bytes); tiles whose halo
                            does not fit in LDS use the other kernels. */
  uint32_t hash_mul;     /* owner fold, short-row kernel: the odd multiplier of its R_I hash (slot =
                            top 6 bits of key * hash_mul).  0: chosen at symbolic time from a
                            sample of C's rows (the golden ratio unless a fixed candidate needs
                            far fewer probes).  Any odd value gives the same C; an even value is
                            PTAP_ERR_INPUT. */
  int32_t reserved[3];
} ptap_options;

typedef struct ptap_stats {
  int64_t nnz_C;
  int64_t nnz_AP;              /* two-step: entries of the stored auxiliary AP; else 0 */
  int64_t workspace_bytes;     /* device bytes held by the plan now (includes C's pattern) */
  int64_t peak_bytes;          /* high-water mark of the plan's device allocations */
  int64_t pattern_bytes;       /* bytes of C's row pointers and column indices */
  int64_t rows_formed;         /* AP rows formed by one numeric call (with recomputation) */
  int64_t rows_needed;         /* fine rows with a nonempty row of P (formed once each at best) */
  int64_t fold_terms;          /* products P(I,i) * R_I(j) added into C by one numeric call */
  int32_t n_tiles;             /* owner fold: number of C-row tiles */
  int32_t fold_used;           /* ptap_fold actually used */
  int32_t algo;                /* ptap_algo of the plan */
  int32_t nblocks;
  int64_t cache_bytes;         /* device bytes of the numeric cache (ptap_options.cache); else 0 */
  int64_t block_size;          /* bs of a block-sparse plan (ptap_plan_create_bsr); else 1 */
  int64_t staged_tiles;        /* owner fold: tiles that take the staged-tile kernel */
  int64_t staged_lds_bytes;    /* LDS bytes per workgroup of that kernel's launch (0: none) */
  int64_t table_slots;         /* device-memory hash-table slots the general kernels use (rows
                                  whose tables do not fit in LDS); 0 when every table is in LDS */
  int64_t tile_entries;        /* owner fold: entries of C a tile holds at most (0: no tiles) */
  double est_owner_ms;         /* PTAP_FOLD_AUTO: the fold cost model's estimate of the numeric */
  double est_atomic_ms;        /* time with the owner and with the atomic fold (0 otherwise) */
  int64_t hash_mul;            /* owner fold: the short-row kernel's R_I hash multiplier in use
                                  (ptap_options.hash_mul, or the one symbolic chose); 0 without tiles */
} ptap_stats;

typedef struct ptap_plan ptap_plan;
typedef struct ptap_batch ptap_batch;

/* Fill *opts with the defaults: merged, owner fold, K = 1, automatic sizes, validation on. */
void ptap_options_default(ptap_options* opts);

/*
 * Create a plan for C = P^T A P on the patterns of A (n x n, A_nnz entries) and P (n x m,
 * P_nnz entries).  The pattern arrays are caller-owned device arrays and must stay alive and
 * unchanged for the life of the plan.  opts may be NULL (defaults), alloc may be NULL
 * (hipMalloc/hipFree).  On success *out owns a host object released by ptap_plan_destroy.
 * Errors: PTAP_ERR_INPUT (NULL pointer, n or m negative, nnz mismatch, unsorted, duplicate or
 * out-of-range columns, non-monotone row pointers, bad options), PTAP_ERR_TOO_LARGE,
 * PTAP_ERR_OOM, PTAP_ERR_HIP.
 */
ptap_status ptap_plan_create(ptap_plan** out, int32_t n, int32_t m, const int32_t* A_rowptr,
                             const int32_t* A_col, int64_t A_nnz, const int32_t* P_rowptr,
                             const int32_t* P_col, int64_t P_nnz, const ptap_options* opts,
                             const ptap_allocator* alloc, hipStream_t stream);

/*
 * Block-sparse (BSR) plan: A (nb x nb blocks) and P (nb x mb blocks) hold dense bs x bs blocks
 * on the given block patterns, for systems with bs coupled unknowns per node (Section 4.2's
 * neutron-transport problem has many variables per vertex).  The triple product is the same,
 * C(i,j) = sum_{I,J} P(I,i)^T A(I,J) P(J,j) block by block; C comes back as blocks on the block
 * pattern that ptap_get_pattern returns (mb + 1 row pointers, nnz(C) block columns).  Values
 * passed to ptap_numeric are nnz blocks of bs*bs doubles each, row-major, in pattern order (A:
 * A_nnzb blocks, P: P_nnzb blocks, C: nnz(C) blocks).  The numeric phase uses the row form of
 * the all-at-once product (Eq. allatoncerow), one workgroup per block row of C accumulating in
 * LDS; rows too long for LDS add into C with device atomics.  1 <= bs <= 8.  Options: algo must
 * not be two-step; fold and cache are ignored; backward is not supported; ptap_backward and
 * ptap_batch_create reject block plans.  Errors: as ptap_plan_create, plus PTAP_ERR_UNSUPPORTED.
 */
ptap_status ptap_plan_create_bsr(ptap_plan** out, int32_t nb, int32_t mb, int32_t bs,
                                 const int32_t* A_rowptr, const int32_t* A_col, int64_t A_nnzb,
                                 const int32_t* P_rowptr, const int32_t* P_col, int64_t P_nnzb,
                                 const ptap_options* opts, const ptap_allocator* alloc,
                                 hipStream_t stream);

/*
 * Symbolic phase (Section 2; Alg. 7/9 for all-at-once and merged, Alg. 5 for two-step):
 * computes and keeps the pattern of C and every index structure the numeric phase needs.
 * Runs on the device and synchronises the stream: the host reads back counters (nnz(C), the
 * sizes of the row classes built on the device) and, for the owner fold, C's pattern, from
 * which it groups C's rows into tiles with up to 8 threads of its own (one more chooses the hash
 * multiplier; all joined before it returns); the tiles depend on the patterns only, not on the
 * machine.  Host copies go through page-locked buffers that the library allocates itself and
 * keeps in a process-wide pool for later plans (buffers above 256 MiB are freed after use).
 * Temporary device memory comes from the plan's allocator and is released before it returns.
 * Errors: PTAP_ERR_STATE if already done, PTAP_ERR_TOO_LARGE, PTAP_ERR_OOM, PTAP_ERR_HIP.
 */
ptap_status ptap_symbolic(ptap_plan* plan, hipStream_t stream);

/* Pointers to the plan-owned pattern of C (device arrays of m+1 and nnz(C) entries).  Valid
 * until ptap_plan_destroy.  Errors: PTAP_ERR_STATE before symbolic. */
ptap_status ptap_get_pattern(const ptap_plan* plan, int64_t* nnz_C, const int32_t** C_rowptr,
                             const int32_t** C_col);

/*
 * Copy the pattern of C into caller-owned device buffers: C_rowptr (m + 1 entries) and C_col
 * (nnz(C) entries), asynchronously on the stream (device-to-device).  Either pointer may be NULL
 * to skip that array.  The plan keeps its own copy.  Errors: PTAP_ERR_INPUT (NULL plan),
 * PTAP_ERR_STATE before symbolic, PTAP_ERR_HIP.
 */
ptap_status ptap_copy_pattern(const ptap_plan* plan, int32_t* C_rowptr, int32_t* C_col,
                              hipStream_t stream);

/*
 * Numeric phase (Alg. 8 all-at-once, Alg. 10 merged, Alg. 6 two-step): writes the nnz(C)
 * values of C, in the order of the pattern, into the caller's device array C_val.  A_val and
 * P_val hold the values of A and P in the order of their patterns.  Asynchronous on the
 * stream; allocates nothing.  Inputs must not alias C_val.
 * Errors: PTAP_ERR_STATE before symbolic, PTAP_ERR_INPUT (NULL), PTAP_ERR_HIP.
 */
ptap_status ptap_numeric(ptap_plan* plan, const double* A_val, const double* P_val, double* C_val,
                         hipStream_t stream);

/*
 * For callers that cannot allocate device memory at all during the numeric call (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the numeric phase of
 * ptap_numeric with the same kernels and the same result, which neither allocates nor uses the
 * plan's workspace for scratch.  The general kernels' device-memory hash tables (rows whose tables
 * do not fit in LDS) live in a fixed array of the library instead: 2^20 slots (4-byte keys and
 * 8-byte values, 12 MiB), one array per GPU, held from the first call on that GPU until the
 * process ends, and cleared at the start of every call by fill kernels on the stream (no memset).
 * Every call on a GPU shares that GPU's array, so calls that overlap on one GPU (other streams,
 * other threads) race and must not be made.  Errors: as ptap_numeric, plus PTAP_ERR_TOO_LARGE when
 * the plan's tables need more than 2^20 slots (ptap_numeric then still works).
 */
ptap_status ptap_numeric_noalloc(ptap_plan* plan, const double* A_val, const double* P_val,
                                 double* C_val, hipStream_t stream);

/*
 * Adjoint of the numeric phase.  Given dC = dL/dC on the pattern of C, writes
 *   dA = P dC P^T                 restricted to the pattern of A  (A_nnz values), and
 *   dP = A P dC^T + A^T P dC      restricted to the pattern of P  (P_nnz values),
 * the derivatives of L with respect to the stored entries of A and P.  Either output may be
 * NULL to skip it.  Rows of AP are formed again, never stored.  Outputs are overwritten.
 * Asynchronous; allocates nothing.  Errors: as ptap_numeric.
 */
ptap_status ptap_backward(ptap_plan* plan, const double* A_val, const double* P_val,
                          const double* dC_val, double* dA_val, double* dP_val,
                          hipStream_t stream);

/* Statistics of the plan (host struct filled by the call): the device memory the plan holds and
 * its high-water mark (the counterpart of the "Mem" column of Section 4's tables, which reports
 * the memory of each algorithm), and the work one numeric call does (rows of AP formed, with
 * recomputation, against the rows needed; fold terms).  Errors: PTAP_ERR_INPUT (NULL). */
ptap_status ptap_plan_stats(const ptap_plan* plan, ptap_stats* out);

/* Release the plan and all its device workspace (through the plan's allocator).  Accepts
 * NULL.  The caller must make sure no work of the plan is still running. */
void ptap_plan_destroy(ptap_plan* plan);

/*
 * Batched numeric over several plans (levels of a hierarchy or independent problems).
 * plans[k] must have finished its symbolic phase; the plans stay owned by the caller and
 * must outlive the batch.  level[k] orders the work: every product with level L runs after
 * every product with a smaller level (a coarse level's A is the previous level's C).  The
 * products of one level run together in one persistent launch that takes (plan, tile) work
 * items from per-XCD counters; a level holding a single plan uses that plan's own launch.
 * level may be NULL (all 0).  Plans with the owner or the atomic fold can be batched (a plan
 * with the atomic fold records its own launches into the graph); two-step plans are rejected.
 * The batch records its launches once into a HIP graph at the first ptap_batch_numeric call
 * and replays the graph afterwards; pointer arguments must therefore stay the same on every
 * call (their contents may change).
 * Errors: PTAP_ERR_INPUT, PTAP_ERR_STATE (a plan without symbolic, two-step plans),
 * PTAP_ERR_OOM, PTAP_ERR_HIP.
 */
ptap_status ptap_batch_create(ptap_batch** out, ptap_plan* const* plans, const int32_t* level,
                              int32_t count, const ptap_allocator* alloc, hipStream_t stream);

/* A_vals[k], P_vals[k], C_vals[k]: host arrays of device pointers, one per plan. */
ptap_status ptap_batch_numeric(ptap_batch* batch, const double* const* A_vals,
                               const double* const* P_vals, double* const* C_vals,
                               hipStream_t stream);

void ptap_batch_destroy(ptap_batch* batch);

/* Static description of a status code.  Never NULL. */
const char* ptap_status_string(ptap_status status);

/* The hipError_t of the last failing HIP call made by the library on this thread (0 if none). */
int32_t ptap_last_hip_error(void);

/*
 * Measurement helper, not part of the product: *out = sum of x[0..n), a plain streaming read of
 * n FP64 values (every value read once, in coalesced 16-byte loads).  Timing it gives the HBM
 * read bandwidth this device reaches, the measured counterpart of the published peak that the
 * numeric kernels are compared against.  x and out are device pointers; x holds n values and
 * must be 16-byte aligned; out is overwritten.  Asynchronous on stream.
 * Errors: PTAP_ERR_INPUT (NULL pointer with n > 0, n < 0, misaligned x), PTAP_ERR_HIP.
 */
ptap_status ptap_stream_sum(const double* x, int64_t n, double* out, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* PTAP_H_ */
