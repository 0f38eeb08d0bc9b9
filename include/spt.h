/*
 * spt.h — C-ABI of the MI355X (gfx950) sparse MTTKRP / CP-ALS library.
 *
 * The library stores a sparse tensor as a linearized, bit-interleaved
 * coordinate list: every nonzero keeps its value and one integer position
 * whose bits interleave the bits of its coordinates (Section III-C, problem
 * formulation).  On that single, mode-agnostic copy it computes the mode-n
 * MTTKRP for any n (Section II-B, Fig. 2) and the CP-ALS iteration that
 * calls it along every mode (Section II-B).
 *
 * Conventions shared by every call:
 *  - Modes and coordinates are 0-based.  1 <= nmodes <= SPT_MAX_MODES, every
 *    mode length 1 <= I_n <= 2^32 - 2.
 *  - Pointers are DEVICE pointers unless the comment says "host".  Arrays of
 *    device pointers (factors) are themselves host arrays.
 *  - Factor matrices and MTTKRP outputs are row-major FP32 I_n x rank with
 *    leading dimension rank, 16-byte aligned.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls are stream-ordered; a call that must synchronise says so.
 *  - Every call returns an spt_status and never throws or aborts; on a
 *    non-OK status out-parameters are left untouched and spt_last_error()
 *    returns a message (thread-local).
 *  - The caller owns every buffer it passes; the library owns the memory
 *    behind an spt_tensor until spt_tensor_free.
 *  - Every device buffer the library owns is taken from and returned to its
 *    source in stream order: releasing memory never synchronises the device
 *    or a stream.  The source is the library's block cache (spt_memory_stats)
 *    unless an allocator hook is set (spt_set_allocator).
 */
#ifndef SPT_H
#define SPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPT_MAX_MODES 8
#define SPT_MAX_KEY_BITS 128
#define SPT_MAX_RANK 256      /* mttkrp */
#define SPT_MAX_ALS_RANK 64   /* cp_als (the R x R solve keeps V^-1 in LDS) */

typedef enum {
    SPT_OK = 0,
    SPT_E_INVALID_ARG = -1,   /* bad argument, detected on the host */
    SPT_E_INDEX_RANGE = -2,   /* a coordinate i_n >= I_n (detected on the GPU by encode) */
    SPT_E_TOO_MANY_BITS = -3, /* sum of ceil(log2 I_n) exceeds 128 */
    SPT_E_BAD_LAYOUT = -4,    /* layout is not an interleaving of the modes' bits */
    SPT_E_OOM = -5,           /* device allocation failed */
    SPT_E_NOT_SPD = -6,       /* normal-equation matrix not positive definite after ridge retries */
    SPT_E_DEVICE = -7,        /* a HIP runtime call failed */
    SPT_E_BUSY = -8,          /* server: request does not fit the memory budget / queue closed */
    SPT_E_NOT_FOUND = -9      /* server: unknown ticket */
} spt_status;

typedef struct spt_tensor_s *spt_tensor;

/* Host-side description of an encoded tensor. */
typedef struct {
    int64_t nnz;
    int nmodes;
    int lp;                              /* total key bits, sum of ceil(log2 I_n) */
    int key_words;                       /* 1 (u64 keys) or 2 (u128 keys, two u64 words) */
    int64_t dims[SPT_MAX_MODES];
    int lbits[SPT_MAX_MODES];            /* ceil(log2 I_n); 0 when I_n == 1 */
    uint8_t layout[SPT_MAX_KEY_BITS];    /* layout[t] = mode whose next low bit is key bit t */
    size_t encoded_bytes;                /* nnz * (8 * key_words + 4): keys + values */
    double norm_x2;                      /* sum of squared values, FP64 */
} spt_tensor_info;

/*
 * Per-mode execution plan of MTTKRP (chosen by a heuristic or spt_autotune).
 * Every strategy computes the same result; they differ in how the partial
 * sums of nonzeros that share an output row are combined.
 */
#define SPT_STRATEGY_DIRECT 0   /* walk nonzeros in key order; FP32 atomics at every change of output row */
#define SPT_STRATEGY_REGROUP 1  /* regroup each tile by output row in LDS; atomics once per (tile chunk, row) */
#define SPT_STRATEGY_TABLE 2    /* persistent workgroups accumulate rows in an LDS table; flushed rows are
                                   written as records and summed per row after a radix sort (no atomics
                                   except for rows split between two reducer chunks) */
#define SPT_STRATEGY_PRIV 3     /* the whole output (or column slices of it) lives in each workgroup's LDS;
                                   workgroup partials are summed (small modes) */
#define SPT_STRATEGY_AUTO 4     /* SEGMENT (measured fastest for small and large output modes);
                                   the autotuner also tries PRIV where it fits */
#define SPT_STRATEGY_SEGMENT 5  /* each tile regrouped by output row (the plan: positions of every
                                   nonzero, pieces of at most 64 nonzeros of one row); every piece
                                   becomes a record written with plain stores at a slot that keeps the
                                   records grouped by row; records are summed per row (no atomics
                                   except for rows split between two reducer chunks).  The plan is
                                   built by spt_tensor_prepare: 2 B per nonzero plus 16 B per piece */
typedef struct {
    int tile[SPT_MAX_MODES];      /* nonzeros per workgroup tile: 256..1024 for DIRECT/REGROUP (larger
                                     values act as 1024), 1024/2048/4096 for SEGMENT (smaller values,
                                     or a tile that does not fit LDS for this mode count, act as the
                                     largest that fits); default 4096 */
    int strategy[SPT_MAX_MODES];  /* SPT_STRATEGY_* */
    int row_cache;                /* SEGMENT with 4096-nonzero tiles on tensors of 2..4 modes: 1
                                     (default) keeps each tile's most used factor rows in LDS, read
                                     through the tile dictionaries (built by spt_tensor_prepare: 2 B
                                     per nonzero per mode plus 4 B per distinct (tile, row) pair);
                                     0 reads every factor row from memory */
    int batch_tile;               /* nonzeros per tile of this tensor in batched launches: 1024, 2048
                                     (default; 0 means the default) or 4096.  One batched launch runs
                                     one tile size, its first member's: spt_mttkrp_batched needs every
                                     member prepared at it, spt_cp_als_batched re-plans members at it.
                                     spt_autotune_batched picks it by measurement */
} spt_plan;

/* ---------------------------------------------------------------------- */
/* Device memory.                                                          */
/* ---------------------------------------------------------------------- */

/*
 * Allocator hook: alloc(bytes, stream, ctx) returns device memory usable by
 * work ordered after the call on `stream` (NULL on failure; the library
 * reports SPT_E_OOM); release(ptr, stream, ctx) returns it once all work the
 * library ordered on `stream` before the call is done with it.  The library
 * releases a buffer on the stream of the call that frees it; a hook whose
 * memory is reused per stream (PyTorch's caching allocator) therefore needs
 * that a buffer is used on one stream, which holds for every call except the
 * server, whose requests the library synchronises before release.  Requests
 * are rounded up to 256 bytes and the returned pointer must be 256-byte
 * aligned.  Passing NULL for both restores the default (the block cache
 * below).  Every buffer goes back to the allocator that supplied it,
 * whatever hook is set when it is released.
 * Errors: SPT_E_INVALID_ARG (exactly one hook NULL).
 */
typedef void *(*spt_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*spt_release_fn)(void *ptr, void *stream, void *ctx);
spt_status spt_set_allocator(spt_alloc_fn alloc, spt_release_fn release, void *ctx);

/*
 * The default source of device memory is a block cache per device: blocks
 * come from hipMalloc and are kept after release.  A block released on a
 * stream serves later requests on that stream at once (stream order); a
 * request on another stream takes it only after the work ordered before the
 * release has completed.  Requests of 2 MiB or more round up to a multiple
 * of 2 MiB and may take an idle block up to 1/8 + 2 MiB larger; smaller
 * requests round up to a power of two (at least 512 bytes).  hipMalloc runs
 * only when no idle block fits, so repeating a call with the same sizes
 * allocates nothing from the driver.  If hipMalloc fails, the idle blocks of
 * the device are returned to the driver and the request retried once
 * (SPT_E_OOM if that fails too).  A stream handle that released library
 * memory must not be destroyed and re-created while that work is pending
 * (reuse on "the same stream" is decided by handle value).
 *
 * spt_memory_stats fills a host array of 4: bytes held by live buffers,
 * bytes of idle cached blocks, hipMalloc calls so far and requests served
 * from idle blocks so far (all devices; hook-supplied memory not included).
 * Errors: SPT_E_INVALID_ARG (NULL).
 *
 * spt_empty_cache returns every idle block to the driver (waits for the
 * work ordered before each release, then hipFree).  Live buffers stay.
 * Errors: SPT_E_DEVICE.
 */
spt_status spt_memory_stats(int64_t *stats);
spt_status spt_empty_cache(void);

/* ---------------------------------------------------------------------- */
/* Encoding (Section III-C: linearized tensor, positions of l(p) bits).    */
/* ---------------------------------------------------------------------- */

/*
 * Build the linearized tensor of a COO tensor on the GPU.
 *   dims    host, nmodes mode lengths.
 *   coords  device, uint32 structure-of-arrays: coords[n * nnz + e] = i_n of nonzero e.
 *   vals    device, nnz FP32 values.
 *   layout  host, NULL for the default (ALTO) interleaving — level by level,
 *           modes of shorter bit length first, equal lengths in mode order —
 *           else layout_len == l(p) mode ids, layout[t] = mode whose next
 *           unused low bit becomes key bit t (the encoding matrix of the
 *           paper's environment state, Section III-C.1).
 * Keys are l(p)-bit integers (64-bit words, two when l(p) > 64), sorted
 * ascending by a stable LSD radix sort: equal keys (duplicate coordinates)
 * keep input order and stay separate elements.  The inputs are not kept.
 * Synchronises `stream` once (coordinate-range check, norm).
 * Errors: SPT_E_INVALID_ARG, SPT_E_TOO_MANY_BITS, SPT_E_BAD_LAYOUT,
 * SPT_E_INDEX_RANGE (no handle is created), SPT_E_OOM, SPT_E_DEVICE.
 */
spt_status spt_encode(const int64_t *dims, int nmodes, const uint32_t *coords, const float *vals,
                      int64_t nnz, const uint8_t *layout, int layout_len, void *stream,
                      spt_tensor *out);

/* Fill *info (host). */
spt_status spt_tensor_get_info(spt_tensor t, spt_tensor_info *info);

/*
 * Copy the encoded tensor out (device buffers, any may be NULL):
 *   keys  nnz * key_words uint64, element-major, low word first;
 *   vals  nnz FP32 in key order;  perm  nnz uint32, input index of each element.
 */
spt_status spt_tensor_export(spt_tensor t, uint64_t *keys, float *vals, uint32_t *perm, void *stream);

/* Decode every key back to coordinates: coords[n * nnz + j] (device, uint32 SoA). */
spt_status spt_tensor_decode(spt_tensor t, uint32_t *coords, void *stream);

/* Plan of the tensor (host copy). */
spt_status spt_tensor_get_plan(spt_tensor t, spt_plan *plan);

/*
 * Replace the plan.  The per-mode state built for the old plan is released
 * in stream order on `stream` (the caller orders this call after every use
 * of the tensor on other streams) and the tensor becomes unprepared: call
 * spt_tensor_prepare before the next spt_mttkrp.  Does not synchronise.
 */
spt_status spt_tensor_set_plan(spt_tensor t, const spt_plan *plan, void *stream);

#define SPT_PREPARE_SINGLE 1   /* per-mode plans of spt_mttkrp (and the tile dictionaries) */
#define SPT_PREPARE_BATCHED 2  /* per-mode plans of the batched launch (spt_mttkrp_batched) */

/*
 * Build the per-mode state MTTKRP needs under the tensor's plan, for every
 * mode: the SEGMENT plan (a counting pass and one emission pass over the
 * nonzeros: 2 B per nonzero plus 16 B per piece), the tile dictionaries of
 * the row cache (2 B per nonzero per mode plus 4 B per distinct (tile, row)
 * pair) and, under the TABLE strategy, that strategy's plan for `rank`
 * (the only rank-dependent plan).  `what` is a mask of SPT_PREPARE_*.  It is
 * derived from the encoding alone (Section III-C keeps one mode-agnostic
 * copy; this is an index over it) and kept until the plan changes or the
 * tensor is freed; preparing again is free.  Synchronises `stream` (the
 * sizes of the plans are read back).  1 <= rank <= SPT_MAX_RANK.
 * Errors: SPT_E_INVALID_ARG, SPT_E_OOM, SPT_E_DEVICE.
 */
spt_status spt_tensor_prepare(spt_tensor t, int rank, int what, void *stream);

/*
 * Release the handle in stream order on `stream`: the caller orders this
 * call after the tensor's last use (on `stream`, or on another stream that
 * `stream` waits for).  Does not synchronise.
 */
void spt_tensor_free(spt_tensor t, void *stream);

/* ---------------------------------------------------------------------- */
/* MTTKRP (Section II-B, Fig. 2).                                          */
/* ---------------------------------------------------------------------- */

/*
 * out = X_(mode) times the Khatri-Rao product of the other factors, i.e. for
 * every nonzero v at (i_0..i_{N-1}): out[i_mode, :] += v * prod_{k != mode}
 * factors[k][i_k, :].  FP32 inputs, FP32 accumulation (order unspecified).
 *   factors  host array of nmodes device pointers (factors[mode] is not read).
 *   out      device, I_mode x rank, OVERWRITTEN (rows without nonzeros are 0).
 * Asynchronous and free of synchronisation: host-side argument checks
 * only; the record workspace of the call is taken from the allocator hook and
 * released in stream order on `stream`, so calls on different streams over
 * one tensor may overlap.  The tensor must be prepared (spt_tensor_prepare,
 * SPT_PREPARE_SINGLE; under the TABLE strategy for this rank), else
 * SPT_E_INVALID_ARG.  1 <= rank <= SPT_MAX_RANK.
 */
spt_status spt_mttkrp(spt_tensor t, const float *const *factors, int rank, int mode, float *out,
                      void *stream);

/*
 * spt_mttkrp for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same arguments, result and kernels, with the record workspace of the
 * SEGMENT strategy in a fixed device array of the library
 * (SPT_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends) instead of
 * memory taken from the allocator.  It calls no allocating routine.  The
 * tensor must be prepared (SPT_PREPARE_SINGLE) and its plan for `mode` must
 * be SEGMENT (or AUTO), DIRECT or REGROUP; a workspace above the maximum
 * (records x (8 + 4 rank) bytes, about 0.1 records per nonzero) is rejected
 * with SPT_E_INVALID_ARG.  Every call on one GPU shares the array: calls that
 * overlap on one GPU (on different streams or threads) race, so the caller
 * orders them.  Asynchronous, free of synchronisation.
 */
#define SPT_NOALLOC_SCRATCH_BYTES (64u << 20)
spt_status spt_mttkrp_noalloc(spt_tensor t, const float *const *factors, int rank, int mode, float *out,
                              void *stream);

/*
 * FP64 values for the FP64 MTTKRP (the paper's precision: FP64 values and
 * factors, 64-bit keys; Section IV-A).  vals: device, nnz FP64 values in the
 * caller's input order (the order of spt_encode's coords); they are copied
 * into key order.  Replaces earlier FP64 values; spt_autotune keeps them.
 * Asynchronous.  Errors: SPT_E_INVALID_ARG, SPT_E_OOM, SPT_E_DEVICE.
 */
spt_status spt_tensor_attach_f64(spt_tensor t, const double *vals, void *stream);

/*
 * spt_mttkrp in FP64: out[i_mode, :] += v * prod_{k != mode} factors[k][i_k, :]
 * with FP64 values (spt_tensor_attach_f64), FP64 factors (host array of
 * device pointers, row-major I_k x rank) and FP64 accumulation into out
 * (device, I_mode x rank, overwritten).  It runs the tensor's SEGMENT plan
 * (the mode's strategy must be SEGMENT or AUTO; the tensor prepared) with
 * FP64 records.  Asynchronous and free of synchronisation.
 * 1 <= rank <= SPT_MAX_RANK.  Errors: SPT_E_INVALID_ARG, SPT_E_OOM, SPT_E_DEVICE.
 */
spt_status spt_mttkrp_f64(spt_tensor t, const double *const *factors, int rank, int mode, double *out,
                          void *stream);

/* ---------------------------------------------------------------------- */
/* CP-ALS (Section II-B; the update follows Kolda and Bader's ALS).        */
/* ---------------------------------------------------------------------- */

/*
 * Run up to max_iters CP-ALS iterations from the factors the caller passes.
 * Per iteration, for n = 0..N-1: M = MTTKRP(n); V = Hadamard product of the
 * Grams of the other factors (FP64, Gram via FP64 MFMA); factor n = M V^-1
 * (FP64 Cholesky, ridge retry if V is not positive definite), columns
 * normalised to unit 2-norm with the norms in lambda, rounded to FP32.
 * Then fit = 1 - |X - Xhat| / |X| in FP64 (direct residual over the
 * nonzeros once 1 - fit < 1e-2).  Stops after max_iters, or earlier when
 * tol > 0 and |fit - previous fit| < tol (previous fit starts at 0).
 *   factors  host array of nmodes device pointers, in: initial, out: normalised.
 *   lambda   device, rank FP64 (out).
 *   fit_out, iters_out  host (out).
 * The iterations run on library-owned copies of the factors: factors and
 * lambda are written only when the call returns SPT_OK.  Prepares the
 * tensor for `rank` if needed.  Synchronises `stream` once per iteration
 * (and while preparing).  1 <= rank <= SPT_MAX_ALS_RANK.
 * Errors: SPT_E_INVALID_ARG (also when |X| = 0), SPT_E_NOT_SPD, SPT_E_OOM, SPT_E_DEVICE.
 */
spt_status spt_cp_als(spt_tensor t, int rank, int max_iters, double tol, float *const *factors,
                      double *lambda, double *fit_out, int *iters_out, void *stream);

/*
 * One ALS mode update on dense operands (the solve step of spt_cp_als, for
 * callers that form M themselves): V = Hadamard product of grams[k] over
 * k != mode (FP64), Cholesky V = L L^T with the ridge retry (V + d_k I,
 * d_k = 1e-12 tr(V)/R * 1e3^(k-1) on retry k = 1..3), C = M V^-1 with
 * columns normalised to unit 2-norm, their norms in lambda (a zero column
 * keeps norm 1), rounded to FP32.  Kolda and Bader's ALS, which Section II-B
 * cites for CP-ALS.
 *   grams    device, nmodes x rank x rank FP64 (grams[mode] is not read).
 *   M        device, rows x rank FP32 (the mode's MTTKRP output).
 *   C        device out, rows x rank FP32 (may alias nothing else).
 *   lambda   device out, rank FP64.
 *   retries_out  host out: ridge retries taken (0 when V was positive definite).
 * Synchronises `stream` once (the factorisation status).  C, lambda and
 * retries_out are written only on SPT_OK.  1 <= rank <= SPT_MAX_ALS_RANK.
 * Errors: SPT_E_INVALID_ARG, SPT_E_NOT_SPD (V + d_3 I still not positive
 * definite, or not finite), SPT_E_OOM, SPT_E_DEVICE.
 */
spt_status spt_als_update(const double *grams, int nmodes, int mode, int rank, const float *M, int64_t rows,
                          float *C, double *lambda, int *retries_out, void *stream);

/* ---------------------------------------------------------------------- */
/* Batches of independent tensors (many decompositions, Section IV-D).     */
/* ---------------------------------------------------------------------- */

/*
 * Mode-`mode` MTTKRP of every tensor in the batch with one SEGMENT launch
 * over all tensors' tiles (2048 nonzeros each), one radix sort of all
 * records and one reduction; tensors with nmodes <= mode are skipped and
 * their outs[b] is not touched.  factors[b] is a host array of device
 * pointers for tensor b, outs[b] its output (I_mode x ranks[b], overwritten),
 * 1 <= ranks[b] <= 64.  Every tensor must be prepared with
 * SPT_PREPARE_BATCHED (else SPT_E_INVALID_ARG).  Asynchronous and free of
 * synchronisation: the call's workspaces are released in stream order.
 */
spt_status spt_mttkrp_batched(const spt_tensor *ts, int count, const float *const *const *factors,
                              const int *ranks, int mode, float *const *outs, void *stream);

/*
 * CP-ALS of every tensor of the batch, advanced in lock step with the same
 * update and fit as spt_cp_als: per mode index, one batched MTTKRP (as
 * spt_mttkrp_batched, into one concatenated output) and one launch each of
 * the batched Gram, FP64 solve and apply kernels (one workgroup per tensor;
 * apply over all row blocks); then one fit launch for all tensors.  Tensors
 * stop individually (max_iters, tol) and leave the batch.  factors[b] is a
 * host array of device pointers (in: initial, out: normalised), lambdas[b]
 * a device array of ranks[b] doubles, fits[b] and iters[b] host outputs.
 * Synchronises once per iteration (plus once when a fit takes the direct
 * residual; plus the batched plans of tensors not yet prepared with
 * SPT_PREPARE_BATCHED).  The iterations run on library-owned copies:
 * factors and lambdas are written only when the call returns SPT_OK.
 * Errors: as spt_cp_als, for the first failing tensor.
 */
spt_status spt_cp_als_batched(const spt_tensor *ts, int count, const int *ranks, int max_iters,
                              double tol, float *const *const *factors, double *const *lambdas,
                              double *fits, int *iters, void *stream);

/* ---------------------------------------------------------------------- */
/* Autotuner (the measured search over encodings of Section III-C).        */
/* ---------------------------------------------------------------------- */

/* Outcome of spt_autotune (host).  Times are all-mode MTTKRP milliseconds,
 * each mode at its best plan for the layout. */
typedef struct {
    double best_ms;      /* the winning layout (the tensor holds it on return) */
    double alto_ms;      /* the default (ALTO) layout: alto_ms / best_ms is the paper's reward */
    double start_ms;     /* the layout the tensor had on entry */
    int candidates;      /* layouts measured, cache hits included */
    int random_samples;  /* of which drawn uniformly from the interleaving space */
    int cache_hits;      /* of which answered by the measurement cache */
    int pad;
} spt_tune_result;

/*
 * Measured search over the tensor's bit layout (the interleavings of Section
 * III-C, counted by Eq. (1)) and the per-mode plan (strategy, tile), with the
 * paper's reward: all-mode MTTKRP time against the default (ALTO) layout.
 * Candidates: the tensor's layout, the ALTO layout, `random_samples` layouts
 * drawn uniformly from the interleaving space (seeded by `seed`), then a hill
 * climb of adjacent-bit exchanges from the best so far, within budget_ms of
 * wall time.  Each layout is measured with every mode at its best plan and
 * cached per (mode lengths, nnz, rank, layout, content fingerprint).
 * Re-encodes *t in place when another layout wins (export keeps naming the
 * caller's input order) and leaves it prepared (SPT_PREPARE_SINGLE) for
 * `rank` under the winning plan.  Synchronises.
 */
spt_status spt_autotune(spt_tensor *t, const float *const *factors, int rank, double budget_ms, int random_samples,
                        uint64_t seed, spt_tune_result *result, void *stream);

/* Outcome of spt_autotune_batched (host). */
typedef struct {
    double ms[3];           /* all-mode batched MTTKRP milliseconds at batch tiles 1024, 2048, 4096
                               (0: that tile does not fit the batch's mode count) */
    int best_tile;          /* the tile every member holds on return */
    int layouts_tuned;      /* members whose layout was searched */
    double layout_speedup;  /* geometric mean over those members of start_ms / best_ms */
} spt_batch_tune_result;

/*
 * Autotuner for batches (the measured search of spt_autotune, applied to the
 * encoding and tile of batched launches).  With layout_budget_ms > 0 every
 * member's bit layout is searched first, as spt_autotune does for one tensor
 * (its own factors[b] and ranks[b], seed + b, re-encoding ts[b] in place).
 * Then the all-mode batched MTTKRP (spt_mttkrp_batched over every mode) is
 * timed at each batched tile that fits the batch's mode count, and every
 * member's plan takes the fastest (plan batch_tile); members are left
 * prepared for batched launches at it (SPT_PREPARE_BATCHED).
 *   ts       host array of count handles (in/out: a re-encoded member keeps
 *            its handle).
 *   factors  host array of count host arrays of device pointers.
 * Synchronises.  Errors: SPT_E_INVALID_ARG, SPT_E_OOM, SPT_E_DEVICE.
 */
spt_status spt_autotune_batched(spt_tensor *ts, int count, const float *const *const *factors, const int *ranks,
                                double layout_budget_ms, int random_samples, uint64_t seed,
                                spt_batch_tune_result *result, void *stream);

/* ---------------------------------------------------------------------- */
/* Serving: continuous batching of CP-ALS requests.                        */
/* ---------------------------------------------------------------------- */

typedef struct spt_server_s *spt_server;

typedef struct {
    int nmodes;
    int64_t dims[SPT_MAX_MODES];
    int64_t nnz;
    const uint32_t *coords;      /* host, SoA nmodes x nnz (copied at submit) */
    const float *vals;           /* host, nnz (copied at submit) */
    const float *const *init;    /* host array of nmodes host pointers, I_n x rank FP32 (copied) */
    int rank;                    /* 1..SPT_MAX_ALS_RANK */
    int max_iters;
    double tol;
} spt_request;

typedef struct {
    spt_status status;
    double fit;
    int iters;
    double t_arrive, t_admit, t_done;   /* seconds on the server's monotonic clock */
} spt_result;

/*
 * Create a server that owns one HIP stream and a worker thread.  Requests
 * are admitted while their device bytes (encoded tensor, factors, MTTKRP
 * output, Grams, workspace) fit hbm_budget_bytes and fewer than max_slots
 * are active; every admitted request joins the running set at the next
 * iteration boundary, so requests that arrive while others run share the
 * GPU (continuous batching).
 */
spt_status spt_server_create(size_t hbm_budget_bytes, int max_slots, spt_server *out);

/* Enqueue a copy of *req; returns a ticket (host). */
spt_status spt_server_submit(spt_server s, const spt_request *req, uint64_t *ticket);

/*
 * Wait for a ticket; on completion copies the normalised factors into
 * factors_out (host array of nmodes host pointers, may be NULL) and lambda
 * (host, rank doubles, may be NULL).  timeout_s < 0 waits forever.
 * Returns SPT_E_BUSY on timeout.
 */
spt_status spt_server_wait(spt_server s, uint64_t ticket, double timeout_s, spt_result *res,
                           float *const *factors_out, double *lambda);

/* Server clock (seconds), for callers that time arrivals. */
double spt_server_now(spt_server s);

/*
 * The server's admission policy run against a modelled executor, on the host
 * only (capacity planning; no device work): request i of `bytes[i]` device
 * bytes arrives at arrive[i] (host array, sorted) and, once admitted, runs for
 * service[i] seconds.  Admission is in arrival order while a slot is free and
 * the bytes fit the unused budget; a request above the whole budget is
 * rejected on reaching the head of the queue (status SPT_E_OOM).  Host
 * outputs: admit_out[i], done_out[i] (seconds) and status_out[i].
 */
spt_status spt_server_simulate(size_t hbm_budget_bytes, int max_slots, int count, const size_t *bytes,
                               const double *arrive, const double *service, double *admit_out, double *done_out,
                               int *status_out);

/* Stop accepting, finish active work, join the worker and free everything. */
void spt_server_destroy(spt_server s);

/* ---------------------------------------------------------------------- */

/* ---------------------------------------------------------------------- */
/* Instrumentation.                                                        */
/* ---------------------------------------------------------------------- */

/*
 * on != 0: from now on bracket every MTTKRP call (spt_mttkrp, and the
 * MTTKRP steps inside spt_cp_als) with two HIP events on its stream.  Any
 * call clears what was recorded.  Adds two event records per call.
 */
spt_status spt_profile_enable(int on);

/*
 * Host out: ms[n] = summed GPU time of the recorded MTTKRP calls of mode n,
 * launches[n] = their count (arrays of SPT_MAX_MODES).  Waits for the
 * recorded events.
 */
spt_status spt_profile_read(double *ms, int64_t *launches);

/* Message for the last non-OK status on this thread ("" if none). */
const char *spt_last_error(void);

/* Library version string. */
const char *spt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SPT_H */
