// Internal declarations shared by the library's HIP and host sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "spt.h"  // include/ is on the include path

namespace spt {

constexpr int kMaxModes = SPT_MAX_MODES;
constexpr int kMaxRuns = 160;          // l(p) <= 128 bits plus splits at 32-bit word boundaries
constexpr uint32_t kNoRow = 0xFFFFFFFFu;
constexpr uint32_t kDictMiss = 0x80000000u;  // row-cache entry flag of a global row (global rows stay below it)
constexpr int kDictTile = 4096;             // tile of the dictionaries and the row-cached kernel
#ifndef SPT_DICT_LDS_KB
#define SPT_DICT_LDS_KB 80
#endif
constexpr size_t kDictLdsBudget = (size_t)SPT_DICT_LDS_KB * 1024;  // LDS of one row-cached workgroup
constexpr int kDictMinCap = 16;

// A maximal group of consecutive coordinate bits that land on consecutive key
// bits inside one 32-bit word of the key: coordinate bits [cpos, cpos+len) of
// mode n  <->  bits [kpos, kpos+len) of 32-bit key word `word`.  Packed as
// word | kpos << 8 | cpos << 16 | len << 24.
__host__ __device__ inline uint32_t pack_run(int word, int kpos, int cpos, int len) {
    return (uint32_t)word | ((uint32_t)kpos << 8) | ((uint32_t)cpos << 16) | ((uint32_t)len << 24);
}

// Bit map between coordinates and keys, passed by value to kernels.
// Runs of mode n that live in 32-bit key word w are run[rb[n][w] .. rb[n][w+1]).
struct Codec {
    int nmodes;
    int key_words;  // 64-bit words per key: 1 or 2
    int nruns;
    int pad;
    uint8_t rb[kMaxModes][5];
    uint32_t run[kMaxRuns];
};

// The default (ALTO) layout of modes with bit lengths lbits.
void default_layout(int nmodes, const int *lbits, uint8_t *layout);

// Build the codec of a layout (layout[t] = mode feeding key bit t).
void make_codec(int nmodes, const int *lbits, const uint8_t *layout, int lp, Codec *c);

// ---------------------------------------------------------------- device memory
void *dev_alloc(size_t bytes, hipStream_t s);
void dev_free(void *p, hipStream_t s);
spt_status memory_stats(int64_t *stats);
spt_status empty_cache();

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
spt_status fail(spt_status st, const std::string &msg);
spt_status hip_fail(hipError_t e, const char *what);

#define SPT_HIP(call)                                                   \
    do {                                                                \
        hipError_t e__ = (call);                                        \
        if (e__ != hipSuccess) return ::spt::hip_fail(e__, #call);      \
    } while (0)

// ---------------------------------------------------------------- tensor handle
// Resolved launch plan of one mode at one rank (plan.cpp).
struct ModePlan {
    int valid = 0;
    int rank = 0;
    int strategy = -1;       // resolved: DIRECT, REGROUP, TABLE or PRIV
    int cap = 0, hbits = 0, stride = 0, rs = 0, npass = 1, ts = 512, nwg = 0;
    int64_t sub_per_wg = 0;
    int64_t records = 0;     // TABLE / SEGMENT: records written per call
    int64_t *rec_off = nullptr;  // TABLE: device, nwg offsets
    // SEGMENT plan: per nonzero its position in the tile's row-grouped order;
    // per piece (tile-major, pl_off[tile] .. pl_off[tile + 1]) its
    // start | length << 16, row and record (records of one row contiguous):
    // packed as 4 u32 {desc, row, record, 0} per piece in pl_piece (one
    // tensor), in the three arrays pl_desc / pl_row / pl_dest (batched plans)
    uint16_t *pl_pos = nullptr;
    int64_t *pl_off = nullptr;
    uint32_t *pl_piece = nullptr;
    uint32_t *pl_desc = nullptr, *pl_row = nullptr, *pl_dest = nullptr;
};

struct Tensor {
    int nmodes = 0;
    int64_t nnz = 0;
    int64_t dims[kMaxModes] = {};
    int lbits[kMaxModes] = {};
    int lp = 0;
    int key_words = 1;
    uint8_t layout[SPT_MAX_KEY_BITS] = {};
    Codec codec{};
    uint64_t *lo = nullptr;   // nnz key words (bits 0..63)
    uint64_t *hi = nullptr;   // nnz key words (bits 64..127), only when key_words == 2
    float *vals = nullptr;    // nnz values in key order
    double *vals64 = nullptr; // nnz FP64 values in key order (spt_tensor_attach_f64), else null
    uint32_t *perm = nullptr; // input index of each element
    double norm_x2 = 0.0;
    spt_plan plan{};
    ModePlan mplan[kMaxModes];
    // batched SEGMENT plan per mode (tiles of bplan[n].ts nonzeros; stream-ordered allocations)
    ModePlan bplan[kMaxModes];
    // tile dictionaries (tiles of kDictTile, built by spt_tensor_prepare): per mode slot[nnz] u16,
    // row[distinct (tile, row) pairs] u32, off[ntiles + 1]
    uint16_t *dict_slot[kMaxModes] = {};
    uint32_t *dict_row[kMaxModes] = {};
    int64_t *dict_off[kMaxModes] = {};
    int dict_state = 0;  // -1: not applicable, or a build failed
};

// plan.cpp
int device_cus();
// plan of `mode` at `rank`; SEGMENT/TABLE plans are built (synchronising s)
// only when `build` is set, else a missing plan is SPT_E_INVALID_ARG
spt_status resolve_plan(Tensor *t, int mode, int rank, hipStream_t s, ModePlan **out, bool build);
// every mode's plan at `rank` and the tile dictionaries (synchronises s)
spt_status prepare_single(Tensor *t, int rank, hipStream_t s);
// mode-`mode` MTTKRP into out (overwritten), per the tensor's prepared plan
// A caller-owned record workspace: an MTTKRP call whose SEGMENT records fit
// writes them there instead of allocating (a driver that calls every mode in
// turn on one stream allocates once).
struct RecordWs {
    uint64_t *row = nullptr;
    float *val = nullptr;
    int64_t records = 0;    // capacity in records
    int64_t val_floats = 0;  // capacity of val
};
// the largest record count over the tensor's modes under its prepared plans
int64_t max_plan_records(const Tensor *t);
spt_status run_mttkrp(Tensor *t, const float *const *factors, int rank, int mode, float *out, hipStream_t s,
                      const RecordWs *ws = nullptr);
// FP64 MTTKRP (FP64 values, factors, records and accumulation) on the SEGMENT plan
spt_status run_mttkrp_f64(Tensor *t, const double *const *factors, int rank, int mode, double *out, hipStream_t s);
// the same with the record workspace in the library's fixed device array
spt_status run_mttkrp_noalloc(Tensor *t, const float *const *factors, int rank, int mode, float *out, hipStream_t s);
size_t noalloc_scratch_bytes();
// The release functions free in stream order on s (after the work already
// ordered on s); none synchronises.
void release_plans(Tensor *t, hipStream_t s);
void release_dict(Tensor *t, hipStream_t s);
void tensor_release(Tensor *t, hipStream_t s);
void release_mode_plan(Tensor *t, int mode, hipStream_t s);
void release_batch_plan(Tensor *t, int mode, hipStream_t s);
bool seg_tile_ok(int tile, int nmodes);
bool priv_feasible(const Tensor *t, int mode, int rank);
spt_status profile_enable(int on);
spt_status profile_read(double *ms, int64_t *launches);

// ---------------------------------------------------------------- kernels (launchers)
// encode.hip
spt_status launch_encode(Tensor *t, const uint32_t *coords, const float *vals, hipStream_t s);
spt_status launch_decode(const Tensor *t, uint32_t *coords, hipStream_t s);
spt_status launch_export(const Tensor *t, uint64_t *keys, hipStream_t s);
// Stable LSD radix sort of n 64-bit keys over their low nbits bits in
// caller-owned buffers (see encode.hip).
size_t sort_ws_counts(int64_t n);
spt_status launch_gather_u32(const uint32_t *src, const uint32_t *idx, uint32_t *out, int64_t n, hipStream_t s);
// dst[idx[j]] = src[j]
spt_status launch_scatter_u32(const uint32_t *src, const uint32_t *idx, uint32_t *dst, int64_t n, hipStream_t s);
// exclusive prefix sum of n u32 values (totals below 2^32); ws of exclusive_scan_ws(n) u32
size_t exclusive_scan_ws(int64_t n);
spt_status launch_exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *ws, hipStream_t s);
spt_status sort_u64_keys_ws(uint64_t *keys, uint64_t *keys2, uint32_t *idx_a, uint32_t *idx_b, uint32_t *counts,
                            int64_t n, int nbits, uint64_t **sorted_out, uint32_t **idx_out, hipStream_t s);

// mttkrp.hip
struct MttkrpArgs {
    const uint64_t *lo;
    const uint64_t *hi;
    const float *vals;
    int64_t nnz;
    int nmodes;
    int mode;
    int rank;
    int tile;
    const float *f[kMaxModes];
    uint32_t frows[kMaxModes];  // rows of each factor (clamped to 2^32 - 1)
    float *out;
    // SEGMENT strategy: record output
    uint64_t *rec_row;
    float *rec_val;
    const int64_t *rec_off;   // per tile, ntiles + 1 entries
    // SEGMENT plan (see ModePlan)
    const uint16_t *pl_pos;
    const int64_t *pl_off;
    const uint32_t *pl_piece;  // one tensor: 4 u32 per piece, 16-byte aligned
    const uint32_t *pl_desc, *pl_row, *pl_dest;  // batched members
    int64_t rec_cap;          // records the plan laid out (writes beyond are dropped)
    // row cache (SEGMENT, tiles of kDictTile): the tile dictionaries of the
    // non-output modes in order (o-th non-output mode), and the cached rows
    // per mode (0: no cache)
    const uint16_t *d_slot[kMaxModes - 1];
    const uint32_t *d_row[kMaxModes - 1];
    const int64_t *d_off[kMaxModes - 1];
    int d_cap;
    Codec codec;
};
spt_status launch_fill_zero(float *p, int64_t n, hipStream_t s);
MttkrpArgs make_args(const Tensor *t, const float *const *factors, int rank, int mode, float *out, int tile);
spt_status launch_mttkrp(const MttkrpArgs &a, int strategy, hipStream_t s);
bool seg_tile_ok(int tile, int nmodes);
// per tile: pieces | distinct rows << 32
spt_status launch_count_pieces(const MttkrpArgs &a, int64_t *counts, hipStream_t s);
// outputs of the plan-emission pass (a.pl_off must hold the piece offsets)
struct PlanOut {
    const int64_t *pair_off;  // per tile, distinct (tile, row) pairs
    uint16_t *pos;            // nnz
    uint32_t *desc, *prow, *ppair, *psub;  // per piece
    uint64_t *pair_key;       // per pair: its row (sort key)
    uint32_t *pair_np;        // per pair: its pieces
};
spt_status launch_emit_plan(const MttkrpArgs &a, const PlanOut &o, hipStream_t s);
// packed[k] = {desc[k], prow[k], first record of piece k's pair + its index, 0}
spt_status launch_piece_pack(const uint32_t *ppair, const uint32_t *psub, const uint32_t *pair_first,
                             const uint32_t *desc, const uint32_t *prow, uint32_t *packed, int64_t n, hipStream_t s);
spt_status launch_mttkrp_seg(const MttkrpArgs &a, hipStream_t s);
// mttkrp_f64.hip
bool f64_tile_ok(int tile, int nmodes);
spt_status launch_mttkrp_seg_f64(const MttkrpArgs &a, const double *vals64, const double *const *F, double *rec_val,
                                 hipStream_t s);
spt_status launch_reduce_records_f64(const uint64_t *srow, const double *rec, int64_t P, int R, int64_t rows,
                                     double *out, hipStream_t s);
spt_status launch_gather_f64(const double *src, const uint32_t *idx, double *dst, int64_t n, hipStream_t s);
// Tile dictionary of mode a.mode (tiles of kDictTile): off from the counting
// pass (distinct rows per tile, exclusive prefix), rows and slots written.
spt_status launch_emit_dict(const MttkrpArgs &a, const int64_t *off, uint32_t *rows, uint16_t *slots, hipStream_t s);
// Rows of each non-output factor the row-cached kernel keeps in LDS (0: the
// cache does not fit).
int dict_cap(int nmodes, int rank);

// Batched SEGMENT MTTKRP: every tensor's tiles (one tile size per launch:
// 1024, 2048 or 4096 nonzeros) in one persistent launch, each with the
// tensor's batched plan (a.pl_*); records carry rows of the batch's
// concatenated output (row_base + row) and go to rec_base + the plan's
// record, so the batch's records stay grouped by row.
constexpr int kBatchTileDefault = 2048;
// the batched tile of a tensor: its plan's batch_tile, else the default
int batch_tile_of(const Tensor *t);
struct SegItem {
    MttkrpArgs a;        // a.pl_*: the tensor's batched plan for this mode; a.rec_cap its records
    int64_t first_tile;  // prefix of tiles over the batch
    int64_t rec_base;    // first record of this tensor
    int64_t row_base;    // first row of this tensor in the concatenated output
};
bool seg_batch_fits(int nmodes_max, int tile);
// per global tile: pieces | distinct rows << 32
spt_status launch_count_pieces_batched(const SegItem *items, int count, int64_t total_tiles, int nmodes_max, int tile,
                                       int64_t *counts, hipStream_t s);
spt_status launch_emit_plan_batched(const SegItem *items, int count, int64_t total_tiles, int nmodes_max, int tile,
                                    const int64_t *gpiece_off, const int64_t *gpair_off, uint32_t *ppair,
                                    uint32_t *psub, uint64_t *pair_key, uint32_t *pair_np, hipStream_t s);
spt_status launch_piece_dest_batched(const SegItem *items, int count, const int64_t *piece_base, const uint32_t *ppair,
                                     const uint32_t *psub, const uint32_t *pair_first, int64_t n, hipStream_t s);
// next_tile: a device counter (8 bytes) the launch zeroes and the workgroups pull tiles from
spt_status launch_mttkrp_seg_batched(const SegItem *items, int count, int64_t total_tiles, int nmodes_min,
                                     int nmodes_max, int tile, int ld, bool vec4, uint64_t *rec_row, float *rec_val,
                                     unsigned long long *next_tile, hipStream_t s);

// Batched dense steps (dense.hip): one workgroup per item, except apply
// (a grid over the items' row blocks).
constexpr int kGramSliceRows = 2048;  // rows per workgroup of the batched Gram
struct GramItem {
    const float *C;   // rows x rank, leading dimension ld
    int64_t rows;
    int ld, rank;
    double *G;        // rank x rank (out)
    int64_t first_slice, nslices;  // the item's row slices in the launch (gram_slices(rows) of them)
};
int64_t gram_slices(int64_t rows);
size_t gram_batched_ws_bytes(int64_t total_slices, int rmax);
struct SolveItem {
    const double *grams;  // nmodes x rank x rank
    const double *gram_m; // rank x rank Gram of the MTTKRP output
    double *S, *lambda;
    int *status;          // nmodes entries; entry `mode` is written
    double *gram_new;     // rank x rank: Gram of the updated factor (the member's slot of `mode`)
    int nmodes, rank;
};
struct ApplyItem {
    const float *M;       // rows x rank, leading dimension ldm
    const double *S;
    float *C;             // rows x rank (out)
    const double *lambda;
    double *inner;        // per-block inner-product partials, or null
    int64_t rows, first_block;
    int ldm, rank;
};
struct FitItem {
    const double *grams, *lambda, *inner;
    double *out;          // 4 doubles: fit, |Xhat|^2, <X, Xhat>, residual^2
    double norm_x2;
    int nmodes, rank, nparts, pad;
};
spt_status launch_gram_batched(const GramItem *items, int count, int64_t total_slices, int rmax, double *work,
                               hipStream_t s);
spt_status launch_solve_prep_batched(const SolveItem *items, int count, int mode, hipStream_t s);
int apply_rows_per_launch_block(int rmax);
spt_status launch_apply_batched(const ApplyItem *items, int count, int64_t total_blocks, int rmax, hipStream_t s);
spt_status launch_fit_batched(const FitItem *items, int count, hipStream_t s);

// batch.cpp: lock-step CP-ALS of many tensors.
struct Member {
    Tensor *t = nullptr;
    int R = 0;
    float *F[kMaxModes] = {};   // device factors (in: initial, out: normalised)
    double *lambda = nullptr;   // device, R doubles
    int max_iters = 0;
    double tol = 0.0;
    // results
    double fit = 0.0, fit_prev = 0.0;
    int iters = 0;
    bool done = false;
    spt_status err = SPT_OK;
    // engine-owned device state: Grams of every mode, Gram of M, solve matrix
    bool fresh = true;
    void *state = nullptr;
    double *grams = nullptr, *gram_m = nullptr, *S = nullptr;
    void *user = nullptr;
};

struct ModeItems {
    int count = 0, ld = 0, rmax = 0;
    bool vec4 = true;
    int64_t tiles = 0, records = 0, rows = 0, blocks = 0;
    size_t seg_off = 0, gm_off = 0, sv_off = 0, ap_off = 0;
    std::vector<int> member_idx;
    std::vector<SegItem> seg_v;
    std::vector<GramItem> gm_v;
    int64_t gm_slices = 0;
    std::vector<SolveItem> sv_v;
    std::vector<ApplyItem> ap_v;
};

// Grow-only device buffer; a smaller buffer is released in stream order on
// the stream that asks for a larger one (no synchronisation).
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    void *get(size_t need, hipStream_t s) {
        if (need <= bytes && p) return p;
        dev_free(p, s);
        p = nullptr;
        bytes = 0;
        need = need < 256 ? 256 : need;
        p = dev_alloc(need, s);
        if (p) bytes = need;
        return p;
    }
    void release(hipStream_t s) {
        dev_free(p, s);
        p = nullptr;
        bytes = 0;
    }
};

// record and sort buffers of the batched MTTKRP
struct BatchMttkrpWs {
    DevBuf rec_row, rec_val, counter;
    void release(hipStream_t s) {
        rec_row.release(s);
        rec_val.release(s);
        counter.release(s);
    }
};
spt_status run_mttkrp_batched_mode(const SegItem *d_items, int count, int64_t total_tiles, int nmodes_min, int nmodes_max,
                                   int tile, int64_t records, int64_t rows, int ld, bool vec4, float *M_all,
                                   BatchMttkrpWs &ws, hipStream_t s);
// batched plans of `mode` at `tile` for the tensors that lack them (a plan
// at another tile is released and rebuilt); synchronises s when it builds
spt_status ensure_batch_plans(const std::vector<Tensor *> &ts, int mode, int tile, hipStream_t s);
// every mode's batched plan of one tensor (synchronises s)
spt_status prepare_batched(Tensor *t, hipStream_t s);
// host-to-device copy through a pinned staging ring (asynchronous)
spt_status upload_staged(void *dst, const void *src, size_t bytes, hipStream_t s);

class BatchEngine {
public:
    explicit BatchEngine(hipStream_t s);
    ~BatchEngine();
    BatchEngine(const BatchEngine &) = delete;
    BatchEngine &operator=(const BatchEngine &) = delete;
    // joins at the next step (computes the initial Grams then)
    spt_status add(Member *m);
    // leaves now (the stream is synchronised first)
    void remove(Member *m);
    // one CP-ALS iteration of every active member; synchronises the stream.
    // *before_kernels (if given) is set when a failure came before any kernel
    // of the step was launched (while re-planning for changed members).
    spt_status step(bool *before_kernels = nullptr);
    // remove the members marked done from the batch (their state is released)
    void drop_done();
    bool any_active() const;
    const std::vector<Member *> &members() const { return members_; }

private:
    spt_status rebuild();
    void release_buffers();
    void free_member_state(Member *m);
    hipStream_t s_;
    std::vector<Member *> members_, active_;
    bool dirty_ = true;
    int nmodes_max_ = 0, nmodes_min_ = 0;
    std::vector<ModeItems> modes_;
    char *d_items_ = nullptr;
    size_t fit_off_ = 0, init_off_ = 0;
    int init_count_ = 0, init_rmax_ = 0;
    int64_t init_slices_ = 0;
    DevBuf gram_ws_;  // partial Grams of the batched Gram launches
    DevBuf items_buf_, M_buf_, fit_buf_, status_buf_, inner_buf_, resid_buf_, resid_items_buf_;
    std::vector<char> blob_;  // host image of the item arrays (kept until the next upload)
    float *M_all_ = nullptr;
    double *fit_all_ = nullptr, *inner_all_ = nullptr, *resid_ = nullptr;
    int *status_all_ = nullptr;
    std::vector<double> hfit_;
    std::vector<int> hstat_;
    BatchMttkrpWs ws_;
    int tile_ = kBatchTileDefault;  // batched tile of the current members
};


// mttkrp_table.hip: persistent-workgroup LDS accumulation (see that file).
struct TableArgs {
    MttkrpArgs a;
    int cap;      // accumulator rows (TABLE) or output rows (PRIV)
    int hbits;    // log2 of the accumulator hash index size (TABLE)
    int stride;   // floats per accumulator row (columns + 1 padding)
    int rs;       // PRIV: columns per pass
    int ts;       // nonzeros per sub-tile: 256 or 512
    int pad;
    int64_t sub_per_wg;
    uint64_t *rec_row;        // TABLE: record rows
    float *rec_val;           // TABLE: records [P][R]; PRIV: partials [W][rows][R]
    const int64_t *rec_off;   // TABLE: first record of each workgroup
    int64_t *rec_cnt;         // counting pass: records of each workgroup
};
size_t table_lds_needed(int nmodes, int ts, int cap, int hbits, int stride, bool priv, bool with_acc);
spt_status launch_table_count(const TableArgs &t, int nwg, hipStream_t s);
spt_status launch_table(const TableArgs &t, int nwg, hipStream_t s);
spt_status launch_priv(const TableArgs &t, int nwg, int npass, hipStream_t s);
spt_status launch_reduce_priv(const float *part, int nwg, int64_t rows, int R, float *out, hipStream_t s);
spt_status launch_reduce_records(const uint64_t *srow, const uint32_t *sidx, const float *rec_val, int64_t P, int R,
                                 int64_t rows, float *out, hipStream_t s);

// residual over the nonzeros (direct fit): out2[0] += sum (v - xhat)^2, out2[1] += sum xhat^2
spt_status launch_resid(const MttkrpArgs &a, const double *lam, double *partials, int nparts, hipStream_t s);
// the same for many tensors in one launch: item b's tiles (of kResidTile
// nonzeros; a.tile must be kResidTile) start at first_tile of the launch and
// write 2 doubles each to partials[2 * local tile]
constexpr int kResidTile = 1024;
struct ResidItem {
    MttkrpArgs a;
    const double *lambda;
    double *partials;
    int64_t first_tile;
};
spt_status launch_resid_batched(const ResidItem *items, int count, int64_t total_tiles, int nmodes_max, int rmax,
                                bool vec4, hipStream_t s);
// the direct fit of many tensors, one workgroup each (as launch_fit_direct)
struct FitDirectItem {
    const double *parts;
    double *out;
    double norm_x2;
    int64_t nparts;
};
spt_status launch_fit_direct_batched(const FitDirectItem *items, int count, hipStream_t s);

// dense.hip
spt_status launch_gram(const float *C, int64_t rows, int rank, double *G, double *work, size_t work_bytes,
                       hipStream_t s);
size_t gram_work_bytes(int64_t rows, int rank);
// solve preparation: V = Hadamard of grams[k != mode]; Cholesky with ridge; W = V^-1;
// lambda_r = sqrt((W Gm W)_rr) (1 if 0); S = W diag(1/lambda).  status_out: 0 ok, >0 ridge retries, <0 failure.
// gram_new (or null): the Gram S^T Gm S of the updated factor M S, in FP64 (may be grams + mode * rank^2).
spt_status launch_solve_prep(const double *grams, int nmodes, int mode, int rank, const double *gram_m,
                             double *S, double *lambda, int *status_out, double *gram_new, hipStream_t s);
// C = fp32(M S) row by row; optional fused inner-product partials sum_{i,r} M C lambda.
spt_status launch_apply(const float *M, int64_t rows, int rank, const double *S, float *C,
                        const double *lambda, double *inner_partials, int *nparts_out, hipStream_t s);
int apply_blocks(int64_t rows, int rank);
// fit: out[0] = fit (shortcut), out[1] = |Xhat|^2; reads inner partials
spt_status launch_fit(const double *grams, int nmodes, int rank, const double *lambda,
                      const double *inner_partials, int nparts, double norm_x2, double *out, hipStream_t s);
spt_status launch_fit_direct(const double *resid_partials, int nparts, double norm_x2, double *out,
                             hipStream_t s);
spt_status launch_sum_f64(const double *parts, int n, double *out, hipStream_t s);

}  // namespace spt

// The opaque handle of the C-ABI is the tensor itself.
struct spt_tensor_s : spt::Tensor {};
