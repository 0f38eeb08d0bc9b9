// Internal declarations shared by the library's HIP and host sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "spt.h"  // include/ is on the include path

namespace spt {

constexpr int kMaxModes = SPT_MAX_MODES;
constexpr int kMaxRuns = 160;          // l(p) <= 128 bits plus splits at 32-bit word boundaries
constexpr uint32_t kNoRow = 0xFFFFFFFFu;

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

// Build the codec of a layout (layout[t] = mode feeding key bit t).
void make_codec(int nmodes, const int *lbits, const uint8_t *layout, int lp, Codec *c);

// ---------------------------------------------------------------- device memory
void *dev_alloc(size_t bytes, hipStream_t s);
void dev_free(void *p, hipStream_t s);

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
    int64_t records = 0;     // TABLE: records written per call
    int64_t *rec_off = nullptr;  // TABLE: device, nwg offsets
};

// Grow-only device buffers owned by a tensor handle and reused by its MTTKRP
// calls (records and sort buffers), so steady-state calls allocate nothing.
enum WsSlot { WS_REC_ROW, WS_REC_VAL, WS_KEYS2, WS_IDX_A, WS_IDX_B, WS_COUNTS, WS_PART, WS_NSLOTS };

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
    uint32_t *perm = nullptr; // input index of each element
    double norm_x2 = 0.0;
    spt_plan plan{};
    ModePlan mplan[kMaxModes];
    void *ws[WS_NSLOTS] = {};
    size_t ws_bytes[WS_NSLOTS] = {};
};

// plan.cpp
int device_cus();
spt_status resolve_plan(Tensor *t, int mode, int rank, hipStream_t s, ModePlan **out);
// mode-`mode` MTTKRP into out (overwritten), per the tensor's plan
spt_status run_mttkrp(Tensor *t, const float *const *factors, int rank, int mode, float *out, hipStream_t s);
void release_plans(Tensor *t);
// workspace slot of at least `bytes` (synchronises s before replacing a smaller buffer)
void *tensor_ws(Tensor *t, int slot, size_t bytes, hipStream_t s);
void release_ws(Tensor *t);
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
    float *out;
    // SEGMENT strategy: record output
    uint64_t *rec_row;
    float *rec_val;
    const int64_t *rec_off;   // per tile, ntiles + 1 entries
    Codec codec;
};
spt_status launch_fill_zero(float *p, int64_t n, hipStream_t s);
MttkrpArgs make_args(const Tensor *t, const float *const *factors, int rank, int mode, float *out, int tile);
spt_status launch_mttkrp(const MttkrpArgs &a, int strategy, hipStream_t s);
bool seg_tile_ok(int tile, int nmodes);
spt_status launch_count_pieces(const MttkrpArgs &a, int64_t *counts, hipStream_t s);
spt_status launch_mttkrp_seg(const MttkrpArgs &a, hipStream_t s);

// Per-tensor descriptor of the batched persistent MTTKRP.
struct BatchItem {
    MttkrpArgs a;
    int64_t first_tile;  // prefix sum of tiles over the batch
    int strategy;
    int pad;
};
spt_status launch_mttkrp_batched(const BatchItem *items_dev, int count, int64_t total_tiles,
                                 int nmodes_max, int *counter_dev, hipStream_t s);

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

// dense.hip
spt_status launch_gram(const float *C, int64_t rows, int rank, double *G, double *work, size_t work_bytes,
                       hipStream_t s);
size_t gram_work_bytes(int64_t rows, int rank);
// solve preparation: V = Hadamard of grams[k != mode]; Cholesky with ridge; W = V^-1;
// lambda_r = sqrt((W Gm W)_rr) (1 if 0); S = W diag(1/lambda).  status_out: 0 ok, >0 ridge retries, <0 failure.
spt_status launch_solve_prep(const double *grams, int nmodes, int mode, int rank, const double *gram_m,
                             double *S, double *lambda, int *status_out, hipStream_t s);
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
