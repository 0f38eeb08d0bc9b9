// Linearized-tensor construction on gfx950 (Section III-C, problem formulation):
// bit deposit of every coordinate into an l(p)-bit key, then a stable LSD radix
// sort of (key, input index) over the l(p) significant bits, then the value
// gather and the FP64 sum of squares.
//
// Radix sort design (one pass per 8-bit digit):
//   hist    : per 4096-element tile, a 256-bin digit histogram (per-wave LDS bins)
//   scan    : one workgroup per digit scans the tiles' counts (digit-major array)
//   scatter : each wave ranks a contiguous quarter of the tile stably on its own
//             (ballots order equal digits by lane, the wave's LDS counters carry
//             them across rounds), one barrier merges the waves' counts, then the
//             tile is regrouped by digit in LDS and runs of equal digit are written
//             contiguously so global stores coalesce.
#include "tile_common.h"

namespace spt {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ uint32_t extract_runs(const CodecRegs &c, int n, const uint32_t (&w)[4]) {
    return decode_mode(c, n, 4, w);
}

struct DimsArg {
    uint32_t d[kMaxModes];
};

// key = interleave(coords); idx = e.  err[0] counts out-of-range nonzeros,
// err[1] holds the smallest offending nonzero index, err[2] its mode.  Each
// thread takes kDepositU nonzeros a grid stride apart per round: all their
// coordinates are loaded before any key is formed, and every bit run of the
// codec is applied to all of them.
constexpr int kDepositU = 4;
__global__ __launch_bounds__(kThreads) void k_deposit(const uint32_t *__restrict__ coords, int64_t nnz,
                                                      DimsArg dims, Codec codec, uint64_t *__restrict__ lo,
                                                      uint64_t *__restrict__ hi, int *__restrict__ err) {
    const CodecRegs cl = load_codec_regs(codec);
    const int nm = codec.nmodes;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t e0 = (int64_t)blockIdx.x * kThreads + threadIdx.x; e0 < nnz; e0 += stride * kDepositU) {
        uint32_t c[kMaxModes][kDepositU];
#pragma unroll
        for (int n = 0; n < kMaxModes; ++n)
#pragma unroll
            for (int u = 0; u < kDepositU; ++u) {
                const int64_t e = e0 + u * stride;
                c[n][u] = 0;
                if (n < nm && e < nnz) c[n][u] = __builtin_nontemporal_load(coords + (int64_t)n * nnz + e);
            }
        uint32_t w[kDepositU][4];
#pragma unroll
        for (int u = 0; u < kDepositU; ++u) w[u][0] = w[u][1] = w[u][2] = w[u][3] = 0;
#pragma unroll
        for (int n = 0; n < kMaxModes; ++n) {
            if (n < nm) {
#pragma unroll
                for (int u = 0; u < kDepositU; ++u) {
                    const int64_t e = e0 + u * stride;
                    if (e < nnz && c[n][u] >= dims.d[n]) {
                        atomicAdd(err, 1);
                        atomicMin((unsigned long long *)(err + 2), ((unsigned long long)e << 8) | (unsigned)n);
                    }
                }
#pragma unroll
                for (int word = 0; word < 4; ++word) {
                    const int r0 = __builtin_amdgcn_readlane(cl.rb, n * 5 + word);
                    const int r1 = __builtin_amdgcn_readlane(cl.rb, n * 5 + word + 1);
                    for (int r = r0; r < r1; ++r) {
                        const uint32_t d = run_desc(cl, r);
                        const uint32_t kpos = (d >> 8) & 31u, cpos = (d >> 16) & 31u, len = d >> 24;
#pragma unroll
                        for (int u = 0; u < kDepositU; ++u) w[u][word] |= __builtin_amdgcn_ubfe(c[n][u], cpos, len) << kpos;
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kDepositU; ++u) {
            const int64_t e = e0 + u * stride;
            if (e < nnz) {
                lo[e] = (uint64_t)w[u][0] | ((uint64_t)w[u][1] << 32);
                if (codec.key_words == 2) hi[e] = (uint64_t)w[u][2] | ((uint64_t)w[u][3] << 32);
            }
        }
    }
}

template <int ITEMS>
__global__ __launch_bounds__(kThreads) void k_radix_hist(const uint64_t *__restrict__ keys, int64_t n, int shift,
                                                         uint32_t *__restrict__ counts, int nblocks) {
    __shared__ uint32_t h[4][256];
    const int tid = threadIdx.x, wave = tid >> 6;
#pragma unroll
    for (int w = 0; w < 4; ++w) h[w][tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * (kThreads * ITEMS);
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t e = base + i * kThreads + tid;
        if (e < n) {
            const uint32_t d = (uint32_t)(keys[e] >> shift) & 255u;
            atomicAdd(&h[wave][d], 1u);
        }
    }
    __syncthreads();
    counts[(int64_t)tid * nblocks + blockIdx.x] = h[0][tid] + h[1][tid] + h[2][tid] + h[3][tid];
}

// Exclusive scan of counts[d * nblocks + b] over b for one digit d per workgroup.
__global__ __launch_bounds__(kThreads) void k_radix_scan(uint32_t *__restrict__ counts, int nblocks,
                                                         uint32_t *__restrict__ totals) {
    __shared__ uint32_t wsum[4];
    __shared__ uint32_t carry_s;
    const int d = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t *row = counts + (int64_t)d * nblocks;
    if (tid == 0) carry_s = 0;
    __syncthreads();
    for (int b0 = 0; b0 < nblocks; b0 += kThreads) {
        const int b = b0 + tid;
        const uint32_t v = b < nblocks ? row[b] : 0u;
        uint32_t x = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        uint32_t wbase = 0;
        for (int w = 0; w < wave; ++w) wbase += wsum[w];
        const uint32_t carry = carry_s;
        if (b < nblocks) row[b] = carry + wbase + x - v;
        __syncthreads();
        if (tid == kThreads - 1) carry_s = carry + wbase + x;
        __syncthreads();
    }
    if (tid == 0) totals[d] = carry_s;
}

// Exclusive scan of 256 values held one per thread (block of 256).
__device__ __forceinline__ uint32_t block_scan_256(uint32_t v, uint32_t *wsum) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    uint32_t base = 0;
    for (int w = 0; w < wave; ++w) base += wsum[w];
    __syncthreads();
    return base + x - v;
}

template <int KW, int ITEMS>
__global__ __launch_bounds__(kThreads) void k_radix_scatter(
    const uint64_t *__restrict__ in_lo, const uint64_t *__restrict__ in_hi, const uint32_t *__restrict__ in_idx,
    uint64_t *__restrict__ out_lo, uint64_t *__restrict__ out_hi, uint32_t *__restrict__ out_idx, int64_t n,
    int word, int shift, const uint32_t *__restrict__ counts, const uint32_t *__restrict__ totals, int nblocks) {
    constexpr int TILE = kThreads * ITEMS;
    constexpr int WAVES = kThreads / 64;
    constexpr int WSPAN = 64 * ITEMS;  // consecutive elements ranked by one wave
    static_assert(WSPAN < (1 << 24), "rank field");
    __shared__ uint64_t s_lo[TILE];
    __shared__ uint64_t s_hi[KW == 2 ? TILE : 1];
    __shared__ uint32_t s_idx[TILE];
    __shared__ uint32_t wcnt[WAVES][256];  // per wave and digit: count, then the waves' exclusive offsets
    __shared__ uint32_t digit_off[256];
    __shared__ uint32_t local_start[256];
    __shared__ uint32_t wsum[4];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int b = blockIdx.x;
    const int64_t base = (int64_t)b * TILE;
    const int64_t wbase = base + (int64_t)wave * WSPAN;

    // every load of the wave's span is issued before the ranking waits for one
    uint64_t klo[ITEMS], khi[ITEMS];
    uint32_t idx[ITEMS], dr[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t e = wbase + i * 64 + lane;
        klo[i] = 0;
        khi[i] = 0;
        idx[i] = (uint32_t)e;
        if (e < n) {
            klo[i] = in_lo[e];
            if (KW == 2) khi[i] = in_hi[e];
            if (in_idx) idx[i] = in_idx[e];
        }
    }
#pragma unroll
    for (int w = 0; w < WAVES; ++w) wcnt[w][tid] = 0;
    {
        const uint32_t digit_base = block_scan_256(totals[tid], wsum);  // synchronises the block
        digit_off[tid] = digit_base + counts[(int64_t)tid * nblocks + b];
    }
    __syncthreads();

    // Rank within the wave: equal digits of one round are ordered by lane
    // (ballots), rounds in order through the wave's own LDS counters.  The
    // counter update of a digit's first lane takes the value read by the whole
    // wave, so no other wave and no barrier is involved.
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const bool valid = wbase + i * 64 + lane < n;
        const uint32_t d = (uint32_t)(((word == 0) ? klo[i] : khi[i]) >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t m = __ballot(valid && ((d >> bit) & 1u));
            peers &= ((d >> bit) & 1u) ? m : ~m;
        }
        const uint32_t before = __popcll(peers & lt_mask);
        uint32_t old = 0;
        if (valid) old = wcnt[wave][d];
        if (valid && before == 0) wcnt[wave][d] = old + (uint32_t)__popcll(peers);
        dr[i] = d | ((old + before) << 8);
    }
    __syncthreads();

    // digit d of this tile starts at local_start[d]; wave w's part of it
    // follows the parts of waves 0..w-1
    {
        uint32_t c[WAVES], run = 0;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) c[w] = wcnt[w][tid];
#pragma unroll
        for (int w = 0; w < WAVES; ++w) {
            wcnt[w][tid] = run;
            run += c[w];
        }
        local_start[tid] = block_scan_256(run, wsum);  // synchronises the block
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        if (wbase + i * 64 + lane < n) {
            const uint32_t d = dr[i] & 255u;
            const uint32_t pos = local_start[d] + wcnt[wave][d] + (dr[i] >> 8);
            s_lo[pos] = klo[i];
            if (KW == 2) s_hi[pos] = khi[i];
            s_idx[pos] = idx[i];
        }
    }
    __syncthreads();

    // runs of equal digit are contiguous in LDS and in the output
    const int cnt = (int)((n - base) < TILE ? (n - base) : TILE);
    for (int q = tid; q < cnt; q += kThreads) {
        const uint64_t klo_q = s_lo[q];
        const uint64_t khi_q = (KW == 2) ? s_hi[q] : 0;
        const uint32_t d = (uint32_t)(((word == 0) ? klo_q : khi_q) >> shift) & 255u;
        const int64_t dst = (int64_t)digit_off[d] + (q - (int)local_start[d]);
        out_lo[dst] = klo_q;
        if (KW == 2) out_hi[dst] = khi_q;
        out_idx[dst] = s_idx[q];
    }
}

// vals_out[j] = vals_in[idx[j]]; per-block partial sums of squares in FP64.
__global__ __launch_bounds__(kThreads) void k_gather_vals(const float *__restrict__ vin, const uint32_t *__restrict__ idx,
                                                          float *__restrict__ vout, int64_t n,
                                                          double *__restrict__ partials) {
    __shared__ double ws[4];
    double acc = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x; j < n; j += (int64_t)gridDim.x * kThreads) {
        const float v = vin[idx[j]];
        vout[j] = v;
        acc += (double)v * (double)v;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// out[j] = src[idx[j]] (32-bit words)
__global__ __launch_bounds__(kThreads) void k_gather_u32(const uint32_t *__restrict__ src, const uint32_t *__restrict__ idx,
                                                         uint32_t *__restrict__ out, int64_t n) {
    for (int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x; j < n; j += (int64_t)gridDim.x * kThreads)
        out[j] = src[idx[j]];
}

// dst[idx[j]] = src[j] (32-bit words)
__global__ __launch_bounds__(kThreads) void k_scatter_u32(const uint32_t *__restrict__ src, const uint32_t *__restrict__ idx,
                                                          uint32_t *__restrict__ dst, int64_t n) {
    for (int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x; j < n; j += (int64_t)gridDim.x * kThreads)
        dst[idx[j]] = src[j];
}

// Exclusive prefix sum in three launches: per-block local scans of
// kScanItems values per thread, one block scanning the block totals
// (chunk by chunk with a running carry), then the block offsets added.
constexpr int kScanItems = 16;
constexpr int kScanTile = kThreads * kScanItems;

__global__ __launch_bounds__(kThreads) void k_scan_local(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                         int64_t n, uint32_t *__restrict__ sums) {
    __shared__ uint32_t wsum[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t local = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = base + i < n ? in[base + i] : 0u;
        local += v[i];
    }
    uint32_t run = block_scan_256(local, wsum);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == kThreads - 1) sums[blockIdx.x] = run;
}

__global__ __launch_bounds__(kThreads) void k_scan_sums(uint32_t *__restrict__ sums, int64_t nb) {
    __shared__ uint32_t wsum[4];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nb; c0 += kScanTile) {
        const int64_t base = c0 + (int64_t)threadIdx.x * kScanItems;
        uint32_t v[kScanItems];
        uint32_t local = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            v[i] = base + i < nb ? sums[base + i] : 0u;
            local += v[i];
        }
        const uint32_t c = carry;
        uint32_t run = c + block_scan_256(local, wsum);
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            if (base + i < nb) sums[base + i] = run;
            run += v[i];
        }
        __syncthreads();  // every thread has read carry
        if (threadIdx.x == kThreads - 1) carry = run;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kThreads) void k_scan_add(uint32_t *__restrict__ out, int64_t n,
                                                       const uint32_t *__restrict__ sums) {
    const uint32_t add = sums[blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    for (int i = threadIdx.x; i < kScanTile; i += kThreads)
        if (base + i < n) out[base + i] += add;
}

__global__ __launch_bounds__(kThreads) void k_decode(const uint64_t *__restrict__ lo, const uint64_t *__restrict__ hi,
                                                     int64_t nnz, Codec codec, uint32_t *__restrict__ coords) {
    const CodecRegs cl = load_codec_regs(codec);
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * kThreads) {
        const uint64_t a = lo[e];
        const uint64_t b = codec.key_words == 2 ? hi[e] : 0;
        const uint32_t w[4] = {(uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32)};
        for (int n = 0; n < codec.nmodes; ++n) coords[(int64_t)n * nnz + e] = extract_runs(cl, n, w);
    }
}

__global__ __launch_bounds__(kThreads) void k_export_keys(const uint64_t *__restrict__ lo, const uint64_t *__restrict__ hi,
                                                          int64_t nnz, int kw, uint64_t *__restrict__ keys) {
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * kThreads) {
        if (kw == 2) {
            keys[2 * e] = lo[e];
            keys[2 * e + 1] = hi[e];
        } else {
            keys[e] = lo[e];
        }
    }
}

__global__ void k_init_err(int *err) {
    err[0] = 0;
    err[1] = 0;
    *(unsigned long long *)(err + 2) = ~0ull;
}

__global__ __launch_bounds__(kThreads) void k_sum_f64(const double *__restrict__ parts, int n, double *__restrict__ out) {
    __shared__ double ws[4];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += kThreads) acc += parts[i];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = ws[0] + ws[1] + ws[2] + ws[3];
}

__global__ void k_zero_f64(double *p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0.0;
}

int grid_for(int64_t n, int per_block, int cap) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

__global__ void k_iota(uint32_t *p, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = (uint32_t)e;
}

// Stable LSD sort of (lo[, hi]) keys over the t->lp significant bits.  On
// success *lo_io / *hi_io point at the sorted keys (the other buffers are
// released) and *idx_out at the input index of every sorted element.
template <int KW, int ITEMS>
spt_status radix_sort(int64_t n, int nbits, uint64_t **lo_io, uint64_t **hi_io, uint32_t **idx_out, hipStream_t s) {
    constexpr int TILE = kThreads * ITEMS;
    const int nblocks = (int)((n + TILE - 1) / TILE);
    const int passes = (nbits + 7) / 8;
    uint64_t *lo = *lo_io, *hi = *hi_io;
    uint64_t *lo2 = passes ? (uint64_t *)dev_alloc(sizeof(uint64_t) * n, s) : nullptr;
    uint64_t *hi2 = (KW == 2 && passes) ? (uint64_t *)dev_alloc(sizeof(uint64_t) * n, s) : nullptr;
    uint32_t *idx_a = (uint32_t *)dev_alloc(sizeof(uint32_t) * n, s);
    uint32_t *idx_b = passes > 1 ? (uint32_t *)dev_alloc(sizeof(uint32_t) * n, s) : nullptr;
    uint32_t *counts = (uint32_t *)dev_alloc(sizeof(uint32_t) * 256 * (size_t)nblocks, s);
    uint32_t *totals = (uint32_t *)dev_alloc(sizeof(uint32_t) * 256, s);
    if ((passes && !lo2) || (KW == 2 && passes && !hi2) || !idx_a || (passes > 1 && !idx_b) || !counts || !totals) {
        dev_free(lo2, s); dev_free(hi2, s); dev_free(idx_a, s); dev_free(idx_b, s);
        dev_free(counts, s); dev_free(totals, s);
        return fail(SPT_E_OOM, "radix sort: device allocation failed");
    }
    uint64_t *src_lo = lo, *src_hi = hi, *dst_lo = lo2, *dst_hi = hi2;
    uint32_t *src_idx = nullptr, *dst_idx = idx_a;
    for (int p = 0; p < passes; ++p) {
        const int bit = 8 * p;
        const int word = bit / 64, shift = bit % 64;
        const uint64_t *kw = word == 0 ? src_lo : src_hi;
        hipLaunchKernelGGL((k_radix_hist<ITEMS>), dim3(nblocks), dim3(kThreads), 0, s, kw, n, shift, counts, nblocks);
        hipLaunchKernelGGL(k_radix_scan, dim3(256), dim3(kThreads), 0, s, counts, nblocks, totals);
        hipLaunchKernelGGL((k_radix_scatter<KW, ITEMS>), dim3(nblocks), dim3(kThreads), 0, s, src_lo, src_hi, src_idx,
                           dst_lo, dst_hi, dst_idx, n, word, shift, counts, totals, nblocks);
        SPT_HIP(hipGetLastError());
        std::swap(src_lo, dst_lo);
        std::swap(src_hi, dst_hi);
        src_idx = dst_idx;
        dst_idx = (dst_idx == idx_a) ? idx_b : idx_a;
    }
    if (src_idx == nullptr) {  // no key bits at all: the input order is the sorted order
        hipLaunchKernelGGL(k_iota, dim3(grid_for(n, kThreads, 65536)), dim3(kThreads), 0, s, idx_a, n);
        SPT_HIP(hipGetLastError());
        src_idx = idx_a;
    }
    dev_free(dst_lo, s);  // after the swap, dst_* is the buffer not holding the result
    if (KW == 2) dev_free(dst_hi, s);
    dev_free(src_idx == idx_a ? idx_b : idx_a, s);
    dev_free(counts, s);
    dev_free(totals, s);
    *lo_io = src_lo;
    *hi_io = KW == 2 ? src_hi : nullptr;
    *idx_out = src_idx;
    return SPT_OK;
}

}  // namespace

spt_status launch_encode(Tensor *t, const uint32_t *coords, const float *vals, hipStream_t s) {
    const int64_t n = t->nnz;
    const int64_t n1 = n > 0 ? n : 1;
    t->lo = t->hi = nullptr;
    t->vals = nullptr;
    t->perm = nullptr;
    t->norm_x2 = 0.0;
    int *err = (int *)dev_alloc(64, s);
    double *partials = (double *)dev_alloc(sizeof(double) * 1025, s);
    uint64_t *lo = (uint64_t *)dev_alloc(sizeof(uint64_t) * n1, s);
    uint64_t *hi = t->key_words == 2 ? (uint64_t *)dev_alloc(sizeof(uint64_t) * n1, s) : nullptr;
    float *vout = (float *)dev_alloc(sizeof(float) * n1, s);
    uint32_t *idx = nullptr;
    auto cleanup = [&]() {
        dev_free(err, s); dev_free(partials, s); dev_free(lo, s); dev_free(hi, s); dev_free(vout, s);
        dev_free(idx, s);
    };
    if (!err || !partials || !lo || (t->key_words == 2 && !hi) || !vout) {
        cleanup();
        return fail(SPT_E_OOM, "encode: device allocation failed");
    }
    DimsArg dims{};
    for (int k = 0; k < t->nmodes; ++k) dims.d[k] = (uint32_t)t->dims[k];
    hipLaunchKernelGGL(k_init_err, dim3(1), dim3(1), 0, s, err);
    hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(64), 0, s, partials + 1024, 1);
    if (n > 0) {
        hipLaunchKernelGGL(k_deposit, dim3(grid_for(n, kThreads, 8192)), dim3(kThreads), 0, s, coords, n, dims,
                           t->codec, lo, hi, err);
        SPT_HIP(hipGetLastError());
        // keys whose coordinates were out of range are still valid bit patterns,
        // so sorting them is harmless; the single check below rejects the tensor.
        spt_status st = t->key_words == 2 ? radix_sort<2, 8>(n, t->lp, &lo, &hi, &idx, s)
                                          : radix_sort<1, 16>(n, t->lp, &lo, &hi, &idx, s);
        if (st != SPT_OK) {
            cleanup();
            return st;
        }
        const int g = grid_for(n, kThreads * 8, 1024);
        hipLaunchKernelGGL(k_gather_vals, dim3(g), dim3(kThreads), 0, s, vals, idx, vout, n, partials);
        hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(kThreads), 0, s, partials, g, partials + 1024);
        SPT_HIP(hipGetLastError());
    } else {
        idx = (uint32_t *)dev_alloc(sizeof(uint32_t), s);
    }
    struct {
        int e[4];
        double nx2;
    } h{};
    SPT_HIP(hipMemcpyAsync(h.e, err, sizeof(h.e), hipMemcpyDeviceToHost, s));
    SPT_HIP(hipMemcpyAsync(&h.nx2, partials + 1024, sizeof(double), hipMemcpyDeviceToHost, s));
    SPT_HIP(hipStreamSynchronize(s));
    if (h.e[0] != 0) {
        const unsigned long long packed = (unsigned long long)(uint32_t)h.e[2] | ((unsigned long long)(uint32_t)h.e[3] << 32);
        cleanup();
        return fail(SPT_E_INDEX_RANGE, std::to_string(h.e[0]) + " coordinate(s) out of range; first at nonzero " +
                                           std::to_string(packed >> 8) + ", mode " + std::to_string(packed & 255));
    }
    dev_free(err, s);
    dev_free(partials, s);
    t->lo = lo;
    t->hi = hi;
    t->vals = vout;
    t->perm = idx;
    t->norm_x2 = h.nx2;
    return SPT_OK;
}

spt_status launch_decode(const Tensor *t, uint32_t *coords, hipStream_t s) {
    if (t->nnz == 0) return SPT_OK;
    hipLaunchKernelGGL(k_decode, dim3(grid_for(t->nnz, kThreads, 16384)), dim3(kThreads), 0, s, t->lo, t->hi, t->nnz,
                       t->codec, coords);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

spt_status launch_gather_u32(const uint32_t *src, const uint32_t *idx, uint32_t *out, int64_t n, hipStream_t s) {
    if (n == 0) return SPT_OK;
    hipLaunchKernelGGL(k_gather_u32, dim3(grid_for(n, kThreads, 16384)), dim3(kThreads), 0, s, src, idx, out, n);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

spt_status launch_scatter_u32(const uint32_t *src, const uint32_t *idx, uint32_t *dst, int64_t n, hipStream_t s) {
    if (n == 0) return SPT_OK;
    hipLaunchKernelGGL(k_scatter_u32, dim3(grid_for(n, kThreads, 16384)), dim3(kThreads), 0, s, src, idx, dst, n);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

size_t exclusive_scan_ws(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile) + 1; }

spt_status launch_exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *ws, hipStream_t s) {
    if (n == 0) return SPT_OK;
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(kThreads), 0, s, in, out, n, ws);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kThreads), 0, s, ws, nb);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kThreads), 0, s, out, n, ws);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

spt_status launch_export(const Tensor *t, uint64_t *keys, hipStream_t s) {
    if (t->nnz == 0) return SPT_OK;
    hipLaunchKernelGGL(k_export_keys, dim3(grid_for(t->nnz, kThreads, 16384)), dim3(kThreads), 0, s, t->lo, t->hi,
                       t->nnz, t->key_words, keys);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

size_t sort_ws_counts(int64_t n) { return 256 * (size_t)((n + kThreads * 16 - 1) / (kThreads * 16)) + 256; }

// Stable LSD radix sort of n keys over their low nbits bits in caller-owned
// buffers: keys and keys2 (n each) ping-pong, idx_a / idx_b (n each) receive
// the input index of every sorted key, counts holds sort_ws_counts(n) words.
// *sorted_out / *idx_out point at the buffers holding the result.
spt_status sort_u64_keys_ws(uint64_t *keys, uint64_t *keys2, uint32_t *idx_a, uint32_t *idx_b, uint32_t *counts,
                            int64_t n, int nbits, uint64_t **sorted_out, uint32_t **idx_out, hipStream_t s) {
    constexpr int ITEMS = 16;
    constexpr int TILE = kThreads * ITEMS;
    *sorted_out = keys;
    *idx_out = idx_a;
    if (n <= 0) return SPT_OK;
    const int nblocks = (int)((n + TILE - 1) / TILE);
    const int passes = (nbits + 7) / 8;
    uint32_t *totals = counts + 256 * (size_t)nblocks;
    uint64_t *src = keys, *dst = keys2;
    uint32_t *src_idx = nullptr, *dst_idx = idx_a;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        hipLaunchKernelGGL((k_radix_hist<ITEMS>), dim3(nblocks), dim3(kThreads), 0, s, src, n, shift, counts, nblocks);
        hipLaunchKernelGGL(k_radix_scan, dim3(256), dim3(kThreads), 0, s, counts, nblocks, totals);
        hipLaunchKernelGGL((k_radix_scatter<1, ITEMS>), dim3(nblocks), dim3(kThreads), 0, s, src, (const uint64_t *)nullptr,
                           src_idx, dst, (uint64_t *)nullptr, dst_idx, n, 0, shift, counts, totals, nblocks);
        SPT_HIP(hipGetLastError());
        std::swap(src, dst);
        src_idx = dst_idx;
        dst_idx = (dst_idx == idx_a) ? idx_b : idx_a;
    }
    if (src_idx == nullptr) {
        hipLaunchKernelGGL(k_iota, dim3(grid_for(n, kThreads, 65536)), dim3(kThreads), 0, s, idx_a, n);
        SPT_HIP(hipGetLastError());
        src_idx = idx_a;
    }
    *sorted_out = src;
    *idx_out = src_idx;
    return SPT_OK;
}

spt_status launch_sum_f64(const double *parts, int n, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(kThreads), 0, s, parts, n, out);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

}  // namespace spt
