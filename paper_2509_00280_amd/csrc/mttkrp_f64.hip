// Mode-n MTTKRP in FP64 (Section II-B, Fig. 2) at the paper's own precision
// (FP64 values, factors and accumulation, 64-bit keys; Section IV-A).
//
// It runs the tensor's SEGMENT plan (positions of every nonzero in its tile's
// row-grouped order, pieces of one output row, records laid out grouped by
// row), which does not depend on the value type:
//  1. a workgroup of T/4 threads stages one tile of the key-ordered stream:
//     keys are decoded to the non-output coordinates, which are scattered with
//     the FP64 values to their plan positions in LDS;
//  2. lane groups of G lanes (lane j owns columns j, j + G, ...) take the
//     tile's pieces, gather the N-1 factor rows of each nonzero, form
//     v * Hadamard(rows) and sum the piece in registers;
//  3. each piece is stored as one FP64 record at its plan-given slot; a
//     second kernel sums the records of every row (plain stores for rows whose
//     records lie in one chunk, FP64 atomics at chunk boundaries).
#include "tile_common.h"

namespace spt {

namespace {

__host__ __device__ inline size_t f64_lds_bytes(int T, int nmodes) {
    return (size_t)(nmodes - 1) * T * 4 + (size_t)T * 8;
}

template <int NT, int NMAX, int G, int NB>
__global__ __launch_bounds__(NT) void k_mttkrp_seg_f64(MttkrpArgs a, const double *__restrict__ vals64, int64_t ntiles,
                                                       const double *f0, const double *f1, const double *f2,
                                                       const double *f3, const double *f4, const double *f5,
                                                       const double *f6, const double *f7,
                                                       double *__restrict__ rec_val) {
    constexpr int T = 4 * NT;
    extern __shared__ __align__(16) char lds[];
    const int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    const int nm = a.nmodes, mode = a.mode, tid = threadIdx.x, R = a.rank;
    uint32_t *crdg = (uint32_t *)lds;
    double *valg = (double *)(crdg + (size_t)(nm - 1) * T);
    const CodecRegs cr = load_codec_regs(a.codec);
    const int64_t base = tile * (int64_t)T;
    const int64_t rem = a.nnz - base;
    const int cnt = rem < T ? (int)rem : T;
    const int nwords = 2 * a.codec.key_words;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = tid + u * NT;
        if (e < cnt) {
            const uint64_t klo = a.lo[base + e];
            const uint64_t khi = nwords == 4 ? a.hi[base + e] : 0ull;
            const uint32_t w[4] = {(uint32_t)klo, (uint32_t)(klo >> 32), (uint32_t)khi, (uint32_t)(khi >> 32)};
            const int q = a.pl_pos[base + e] & (T - 1);
#pragma unroll
            for (int k = 0; k < NMAX; ++k)
                if (k < nm && k != mode) crdg[(k - (k > mode)) * T + q] = decode_mode(cr, k, nwords, w);
            valg[q] = vals64[base + e];
        }
    }
    __syncthreads();
    const double *fk[8] = {f0, f1, f2, f3, f4, f5, f6, f7};
    const double *fo[NMAX - 1];
#pragma unroll
    for (int o = 0; o < NMAX - 1; ++o) {
        const int k = o + (o >= mode);
        fo[o] = k < nm ? fk[k] : nullptr;
    }
    const int64_t k0 = a.pl_off[tile], k1 = min(a.pl_off[tile + 1], k0 + T);
    const int npieces = (int)(k1 - k0);
    constexpr int NG = NT / G;
    const int g = tid / G, j = tid % G;
    for (int k = g; k < npieces; k += NG) {
        const spt_u4 pc = reinterpret_cast<const spt_u4 *>(a.pl_piece)[k0 + k];
        const uint32_t d = pc.x, prow = pc.y, dest = pc.z;
        const int p0 = (int)(d & 0xFFFFu), p1 = min(p0 + (int)(d >> 16), T);
        if (dest >= (uint64_t)a.rec_cap || p0 >= p1) continue;
        double acc[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[b] = 0.0;
        for (int q = p0; q < p1; ++q) {
            const double v = valg[q];
            double p[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) p[b] = v;
#pragma unroll
            for (int o = 0; o < NMAX - 1; ++o) {
                if (o < nm - 1) {
                    const uint32_t row = min(crdg[o * T + q], a.frows[o + (o >= mode)] - 1);
                    const double *src = fo[o] + (size_t)row * R;
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const int c = b * G + j;
                        p[b] *= c < R ? src[c] : 0.0;
                    }
                }
            }
#pragma unroll
            for (int b = 0; b < NB; ++b) acc[b] += p[b];
        }
        if (j == 0) a.rec_row[dest] = prow;
        double *dst = rec_val + (size_t)dest * R;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int c = b * G + j;
            if (c < R) dst[c] = acc[b];
        }
    }
}

// Records grouped by row: each lane group sums a chunk of records column by
// column; a row whose records all lie in the chunk is stored, a row cut by a
// chunk boundary is added with FP64 atomics (out zeroed first).
template <int G, int NB>
__global__ __launch_bounds__(256) void k_reduce_records_f64(const uint64_t *__restrict__ srow,
                                                            const double *__restrict__ rec, int64_t P, int R,
                                                            int chunk, int64_t rows, double *__restrict__ out) {
    constexpr int GROUPS = 256 / G;
    const int g = threadIdx.x / G, j = threadIdx.x % G;
    const int64_t c0 = ((int64_t)blockIdx.x * GROUPS + g) * chunk;
    if (c0 >= P) return;
    const int64_t c1 = min(c0 + chunk, P);
    const uint64_t before = c0 > 0 ? srow[c0 - 1] : ~0ull;
    const uint64_t after = c1 < P ? srow[c1] : ~0ull;
    uint64_t cur = srow[c0];
    bool starts_here = cur != before;
    double acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = 0.0;
    auto emit = [&](uint64_t r, bool whole) {
        if (r >= (uint64_t)rows) return;
        double *o = out + (int64_t)r * R;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int c = b * G + j;
            if (c < R) {
                if (whole) o[c] = acc[b];
                else unsafeAtomicAdd(o + c, acc[b]);
            }
        }
    };
    for (int64_t q = c0; q < c1; ++q) {
        const uint64_t r = srow[q];
        if (r != cur) {
            emit(cur, starts_here);
            cur = r;
            starts_here = true;
#pragma unroll
            for (int b = 0; b < NB; ++b) acc[b] = 0.0;
        }
        const double *src = rec + q * R;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int c = b * G + j;
            acc[b] += c < R ? src[c] : 0.0;
        }
    }
    emit(cur, starts_here && cur != after);
}

__global__ __launch_bounds__(256) void k_gather_f64(const double *__restrict__ src, const uint32_t *__restrict__ idx,
                                                    double *__restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        dst[i] = src[idx[i]];
}

template <int NT, int NMAX, int G, int NB>
spt_status launch_f64_k(const MttkrpArgs &a, const double *vals64, const double *const *F, int64_t ntiles,
                        double *rec_val, hipStream_t s) {
    const size_t lds = f64_lds_bytes(4 * NT, a.nmodes);
    const double *f[8] = {};
    for (int k = 0; k < a.nmodes; ++k) f[k] = F[k];
    hipLaunchKernelGGL((k_mttkrp_seg_f64<NT, NMAX, G, NB>), dim3((unsigned)ntiles), dim3(NT), lds, s, a, vals64,
                       ntiles, f[0], f[1], f[2], f[3], f[4], f[5], f[6], f[7], rec_val);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

template <int NT, int NMAX>
spt_status launch_f64_r(const MttkrpArgs &a, const double *vals64, const double *const *F, int64_t ntiles,
                        double *rec_val, hipStream_t s) {
    const int R = a.rank;
    if (R <= 16) return launch_f64_k<NT, NMAX, 16, 1>(a, vals64, F, ntiles, rec_val, s);
    if (R <= 32) return launch_f64_k<NT, NMAX, 32, 1>(a, vals64, F, ntiles, rec_val, s);
    if (R <= 64) return launch_f64_k<NT, NMAX, 64, 1>(a, vals64, F, ntiles, rec_val, s);
    if (R <= 128) return launch_f64_k<NT, NMAX, 64, 2>(a, vals64, F, ntiles, rec_val, s);
    return launch_f64_k<NT, NMAX, 64, 4>(a, vals64, F, ntiles, rec_val, s);
}

template <int NT>
spt_status launch_f64_n(const MttkrpArgs &a, const double *vals64, const double *const *F, int64_t ntiles,
                        double *rec_val, hipStream_t s) {
    if (a.nmodes <= 3) return launch_f64_r<NT, 3>(a, vals64, F, ntiles, rec_val, s);
    if (a.nmodes == 4) return launch_f64_r<NT, 4>(a, vals64, F, ntiles, rec_val, s);
    return launch_f64_r<NT, 8>(a, vals64, F, ntiles, rec_val, s);
}

}  // namespace

bool f64_tile_ok(int tile, int nmodes) {
    return (tile == 1024 || tile == 2048 || tile == 4096) && f64_lds_bytes(tile, nmodes) <= 160 * 1024 - 1024;
}

spt_status launch_mttkrp_seg_f64(const MttkrpArgs &a, const double *vals64, const double *const *F,
                                 double *rec_val, hipStream_t s) {
    const int64_t ntiles = (a.nnz + a.tile - 1) / a.tile;
    if (ntiles == 0) return SPT_OK;
    if (!f64_tile_ok(a.tile, a.nmodes)) return fail(SPT_E_INVALID_ARG, "mttkrp_f64: tile does not fit LDS");
    if (!a.pl_pos || !a.pl_off || !a.pl_piece) return fail(SPT_E_INVALID_ARG, "mttkrp_f64: no plan");
    if (a.rank > 256) return fail(SPT_E_INVALID_ARG, "mttkrp_f64: rank above 256");
    if (a.tile == 1024) return launch_f64_n<256>(a, vals64, F, ntiles, rec_val, s);
    if (a.tile == 2048) return launch_f64_n<512>(a, vals64, F, ntiles, rec_val, s);
    return launch_f64_n<1024>(a, vals64, F, ntiles, rec_val, s);
}

spt_status launch_reduce_records_f64(const uint64_t *srow, const double *rec, int64_t P, int R, int64_t rows,
                                     double *out, hipStream_t s) {
    if (P == 0) return SPT_OK;
    constexpr int chunk = 256;
    auto go = [&](auto kern, int G) -> spt_status {
        const int groups = 256 / G;
        const int64_t nchunks = (P + chunk - 1) / chunk;
        const int64_t blocks = (nchunks + groups - 1) / groups;
        hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), 0, s, srow, rec, P, R, chunk, rows, out);
        SPT_HIP(hipGetLastError());
        return SPT_OK;
    };
    if (R <= 16) return go(k_reduce_records_f64<16, 1>, 16);
    if (R <= 32) return go(k_reduce_records_f64<32, 1>, 32);
    if (R <= 64) return go(k_reduce_records_f64<64, 1>, 64);
    if (R <= 128) return go(k_reduce_records_f64<64, 2>, 64);
    return go(k_reduce_records_f64<64, 4>, 64);
}

spt_status launch_gather_f64(const double *src, const uint32_t *idx, double *dst, int64_t n, hipStream_t s) {
    if (n == 0) return SPT_OK;
    const int64_t g = std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_gather_f64, dim3((unsigned)g), dim3(256), 0, s, src, idx, dst, n);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

}  // namespace spt
