// Mode-n MTTKRP over the linearized tensor (Section II-B, Fig. 2) for gfx950.
//
// One workgroup (4 wave64s) owns a tile of T consecutive nonzeros in key order.
//  1. Stage: every lane loads keys/values of its nonzeros with coalesced
//     non-temporal loads (the stream is read once; factor rows stay cached),
//     decodes all N coordinates from the key bit runs, and writes them to LDS.
//  2. Regroup (REGROUP strategy): the output row i_n of every nonzero is
//     inserted into an LDS hash table (2T slots, linear probing with LDS CAS);
//     an LDS atomic counter per slot gives each nonzero its rank, a block scan
//     turns counts into starts, and a scatter writes the tile's order sorted by
//     output row.  Equal output indices are now contiguous runs.
//  3. Walk: lane groups of G lanes (each lane VEC consecutive columns) take
//     contiguous chunks of that order.  Per nonzero a group gathers the N-1
//     factor rows with vector loads (one row = G*VEC*4 contiguous bytes),
//     forms v * Hadamard(rows) and adds it into a register accumulator while
//     the output row stays the same (segmented reduction).  The accumulator is
//     flushed with FP32 global atomics only when the row changes or the chunk
//     ends, i.e. once per segment.
// The DIRECT strategy skips step 2 and walks key order (runs are short there,
// but no LDS work is spent); the plan chooses per mode.
//
// Workgroups are mapped to tiles XCD-aware: consecutive workgroup ids are
// dealt round-robin over the 8 XCDs, so each XCD gets a contiguous range of
// tiles and its L2 sees the locality of the key order.
#include "tile_common.h"

namespace spt {

namespace {

constexpr int kThreads = 256;
constexpr int kUnroll = 4;

struct TileLds {
    uint32_t *crd;   // [NMAX][T]
    float *val;      // [T]
    uint16_t *ord;   // [T]
    uint16_t *slot;  // [T]
    uint16_t *rnk;   // [T]
    uint32_t *hkey;  // [2T]
    uint32_t *hcnt;  // [2T]
};

__host__ __device__ inline size_t tile_lds_bytes(int T, int nmax, bool regroup) {
    size_t b = (size_t)nmax * T * 4 + (size_t)T * 4 + (size_t)T * 2;
    if (regroup) b += (size_t)T * 4 + (size_t)4 * T * 4;
    return b;
}

__device__ __forceinline__ TileLds carve(char *lds, int T, int nmax) {
    TileLds L;
    L.crd = (uint32_t *)lds;
    L.val = (float *)(L.crd + (size_t)nmax * T);
    L.ord = (uint16_t *)(L.val + T);
    L.slot = L.ord + T;
    L.rnk = L.slot + T;
    L.hkey = (uint32_t *)(L.rnk + T);
    L.hcnt = L.hkey + 2 * T;
    return L;
}

__device__ __forceinline__ uint32_t row_hash(uint32_t r, int hbits) {
    return (r ^ (r >> hbits) ^ (r >> (2 * hbits)));
}

// In-place exclusive scan of n (multiple of 256, <= 2048) u32 values in LDS.
__device__ __forceinline__ void block_exclusive_scan(uint32_t *a, int n, uint32_t *wsum) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int per = n / kThreads;
    uint32_t *p = a + tid * per;
    uint32_t local = 0;
    for (int i = 0; i < per; ++i) local += p[i];
    uint32_t x = local;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    uint32_t run = x - local;
    for (int w = 0; w < wave; ++w) run += wsum[w];
    for (int i = 0; i < per; ++i) {
        const uint32_t v = p[i];
        p[i] = run;
        run += v;
    }
    __syncthreads();
}

// Stage one tile: decode coordinates into LDS; with REGROUP also build the
// tile order sorted by coordinate of mode `gmode`.  Returns the valid count.
template <int NMAX, bool REGROUP>
__device__ __forceinline__ int stage_tile(const MttkrpArgs &a, int64_t tile, const TileLds &L, int gmode,
                                          uint32_t *wsum, const CodecRegs &cr) {
    const int T = a.tile;
    const int tid = threadIdx.x;
    const int64_t base = tile * (int64_t)T;
    const int64_t rem = a.nnz - base;
    const int cnt = rem < T ? (int)rem : T;
    const int ept = T / kThreads;  // 1, 2 or 4
    const int H = 2 * T;
    const int hbits = 31 - __clz(H);
    if (REGROUP) {
        for (int i = tid; i < H; i += kThreads) {
            L.hkey[i] = kNoRow;
            L.hcnt[i] = 0;
        }
    }
    uint32_t w[4][4];
    float v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = tid + u * kThreads;
        const bool ok = u < ept && e < cnt;
        uint64_t klo = 0, khi = 0;
        float x = 0.f;
        if (ok) {
            klo = __builtin_nontemporal_load(a.lo + base + e);
            if (a.codec.key_words == 2) khi = __builtin_nontemporal_load(a.hi + base + e);
            x = __builtin_nontemporal_load(a.vals + base + e);
        }
        w[u][0] = (uint32_t)klo;
        w[u][1] = (uint32_t)(klo >> 32);
        w[u][2] = (uint32_t)khi;
        w[u][3] = (uint32_t)(khi >> 32);
        v[u] = x;
    }
    uint32_t rowv[4] = {0, 0, 0, 0};
    const int nwords = 2 * a.codec.key_words;
#pragma unroll
    for (int k = 0; k < NMAX; ++k) {
        if (k < a.nmodes) {
            uint32_t x[4] = {0, 0, 0, 0};
#pragma unroll
            for (int word = 0; word < 4; ++word) {
                if (word < nwords) {
                    const int r0 = __builtin_amdgcn_readlane(cr.rb, k * 5 + word);
                    const int r1 = __builtin_amdgcn_readlane(cr.rb, k * 5 + word + 1);
                    for (int r = r0; r < r1; ++r) {
                        const uint32_t d = run_desc(cr, r);
                        const uint32_t kpos = (d >> 8) & 31u, cpos = (d >> 16) & 31u, len = d >> 24;
#pragma unroll
                        for (int u = 0; u < 4; ++u) x[u] |= __builtin_amdgcn_ubfe(w[u][word], kpos, len) << cpos;
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = tid + u * kThreads;
                if (u < ept) L.crd[k * T + e] = x[u];
                if (k == gmode) rowv[u] = x[u];
            }
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (u < ept) L.val[tid + u * kThreads] = v[u];
    }
    if (REGROUP) {
        __syncthreads();  // hash table cleared
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + u * kThreads;
            if (u < ept && e < cnt) {
                const uint32_t row = rowv[u];
                uint32_t s = row_hash(row, hbits) & (uint32_t)(H - 1);
                for (;;) {
                    const uint32_t prev = atomicCAS(&L.hkey[s], kNoRow, row);
                    if (prev == kNoRow || prev == row) break;
                    s = (s + 1) & (uint32_t)(H - 1);
                }
                L.rnk[e] = (uint16_t)atomicAdd(&L.hcnt[s], 1u);
                L.slot[e] = (uint16_t)s;
            }
        }
        __syncthreads();
        block_exclusive_scan(L.hcnt, H, wsum);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + u * kThreads;
            if (u < ept && e < cnt) L.ord[L.hcnt[L.slot[e]] + L.rnk[e]] = (uint16_t)e;
        }
    }
    __syncthreads();
    return cnt;
}

template <int G, int VEC, int NB>
struct Acc {
    float v[NB][VEC];
};

template <int G, int VEC, int NB>
__device__ __forceinline__ void flush_row(float *__restrict__ out, uint32_t row, int R, int j, const Acc<G, VEC, NB> &acc) {
    float *o = out + (int64_t)row * R;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int col = (b * G + j) * VEC;
        if (col < R) {
#pragma unroll
            for (int q = 0; q < VEC; ++q) unsafeAtomicAdd(o + col + q, acc.v[b][q]);
        }
    }
}

// Walk the staged tile and accumulate into out (see the file comment).
template <int G, int VEC, int NB, int NMAX, bool REGROUP>
__device__ __forceinline__ void walk_tile(const MttkrpArgs &a, const TileLds &L, int cnt) {
    constexpr int GROUPS = kThreads / G;
    const int T = a.tile;
    const int tid = threadIdx.x;
    const int g = tid / G, j = tid % G;
    const int R = a.rank;
    const int mode = a.mode;
    const int ch = T / GROUPS;
    const int q0 = g * ch;
    const int q1 = min(q0 + ch, cnt);
    uint32_t cur = kNoRow;
    Acc<G, VEC, NB> acc;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int q = 0; q < VEC; ++q) acc.v[b][q] = 0.f;

    for (int q = q0; q < q1; q += kUnroll) {
        uint32_t e[kUnroll], row[kUnroll];
        bool ok[kUnroll];
        float p[kUnroll][NB][VEC];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            ok[u] = (q + u) < q1;
            const int qq = ok[u] ? q + u : q0;
            e[u] = REGROUP ? (uint32_t)L.ord[qq] : (uint32_t)qq;
            row[u] = L.crd[mode * T + e[u]];
            const float x = L.val[e[u]];
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int qv = 0; qv < VEC; ++qv) p[u][b][qv] = x;
        }
#pragma unroll
        for (int k = 0; k < NMAX; ++k) {
            if (k < a.nmodes && k != mode) {
                const float *__restrict__ F = a.f[k];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const uint32_t idx = L.crd[k * T + e[u]];
                    const float *fr = F + (int64_t)idx * R;
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const int col = (b * G + j) * VEC;
                        float x[VEC];
                        if (col < R) {
                            load_vec<VEC>(fr + col, x);
                        } else {
#pragma unroll
                            for (int qv = 0; qv < VEC; ++qv) x[qv] = 0.f;
                        }
#pragma unroll
                        for (int qv = 0; qv < VEC; ++qv) p[u][b][qv] *= x[qv];
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (ok[u]) {
                if (row[u] != cur) {
                    if (cur != kNoRow) flush_row<G, VEC, NB>(a.out, cur, R, j, acc);
                    cur = row[u];
#pragma unroll
                    for (int b = 0; b < NB; ++b)
#pragma unroll
                        for (int qv = 0; qv < VEC; ++qv) acc.v[b][qv] = p[u][b][qv];
                } else {
#pragma unroll
                    for (int b = 0; b < NB; ++b)
#pragma unroll
                        for (int qv = 0; qv < VEC; ++qv) acc.v[b][qv] += p[u][b][qv];
                }
            }
        }
    }
    if (cur != kNoRow) flush_row<G, VEC, NB>(a.out, cur, R, j, acc);
}

template <int G, int VEC, int NB, int NMAX, bool REGROUP>
__global__ __launch_bounds__(kThreads) void k_mttkrp(MttkrpArgs a, int64_t ntiles) {
    extern __shared__ __align__(16) char lds[];
    __shared__ uint32_t wsum[4];
    const int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    const TileLds L = carve(lds, a.tile, NMAX);
    const CodecRegs cr = load_codec_regs(a.codec);
    const int cnt = stage_tile<NMAX, REGROUP>(a, tile, L, a.mode, wsum, cr);
    walk_tile<G, VEC, NB, NMAX, REGROUP>(a, L, cnt);
}

// ------------------------------------------------------------------ direct residual
// partials[2*b] = sum over the tile of (v - xhat)^2, partials[2*b+1] = sum xhat^2 (FP64),
// xhat = sum_r lambda_r prod_k C^(k)[i_k, r].
template <int G, int VEC, int NB, int NMAX>
__device__ __forceinline__ void resid_tile(const MttkrpArgs &a, int64_t tile, const double *__restrict__ lam,
                                           double *__restrict__ partials, char *lds) {
    __shared__ uint32_t wsum[4];
    __shared__ double red[2][kThreads / 64];
    const TileLds L = carve(lds, a.tile, NMAX);
    const CodecRegs cr = load_codec_regs(a.codec);
    const int cnt = stage_tile<NMAX, false>(a, tile, L, -1, wsum, cr);
    constexpr int GROUPS = kThreads / G;
    const int tid = threadIdx.x, g = tid / G, j = tid % G;
    const int R = a.rank, T = a.tile;
    double s_res = 0.0, s_hat = 0.0;
    double lv[NB][VEC];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
            const int col = (b * G + j) * VEC + q;
            lv[b][q] = col < R ? lam[col] : 0.0;
        }
    for (int e = g; e < cnt; e += GROUPS) {
        // the product of the factor entries in FP64 (each FP32 entry widened first)
        double p[NB][VEC];
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int q = 0; q < VEC; ++q) p[b][q] = 1.0;
#pragma unroll
        for (int k = 0; k < NMAX; ++k) {
            if (k < a.nmodes) {
                const float *fr = a.f[k] + (int64_t)L.crd[k * T + e] * R;
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const int col = (b * G + j) * VEC;
                    float x[VEC];
                    if (col < R) load_vec<VEC>(fr + col, x);
                    else
#pragma unroll
                        for (int q = 0; q < VEC; ++q) x[q] = 0.f;
#pragma unroll
                    for (int q = 0; q < VEC; ++q) p[b][q] *= (double)x[q];
                }
            }
        }
        double part = 0.0;
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int q = 0; q < VEC; ++q) part += lv[b][q] * p[b][q];
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
        if (j == 0) {
            const double d = (double)L.val[e] - part;
            s_res += d * d;
            s_hat += part * part;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        s_res += __shfl_down(s_res, off, 64);
        s_hat += __shfl_down(s_hat, off, 64);
    }
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = s_res;
        red[1][tid >> 6] = s_hat;
    }
    __syncthreads();
    if (tid == 0) {
        double r0 = 0.0, r1 = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) {
            r0 += red[0][w];
            r1 += red[1][w];
        }
        partials[2 * tile] = r0;
        partials[2 * tile + 1] = r1;
    }
}

template <int G, int VEC, int NB, int NMAX>
__global__ __launch_bounds__(kThreads) void k_resid(MttkrpArgs a, int64_t ntiles, const double *__restrict__ lam,
                                                    double *__restrict__ partials) {
    extern __shared__ __align__(16) char lds[];
    resid_tile<G, VEC, NB, NMAX>(a, blockIdx.x, lam, partials, lds);
}

// Residual of many tensors in one launch: tile `it` of the launch belongs to
// the last item whose first_tile <= it; its partials go to the item's array.
template <int G, int VEC, int NB, int NMAX>
__global__ __launch_bounds__(kThreads) void k_resid_batched(const ResidItem *__restrict__ items, int count) {
    extern __shared__ __align__(16) char lds[];
    const int64_t it = blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].first_tile <= it) lo = mid;
        else hi = mid - 1;
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    const ResidItem &r = items[lo];
    resid_tile<G, VEC, NB, NMAX>(r.a, it - r.first_tile, r.lambda, r.partials, lds);
}

__global__ __launch_bounds__(kThreads) void k_fill_zero(float4 *__restrict__ p, int64_t n4, float *__restrict__ tail,
                                                        int ntail) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n4; i += (int64_t)gridDim.x * kThreads)
        p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (blockIdx.x == 0 && (int)threadIdx.x < ntail) tail[threadIdx.x] = 0.f;
}

template <int G, int VEC, int NB, int NMAX>
spt_status launch_walk(const MttkrpArgs &a, bool regroup, int64_t ntiles, hipStream_t s) {
    const size_t lds = tile_lds_bytes(a.tile, NMAX, regroup);
    if (regroup)
        hipLaunchKernelGGL((k_mttkrp<G, VEC, NB, NMAX, true>), dim3((unsigned)ntiles), dim3(kThreads), lds, s, a, ntiles);
    else
        hipLaunchKernelGGL((k_mttkrp<G, VEC, NB, NMAX, false>), dim3((unsigned)ntiles), dim3(kThreads), lds, s, a, ntiles);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

template <int NMAX>
spt_status launch_nmax(const MttkrpArgs &a, bool regroup, int64_t ntiles, hipStream_t s) {
    const int R = a.rank;
    if ((R & 3) == 0) {
        const int r4 = R >> 2;
        if (r4 <= 1) return launch_walk<1, 4, 1, NMAX>(a, regroup, ntiles, s);
        if (r4 <= 2) return launch_walk<2, 4, 1, NMAX>(a, regroup, ntiles, s);
        if (r4 <= 4) return launch_walk<4, 4, 1, NMAX>(a, regroup, ntiles, s);
        if (r4 <= 8) return launch_walk<8, 4, 1, NMAX>(a, regroup, ntiles, s);
        if (r4 <= 16) return launch_walk<16, 4, 1, NMAX>(a, regroup, ntiles, s);
        if (r4 <= 32) return launch_walk<32, 4, 1, NMAX>(a, regroup, ntiles, s);
        return launch_walk<64, 4, 1, NMAX>(a, regroup, ntiles, s);
    }
    if (R <= 64) return launch_walk<64, 1, 1, NMAX>(a, regroup, ntiles, s);
    if (R <= 128) return launch_walk<64, 1, 2, NMAX>(a, regroup, ntiles, s);
    if (R <= 192) return launch_walk<64, 1, 3, NMAX>(a, regroup, ntiles, s);
    return launch_walk<64, 1, 4, NMAX>(a, regroup, ntiles, s);
}

template <int NMAX>
spt_status launch_resid_batched_nmax(const ResidItem *items, int count, int64_t total_tiles, int rmax, bool vec4,
                                     hipStream_t s) {
    const size_t lds = tile_lds_bytes(kResidTile, NMAX, false);
    const dim3 g((unsigned)total_tiles), b(kThreads);
    if (vec4 && rmax <= 64) {
        const int r4 = rmax >> 2;
        if (r4 <= 1) hipLaunchKernelGGL((k_resid_batched<1, 4, 1, NMAX>), g, b, lds, s, items, count);
        else if (r4 <= 2) hipLaunchKernelGGL((k_resid_batched<2, 4, 1, NMAX>), g, b, lds, s, items, count);
        else if (r4 <= 4) hipLaunchKernelGGL((k_resid_batched<4, 4, 1, NMAX>), g, b, lds, s, items, count);
        else if (r4 <= 8) hipLaunchKernelGGL((k_resid_batched<8, 4, 1, NMAX>), g, b, lds, s, items, count);
        else hipLaunchKernelGGL((k_resid_batched<16, 4, 1, NMAX>), g, b, lds, s, items, count);
    } else {
        hipLaunchKernelGGL((k_resid_batched<64, 1, 1, NMAX>), g, b, lds, s, items, count);
    }
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

template <int NMAX>
spt_status launch_resid_nmax(const MttkrpArgs &a, const double *lam, double *partials, int64_t ntiles, hipStream_t s) {
    const size_t lds = tile_lds_bytes(a.tile, NMAX, false);
    const int R = a.rank;
    if ((R & 3) == 0 && R <= 64) {
        const int r4 = R >> 2;
        if (r4 <= 1) hipLaunchKernelGGL((k_resid<1, 4, 1, NMAX>), dim3((unsigned)ntiles), dim3(kThreads), lds, s, a, ntiles, lam, partials);
        else if (r4 <= 2) hipLaunchKernelGGL((k_resid<2, 4, 1, NMAX>), dim3((unsigned)ntiles), dim3(kThreads), lds, s, a, ntiles, lam, partials);
        else if (r4 <= 4) hipLaunchKernelGGL((k_resid<4, 4, 1, NMAX>), dim3((unsigned)ntiles), dim3(kThreads), lds, s, a, ntiles, lam, partials);
        else if (r4 <= 8) hipLaunchKernelGGL((k_resid<8, 4, 1, NMAX>), dim3((unsigned)ntiles), dim3(kThreads), lds, s, a, ntiles, lam, partials);
        else hipLaunchKernelGGL((k_resid<16, 4, 1, NMAX>), dim3((unsigned)ntiles), dim3(kThreads), lds, s, a, ntiles, lam, partials);
    } else {
        hipLaunchKernelGGL((k_resid<64, 1, 1, NMAX>), dim3((unsigned)ntiles), dim3(kThreads), lds, s, a, ntiles, lam, partials);
    }
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

}  // namespace

spt_status launch_fill_zero(float *p, int64_t n, hipStream_t s) {
    if (n <= 0) return SPT_OK;
    // p is 16-byte aligned (factor/output contract); zero whole float4s then the tail
    const int64_t n4 = n / 4;
    const int ntail = (int)(n - n4 * 4);
    int64_t g = (n4 + kThreads - 1) / kThreads;
    if (g < 1) g = 1;
    if (g > 16384) g = 16384;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)g), dim3(kThreads), 0, s, (float4 *)p, n4, p + n4 * 4, ntail);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

spt_status launch_mttkrp(const MttkrpArgs &a, int strategy, hipStream_t s) {
    if (a.nnz == 0) return SPT_OK;
    const int64_t ntiles = (a.nnz + a.tile - 1) / a.tile;
    const bool regroup = strategy == SPT_STRATEGY_REGROUP;
    if (a.nmodes <= 4) return launch_nmax<4>(a, regroup, ntiles, s);
    return launch_nmax<8>(a, regroup, ntiles, s);
}

spt_status launch_resid(const MttkrpArgs &a, const double *lam, double *partials, int nparts, hipStream_t s) {
    const int64_t ntiles = (a.nnz + a.tile - 1) / a.tile;
    if (ntiles != nparts) return fail(SPT_E_INVALID_ARG, "resid: partials size mismatch");
    if (ntiles == 0) return SPT_OK;
    if (a.nmodes <= 4) return launch_resid_nmax<4>(a, lam, partials, ntiles, s);
    return launch_resid_nmax<8>(a, lam, partials, ntiles, s);
}

spt_status launch_resid_batched(const ResidItem *items, int count, int64_t total_tiles, int nmodes_max, int rmax,
                                bool vec4, hipStream_t s) {
    if (total_tiles == 0 || count == 0) return SPT_OK;
    if (rmax > 64) return fail(SPT_E_INVALID_ARG, "resid_batched: rank above 64");
    if (nmodes_max <= 4) return launch_resid_batched_nmax<4>(items, count, total_tiles, rmax, vec4, s);
    return launch_resid_batched_nmax<8>(items, count, total_tiles, rmax, vec4, s);
}

}  // namespace spt
