// Mode-n MTTKRP with conflict resolution staged in LDS (Section II-B, Fig. 2;
// the synchronisation cost the paper attributes to MTTKRP is what this file
// organises).
//
// On MI355X a device-scope FP32 atomic row update costs ~40x a plain store
// and serialises on contended rows, so this path keeps atomics out of the
// hot loop entirely:
//
//  * Persistent workgroups (512 threads, one per CU) each own a contiguous
//    range of the key-ordered nonzero stream, processed in sub-tiles of 512.
//  * Every sub-tile is decoded into LDS.  Its distinct output rows are found
//    with a small LDS hash (one CAS per nonzero); one representative lane per
//    distinct row looks the row up in the workgroup's LDS accumulator table
//    (hash index -> accumulator row).  If the new rows do not fit, the table
//    is flushed first.  Flush points depend only on the set of rows seen, so a
//    counting pass of the same loop gives every workgroup's record count
//    ahead of time (deterministic record offsets, no global counters).
//  * The walk: lane groups (G lanes x VEC columns) gather the N-1 factor rows
//    of each nonzero with vector loads, form v * Hadamard, merge runs of equal
//    accumulator row in registers (segmented reduction in key order) and add
//    each run into the LDS accumulator with ds_add_f32.
//  * A flush writes (row, R floats) records with plain coalesced stores.
//    Records are sorted by row (LSD radix sort) and summed per row; a row's
//    sum is stored plainly unless it straddles two reducer chunks.
//  * PRIV: when the whole output (or a column slice of it) fits in LDS, the
//    accumulator is indexed by row directly, each workgroup writes its private
//    partial, and a strided sum over workgroups produces the output.
#include "tile_common.h"

namespace spt {

namespace {

constexpr int kTT = 512;       // threads per workgroup
constexpr int kSubH = 1024;    // sub-tile hash slots (>= 2 x the sub-tile size)
constexpr int kUnroll = 4;
constexpr uint16_t kNewRow = 0xFFFF;

enum Kind { KIND_TABLE = 0, KIND_PRIV = 1, KIND_COUNT = 2 };

struct Lds {
    uint32_t *crd;    // [NMAX][TS]
    float *val;       // [TS]
    uint16_t *sslot;  // [TS] sub-tile hash slot of each nonzero
    uint16_t *ord;    // [TS] sub-tile order grouped by output row
    uint32_t *skey;   // [kSubH] sub-tile hash keys (rows)
    uint32_t *scnt;   // [kSubH] nonzeros per slot, then first position of each slot
    uint16_t *smap;   // [kSubH] slot -> accumulator row (TABLE)
    uint32_t *hkey;   // [H]
    uint16_t *hidx;   // [H]
    uint32_t *arow;   // [cap]
    float *acc;       // [cap][stride]
};

// LDS bytes of one workgroup: staging of TS nonzeros, the accumulator's hash
// index (H = 2^hbits slots, none for PRIV), the accumulator row map and the
// accumulator itself (cap rows of `stride` floats).
__host__ __device__ inline size_t table_lds_bytes(int nmax, int ts, int cap, int hbits, int stride, bool priv,
                                                  bool with_acc) {
    size_t b = (size_t)nmax * ts * 4 + (size_t)ts * 4 + (size_t)ts * 4 + (size_t)kSubH * 8 + (size_t)kSubH * 2;
    if (!priv) b += ((size_t)1 << hbits) * 6 + (size_t)cap * 4;
    b = (b + 15) & ~(size_t)15;
    if (with_acc) b += (size_t)cap * stride * 4;
    return b;
}

__device__ __forceinline__ Lds carve(char *p, int nmax, int ts, int cap, int hbits, bool priv) {
    Lds L;
    const size_t H = priv ? 0 : (size_t)1 << hbits;
    L.crd = (uint32_t *)p;
    L.val = (float *)(L.crd + (size_t)nmax * ts);
    L.sslot = (uint16_t *)(L.val + ts);
    L.ord = L.sslot + ts;
    L.skey = (uint32_t *)(L.ord + ts);
    L.scnt = L.skey + kSubH;
    L.smap = (uint16_t *)(L.scnt + kSubH);
    L.hkey = (uint32_t *)(L.smap + kSubH);
    L.hidx = (uint16_t *)(L.hkey + H);
    L.arow = (uint32_t *)(L.hidx + H);
    size_t off = (size_t)((char *)(L.arow + (priv ? 0 : cap)) - p);
    off = (off + 15) & ~(size_t)15;
    L.acc = (float *)(p + off);
    return L;
}

template <int G, int VEC, int NB, int NMAX, int KIND, int TS>
__global__ __launch_bounds__(kTT) void k_mttkrp_table(TableArgs t) {
    extern __shared__ __align__(16) char lds[];
    __shared__ int s_occ, s_new, s_flush;
    __shared__ long long s_rec;
    __shared__ uint32_t s_wsum[kTT / 64];
    const MttkrpArgs &a = t.a;
    const int tid = threadIdx.x;
    const int nm = a.nmodes, mode = a.mode, R = a.rank;
    const int cap = t.cap;
    const int H = 1 << t.hbits;
    const int stride = t.stride;
    const int colbase = KIND == KIND_PRIV ? blockIdx.y * t.rs : 0;
    const int ncols = KIND == KIND_PRIV ? min(t.rs, R - colbase) : R;
    const Lds L = carve(lds, NMAX, TS, cap, t.hbits, KIND == KIND_PRIV);
    const int64_t w = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t nsub = (a.nnz + TS - 1) / TS;
    const int64_t sub0 = w * t.sub_per_wg;
    const int64_t sub1 = min(sub0 + t.sub_per_wg, nsub);
    const int nwords = 2 * a.codec.key_words;
    const CodecRegs cr = load_codec_regs(a.codec);

    if (KIND != KIND_PRIV) {
        for (int i = tid; i < H; i += kTT) L.hkey[i] = kNoRow;
    }
    if (KIND != KIND_COUNT) {
        for (int i = tid; i < cap * stride; i += kTT) L.acc[i] = 0.f;
    }
    if (tid == 0) {
        s_occ = 0;
        s_rec = 0;
    }
    const int64_t rec_base = (KIND == KIND_TABLE) ? t.rec_off[w] : 0;

    // flush the accumulator table: records (row, R floats), then clear it
    auto flush = [&]() {
        const int occ = s_occ;
        if (KIND == KIND_TABLE) {
            const int64_t o = rec_base + s_rec;
            for (int i = tid; i < occ; i += kTT) t.rec_row[o + i] = (uint64_t)L.arow[i];
            for (int i = tid; i < occ * R; i += kTT) {
                const int r = i / R, c = i - r * R;
                t.rec_val[(o + r) * R + c] = L.acc[r * stride + c];
                L.acc[r * stride + c] = 0.f;
            }
        }
        for (int i = tid; i < H; i += kTT) L.hkey[i] = kNoRow;
        __syncthreads();
        if (tid == 0) {
            s_rec += occ;
            s_occ = 0;
        }
        __syncthreads();
    };

    // keys/values of the next sub-tile, loaded one sub-tile ahead so that their
    // latency hides behind the current sub-tile's walk
    uint64_t n_lo = 0, n_hi = 0;
    float n_x = 0.f;
    auto prefetch = [&](int64_t sub) {
        const int64_t e = sub * TS + tid;
        n_lo = 0;
        n_hi = 0;
        n_x = 0.f;
        if (tid < TS && sub < sub1 && e < a.nnz) {
            n_lo = __builtin_nontemporal_load(a.lo + e);
            if (nwords == 4) n_hi = __builtin_nontemporal_load(a.hi + e);
            n_x = __builtin_nontemporal_load(a.vals + e);
        }
    };
    prefetch(sub0);

    for (int64_t sub = sub0; sub < sub1; ++sub) {
        const int64_t base = sub * TS;
        const int cnt = (int)min((int64_t)TS, a.nnz - base);
        for (int i = tid; i < kSubH; i += kTT) {
            L.skey[i] = kNoRow;
            L.scnt[i] = 0;
        }
        if (tid == 0) s_new = 0;
        // ---- stage: decode the prefetched nonzero of this lane
        const bool valid = tid < cnt;
        uint32_t row = 0;
        {
            const uint32_t wv[4] = {(uint32_t)n_lo, (uint32_t)(n_lo >> 32), (uint32_t)n_hi, (uint32_t)(n_hi >> 32)};
#pragma unroll
            for (int k = 0; k < NMAX; ++k) {
                if (k < nm) {
                    const uint32_t c = decode_mode(cr, k, nwords, wv);
                    if (tid < TS) L.crd[k * TS + tid] = c;
                    if (k == mode) row = c;
                }
            }
            if (tid < TS) L.val[tid] = n_x;
        }
        __syncthreads();
        // distinct rows of the sub-tile (the lane that claims a slot represents
        // its row) and each nonzero's rank among the nonzeros of its row
        bool rep = false;
        uint32_t ss = 0, rk = 0;
        if (valid) {
            ss = mix_hash(row) & (uint32_t)(kSubH - 1);
            for (;;) {
                const uint32_t prev = atomicCAS(&L.skey[ss], kNoRow, row);
                if (prev == kNoRow) {
                    rep = true;
                    break;
                }
                if (prev == row) break;
                ss = (ss + 1) & (uint32_t)(kSubH - 1);
            }
            L.sslot[tid] = (uint16_t)ss;
            rk = atomicAdd(&L.scnt[ss], 1u);
        }
        if (KIND != KIND_PRIV) {
            // representatives look their row up in the accumulator table
            uint32_t hs = 0;
            bool is_new = false;
            if (rep) {
                hs = mix_hash(row) & (uint32_t)(H - 1);
                for (;;) {
                    const uint32_t k = L.hkey[hs];
                    if (k == row) break;
                    if (k == kNoRow) {
                        is_new = true;
                        break;
                    }
                    hs = (hs + 1) & (uint32_t)(H - 1);
                }
                if (is_new) atomicAdd(&s_new, 1);
                else L.smap[ss] = L.hidx[hs];
            }
            __syncthreads();
            if (tid == 0) s_flush = (s_occ + s_new > cap) ? 1 : 0;
            __syncthreads();
            if (s_flush) {
                flush();
                // every row of this sub-tile is new now
                if (rep && !is_new) is_new = true;
            }
            if (rep && is_new) {
                const int ai = atomicAdd(&s_occ, 1);
                L.arow[ai] = row;
                uint32_t h2 = mix_hash(row) & (uint32_t)(H - 1);
                for (;;) {
                    if (atomicCAS(&L.hkey[h2], kNoRow, row) == kNoRow) break;
                    h2 = (h2 + 1) & (uint32_t)(H - 1);
                }
                L.hidx[h2] = (uint16_t)ai;
                L.smap[ss] = (uint16_t)ai;
            }
        }
        __syncthreads();
        if (KIND != KIND_COUNT) {
            // counting sort of the sub-tile by slot: runs of equal row become contiguous
            block_scan_lds(L.scnt, kSubH, kTT, s_wsum);
            if (valid) L.ord[L.scnt[ss] + rk] = (uint16_t)tid;
            __syncthreads();
        }
        prefetch(sub + 1);
        if (KIND == KIND_COUNT) continue;

        // ---- walk: a lane group takes CH consecutive nonzeros of the sub-tile,
        // issues all their factor-row gathers, then merges runs of equal
        // accumulator row in registers and adds each run into LDS
        constexpr int GROUPS = kTT / G;
        constexpr int CH = (TS / GROUPS) > 0 ? TS / GROUPS : 1;
        constexpr int UB = CH < 8 ? CH : 8;
        const int g = tid / G, j = tid % G;
        const int q0 = g * CH, q1 = min(q0 + CH, cnt);
        uint32_t cur = kNoRow;
        float acc[NB][VEC];
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[b][v] = 0.f;
        // accumulator row of the nonzero at sorted position q
        auto acc_row = [&](int q) -> uint32_t {
            const int e = L.ord[q];
            return KIND == KIND_PRIV ? L.crd[mode * TS + e] : (uint32_t)L.smap[L.sslot[e]];
        };
        // a run that is a whole segment of the sub-tile belongs to this group alone
        // and is added with plain LDS read-modify-writes; a run cut by a chunk edge
        // shares its row with the neighbouring group and is added atomically
        const uint32_t row_before = (q0 > 0 && q0 < cnt) ? acc_row(q0 - 1) : kNoRow;
        const uint32_t row_after = (q1 < cnt) ? acc_row(q1) : kNoRow;
        bool run_whole_start = true;
        auto add_run = [&](uint32_t ai, bool whole) {
            float *dst = L.acc + (size_t)ai * stride;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int c = (b * G + j) * VEC;
                if (c < ncols) {
#pragma unroll
                    for (int v = 0; v < VEC; ++v) {
                        if (whole) dst[c + v] += acc[b][v];
                        else atomicAdd(dst + c + v, acc[b][v]);
                    }
                }
            }
        };
        for (int q = q0; q < q1; q += UB) {
            uint32_t ai[UB];
            bool ok[UB];
            int ee[UB];
            float p[UB][NB][VEC];
#pragma unroll
            for (int u = 0; u < UB; ++u) {
                ok[u] = (q + u) < q1;
                const int qq = ok[u] ? q + u : q0;
                ee[u] = L.ord[qq];
                ai[u] = KIND == KIND_PRIV ? L.crd[mode * TS + ee[u]] : (uint32_t)L.smap[L.sslot[ee[u]]];
                const float x = L.val[ee[u]];
#pragma unroll
                for (int b = 0; b < NB; ++b)
#pragma unroll
                    for (int v = 0; v < VEC; ++v) p[u][b][v] = x;
            }
#pragma unroll
            for (int k = 0; k < NMAX; ++k) {
                if (k < nm && k != mode) {
                    const float *__restrict__ F = a.f[k];
                    float xv[UB][NB][VEC];
#pragma unroll
                    for (int u = 0; u < UB; ++u) {
                        const float *fr = F + (int64_t)L.crd[k * TS + ee[u]] * R + colbase;
#pragma unroll
                        for (int b = 0; b < NB; ++b) {
                            const int c = (b * G + j) * VEC;
                            if (c < ncols) {
                                load_vec<VEC>(fr + c, xv[u][b]);
                            } else {
#pragma unroll
                                for (int v = 0; v < VEC; ++v) xv[u][b][v] = 0.f;
                            }
                        }
                    }
#pragma unroll
                    for (int u = 0; u < UB; ++u)
#pragma unroll
                        for (int b = 0; b < NB; ++b)
#pragma unroll
                            for (int v = 0; v < VEC; ++v) p[u][b][v] *= xv[u][b][v];
                }
            }
#pragma unroll
            for (int u = 0; u < UB; ++u) {
                if (ok[u]) {
                    if (ai[u] != cur) {
                        if (cur != kNoRow) {
                            add_run(cur, run_whole_start);
                            run_whole_start = true;
                        } else {
                            run_whole_start = ai[u] != row_before;
                        }
                        cur = ai[u];
#pragma unroll
                        for (int b = 0; b < NB; ++b)
#pragma unroll
                            for (int v = 0; v < VEC; ++v) acc[b][v] = p[u][b][v];
                    } else {
#pragma unroll
                        for (int b = 0; b < NB; ++b)
#pragma unroll
                            for (int v = 0; v < VEC; ++v) acc[b][v] += p[u][b][v];
                    }
                }
            }
        }
        if (cur != kNoRow) add_run(cur, run_whole_start && cur != row_after);
        __syncthreads();
    }

    if (KIND == KIND_TABLE) {
        __syncthreads();
        flush();
    } else if (KIND == KIND_COUNT) {
        __syncthreads();
        if (tid == 0) t.rec_cnt[w] = s_rec + s_occ;
    } else {
        // PRIV: this workgroup's partial of the output column slice
        __syncthreads();
        float *dst = t.rec_val + (size_t)w * cap * R;
        for (int i = tid; i < cap * ncols; i += kTT) {
            const int r = i / ncols, c = i - r * ncols;
            dst[(size_t)r * R + colbase + c] = L.acc[r * stride + c];
        }
    }
}

// out[r][c] = sum over workgroups of part[w][r][c]
__global__ __launch_bounds__(256) void k_reduce_priv(const float *__restrict__ part, int64_t nwg, int64_t rows, int R,
                                                     float *__restrict__ out) {
    const int64_t n = rows * R;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        float s = 0.f;
        for (int64_t w = 0; w < nwg; ++w) s += part[w * n + i];
        out[i] = s;
    }
}

// Records sorted by row: lane groups sum runs of equal row over a chunk of
// records (8 record loads in flight per lane); a run wholly inside the chunk
// is stored, a run crossing a chunk edge is added atomically (out was zeroed).
#ifndef SPT_RED_UB
#define SPT_RED_UB 8
#endif
#ifndef SPT_RED_CHUNK
#define SPT_RED_CHUNK 512
#endif

template <int G, int VEC, int NB>
__global__ __launch_bounds__(256) void k_reduce_records(const uint64_t *__restrict__ srow,
                                                        const uint32_t *__restrict__ sidx,
                                                        const float *__restrict__ rec_val, int64_t P, int R,
                                                        int chunk, int64_t rows, float *__restrict__ out) {
    constexpr int GROUPS = 256 / G;
    constexpr int UB = SPT_RED_UB;
    const int g = threadIdx.x / G, j = threadIdx.x % G;
    const int64_t c0 = ((int64_t)blockIdx.x * GROUPS + g) * chunk;
    if (c0 >= P) return;
    const int64_t c1 = min(c0 + chunk, P);
    const uint64_t before = c0 > 0 ? srow[c0 - 1] : ~0ull;
    const uint64_t after = c1 < P ? srow[c1] : ~0ull;
    uint64_t cur = srow[c0];
    bool starts_here = cur != before;
    float acc[NB][VEC];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[b][v] = 0.f;
    auto emit = [&](uint64_t r, bool whole) {
        if (r >= (uint64_t)rows) return;  // sentinel records of unused slots
        float *o = out + (int64_t)r * R;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int c = (b * G + j) * VEC;
            if (c < R) {
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    if (whole) o[c + v] = acc[b][v];
                    else unsafeAtomicAdd(o + c + v, acc[b][v]);
                }
            }
        }
    };
    for (int64_t q = c0; q < c1; q += UB) {
        uint64_t r[UB];
        float x[UB][NB][VEC];
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            const bool ok = q + u < c1;
            r[u] = ok ? srow[q + u] : ~0ull;
            // sidx null: the records are already grouped by row (identity order)
            const int64_t ri = ok ? (sidx ? (int64_t)sidx[q + u] : q + u) : 0;
            const float *src = rec_val + ri * R;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int c = (b * G + j) * VEC;
                if (ok && c < R) {
                    load_vec<VEC>(src + c, x[u][b]);
                } else {
#pragma unroll
                    for (int v = 0; v < VEC; ++v) x[u][b][v] = 0.f;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            if (q + u < c1) {
                if (r[u] != cur) {
                    emit(cur, starts_here);
                    cur = r[u];
                    starts_here = true;
#pragma unroll
                    for (int b = 0; b < NB; ++b)
#pragma unroll
                        for (int v = 0; v < VEC; ++v) acc[b][v] = x[u][b][v];
                } else {
#pragma unroll
                    for (int b = 0; b < NB; ++b)
#pragma unroll
                        for (int v = 0; v < VEC; ++v) acc[b][v] += x[u][b][v];
                }
            }
        }
    }
    emit(cur, starts_here && cur != after);
}

template <int NMAX, int KIND, int G, int VEC, int NB>
spt_status launch_k(const TableArgs &t, dim3 grid, size_t lds, hipStream_t s) {
    if (t.ts == 256)
        hipLaunchKernelGGL((k_mttkrp_table<G, VEC, NB, NMAX, KIND, 256>), grid, dim3(kTT), lds, s, t);
    else
        hipLaunchKernelGGL((k_mttkrp_table<G, VEC, NB, NMAX, KIND, 512>), grid, dim3(kTT), lds, s, t);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

// column mapping of the walk for `cols` columns (same rules as the plain MTTKRP kernels)
template <int NMAX, int KIND>
spt_status launch_kind(const TableArgs &t, int cols, dim3 grid, size_t lds, hipStream_t s) {
    if ((cols & 3) == 0 && (t.a.rank & 3) == 0) {
        const int c4 = cols >> 2;
        if (c4 <= 1) return launch_k<NMAX, KIND, 1, 4, 1>(t, grid, lds, s);
        if (c4 <= 2) return launch_k<NMAX, KIND, 2, 4, 1>(t, grid, lds, s);
        if (c4 <= 4) return launch_k<NMAX, KIND, 4, 4, 1>(t, grid, lds, s);
        if (c4 <= 8) return launch_k<NMAX, KIND, 8, 4, 1>(t, grid, lds, s);
        if (c4 <= 16) return launch_k<NMAX, KIND, 16, 4, 1>(t, grid, lds, s);
        if (c4 <= 32) return launch_k<NMAX, KIND, 32, 4, 1>(t, grid, lds, s);
        return launch_k<NMAX, KIND, 64, 4, 1>(t, grid, lds, s);
    }
    if (cols <= 64) return launch_k<NMAX, KIND, 64, 1, 1>(t, grid, lds, s);
    if (cols <= 128) return launch_k<NMAX, KIND, 64, 1, 2>(t, grid, lds, s);
    if (cols <= 192) return launch_k<NMAX, KIND, 64, 1, 3>(t, grid, lds, s);
    return launch_k<NMAX, KIND, 64, 1, 4>(t, grid, lds, s);
}

template <int KIND>
spt_status launch_nm(const TableArgs &t, int cols, dim3 grid, size_t lds, hipStream_t s) {
    if (t.a.nmodes <= 4) return launch_kind<4, KIND>(t, cols, grid, lds, s);
    return launch_kind<8, KIND>(t, cols, grid, lds, s);
}

}  // namespace

size_t table_lds_needed(int nmodes, int ts, int cap, int hbits, int stride, bool priv, bool with_acc) {
    return table_lds_bytes(nmodes <= 4 ? 4 : 8, ts, cap, hbits, stride, priv, with_acc);
}

spt_status launch_table_count(const TableArgs &t, int nwg, hipStream_t s) {
    const size_t lds = table_lds_needed(t.a.nmodes, t.ts, t.cap, t.hbits, t.stride, false, false);
    return launch_nm<KIND_COUNT>(t, t.a.rank, dim3(nwg), lds, s);
}

spt_status launch_table(const TableArgs &t, int nwg, hipStream_t s) {
    const size_t lds = table_lds_needed(t.a.nmodes, t.ts, t.cap, t.hbits, t.stride, false, true);
    return launch_nm<KIND_TABLE>(t, t.a.rank, dim3(nwg), lds, s);
}

spt_status launch_priv(const TableArgs &t, int nwg, int npass, hipStream_t s) {
    const size_t lds = table_lds_needed(t.a.nmodes, t.ts, t.cap, 0, t.stride, true, true);
    return launch_nm<KIND_PRIV>(t, t.rs, dim3(nwg, npass), lds, s);
}

spt_status launch_reduce_priv(const float *part, int nwg, int64_t rows, int R, float *out, hipStream_t s) {
    int64_t g = (rows * R + 255) / 256;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_reduce_priv, dim3((unsigned)g), dim3(256), 0, s, part, (int64_t)nwg, rows, R, out);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

spt_status launch_reduce_records(const uint64_t *srow, const uint32_t *sidx, const float *rec_val, int64_t P, int R,
                                 int64_t rows, float *out, hipStream_t s) {
    if (P <= 0) return SPT_OK;
    // Long chunks mean fewer runs cut at a chunk edge (atomics), short ones
    // less serial work per lane group: the longest chunk (up to
    // SPT_RED_CHUNK) that still leaves 4096 lane groups, at least 64 records.
    int chunk = SPT_RED_CHUNK;
    while (chunk > 64 && P / chunk < 4096) chunk >>= 1;
    auto go = [&](auto kern, int G) -> spt_status {
        const int groups = 256 / G;
        const int64_t blocks = (P + (int64_t)groups * chunk - 1) / ((int64_t)groups * chunk);
        hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), 0, s, srow, sidx, rec_val, P, R, chunk, rows, out);
        SPT_HIP(hipGetLastError());
        return SPT_OK;
    };
    if ((R & 3) == 0) {
        const int r4 = R >> 2;
        if (r4 <= 1) return go(k_reduce_records<1, 4, 1>, 1);
        if (r4 <= 2) return go(k_reduce_records<2, 4, 1>, 2);
        if (r4 <= 4) return go(k_reduce_records<4, 4, 1>, 4);
        if (r4 <= 8) return go(k_reduce_records<8, 4, 1>, 8);
        if (r4 <= 16) return go(k_reduce_records<16, 4, 1>, 16);
        if (r4 <= 32) return go(k_reduce_records<32, 4, 1>, 32);
        return go(k_reduce_records<64, 4, 1>, 64);
    }
    if (R <= 64) return go(k_reduce_records<64, 1, 1>, 64);
    if (R <= 128) return go(k_reduce_records<64, 1, 2>, 64);
    if (R <= 192) return go(k_reduce_records<64, 1, 3>, 64);
    return go(k_reduce_records<64, 1, 4>, 64);
}

}  // namespace spt
