// SEGMENT strategy of mode-n MTTKRP (Section II-B, Fig. 2) on gfx950.
//
// A workgroup of NT threads owns a tile of T = 4 NT consecutive nonzeros of
// the key-ordered stream.  Conflicts on output rows are resolved by
// regrouping the tile by output row and cutting every row's run into pieces
// of at most L nonzeros; each piece is summed in registers (a segmented
// reduction over equal output index) and written as one record (row, R
// floats) with plain stores; the records are summed per row afterwards
// (mttkrp_table.hip).  No atomics on the main path.
//
// Plan (once per tensor and mode, the hashing stage below): an LDS hash of
// the tile's output rows (T slots, linear probing, CAS), one block scan of
// packed (nonzeros << 16 | pieces) per slot, giving every nonzero its
// position in row-grouped order and every piece its start, length and row.
// The (tile, row) pairs are then sorted by row across the tensor (or the
// batch) and scanned, which lays the records out grouped by row.
//
// Call (the planned kernel): coalesced non-temporal loads of keys, values and
// plan positions; the non-output coordinates are decoded from the bit runs
// held in VGPRs and scattered once to LDS in row-grouped order; lane groups
// (G lanes x VEC columns) take the tile's pieces (stored longest first) in
// snake order, gather the N-1 factor rows of the piece's nonzeros with
// buffer loads, form v * Hadamard, sum and store the record at its
// plan-given slot.  No hashing, atomics or scans at run time.
//
// Row-cached call (4096-nonzero tiles, 2..4 modes): the tile dictionaries
// (per mode, each tile's distinct rows most frequent first, and each
// nonzero's index in that list) replace the key decode; the first cap rows
// of every non-output mode's list are copied to LDS and a nonzero reads its
// factor row there when its index is below cap.
#include <atomic>

#include "tile_common.h"

#ifndef SPT_SEG_UB
#define SPT_SEG_UB 1
#endif
#ifndef SPT_SEG_PIECE
#define SPT_SEG_PIECE 64
#endif

namespace spt {

namespace {

constexpr int kPiece = SPT_SEG_PIECE;  // nonzeros per piece (L)
constexpr int kUnroll = SPT_SEG_UB;    // nonzeros in flight per lane group
constexpr int kUnrollDict = 2;       // the same, row-cached walk
#ifndef SPT_SEGP_NT4096
#define SPT_SEGP_NT4096 1024
#endif
constexpr int kSegpThreads4096 = SPT_SEGP_NT4096;  // threads of the MTTKRP kernel on 4096-nonzero tiles

// A tile staged together with its hash tables: crdg[nm - 1][T] u32
// (non-output coordinates, row-grouped), valg[T] f32, hkey[T] u32 (slot ->
// row), hcnt[T + 4] u32 (packed counts, then prefixes; entry T holds the
// totals), ptab[T] u16 (piece -> slot).  The budget that decides which tile
// sizes a tensor of nmodes modes may use (seg_tile_ok).
__host__ __device__ inline size_t seg_lds_bytes(int T, int nmodes) {
    return (size_t)(nmodes - 1) * T * 4 + (size_t)T * 4 + (size_t)T * 4 + (size_t)(T + 4) * 4 + (size_t)T * 2;
}

// LDS of the planned kernel: crdg[nm - 1][T] and valg[T].
__host__ __device__ inline size_t segp_lds_bytes(int T, int nmodes) {
    return (size_t)(nmodes - 1) * T * 4 + (size_t)T * 4;
}

struct SegLds {
    uint32_t *crdg;
    float *valg;
    uint32_t *hkey;
    uint32_t *hcnt;
    uint16_t *ptab;
};

// LDS of the plan's counting and emission passes, which stage nothing:
// occ[T] u32 (emission's pair index per slot), hkey[T], hcnt[T + 4] u32 and
// ptab[T] u16.  About half of seg_lds_bytes at 4 modes, so two 1024-thread
// workgroups share a CU.
__host__ __device__ inline size_t seg_plan_lds_bytes(int T) { return (size_t)T * 12 + 16 + (size_t)T * 2; }

__device__ __forceinline__ SegLds seg_carve_plan(char *p, int T) {
    SegLds L;
    L.crdg = nullptr;
    L.valg = (float *)p;
    L.hkey = (uint32_t *)(L.valg + T);
    L.hcnt = L.hkey + T;
    L.ptab = (uint16_t *)(L.hcnt + T + 4);
    return L;
}

// Stage and regroup one tile.  After return: hcnt[s] = (first position of
// slot s) << 16 | (first piece of slot s); hcnt[T] = (cnt << 16) | pieces;
// crdg/valg hold the tile in row-grouped order and ptab maps pieces to slots.
// With SCATTER false only the counts are formed (the plan's counting pass).
// With pos_out (counting mode only) the row-grouped position of every element
// is written to pos_out[tile * T + e] and the piece table is built as well.
template <int NT, int NMAX, bool SCATTER>
__device__ __forceinline__ void seg_stage(const MttkrpArgs &a, int64_t tile, const SegLds &L, const CodecRegs &cr,
                                          uint32_t *wsum, uint16_t *__restrict__ pos_out = nullptr) {
    constexpr int T = 4 * NT;
    const int tid = threadIdx.x;
    const int64_t base = tile * (int64_t)T;
    const int64_t rem = a.nnz - base;
    const int cnt = rem < T ? (int)rem : T;
    for (int i = tid; i < T; i += NT) {
        L.hkey[i] = kNoRow;
        L.hcnt[i] = 0;
    }
    uint32_t w[4][4];
    float v[4];
    const int nwords = 2 * a.codec.key_words;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = tid + u * NT;
        uint64_t klo = 0, khi = 0;
        float x = 0.f;
        if (e < cnt) {
            klo = __builtin_nontemporal_load(a.lo + base + e);
            if (nwords == 4) khi = __builtin_nontemporal_load(a.hi + base + e);
            if (SCATTER) x = __builtin_nontemporal_load(a.vals + base + e);
        }
        w[u][0] = (uint32_t)klo;
        w[u][1] = (uint32_t)(klo >> 32);
        w[u][2] = (uint32_t)khi;
        w[u][3] = (uint32_t)(khi >> 32);
        v[u] = x;
    }
    // coordinates of every mode (only the output mode when counting)
    uint32_t xc[NMAX][4];
#pragma unroll
    for (int k = 0; k < NMAX; ++k) {
#pragma unroll
        for (int u = 0; u < 4; ++u) xc[k][u] = 0;
        if (k < a.nmodes && (SCATTER || k == a.mode)) {
#pragma unroll
            for (int word = 0; word < 4; ++word) {
                if (word < nwords) {
                    const int r0 = __builtin_amdgcn_readlane(cr.rb, k * 5 + word);
                    const int r1 = __builtin_amdgcn_readlane(cr.rb, k * 5 + word + 1);
                    for (int r = r0; r < r1; ++r) {
                        const uint32_t d = run_desc(cr, r);
                        const uint32_t kpos = (d >> 8) & 31u, cpos = (d >> 16) & 31u, len = d >> 24;
#pragma unroll
                        for (int u = 0; u < 4; ++u) xc[k][u] |= __builtin_amdgcn_ubfe(w[u][word], kpos, len) << cpos;
                    }
                }
            }
        }
    }
    uint32_t rowv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        rowv[u] = 0;
#pragma unroll
        for (int k = 0; k < NMAX; ++k)
            if (k == a.mode) rowv[u] = xc[k][u];
    }
    __syncthreads();  // hash cleared
    uint32_t sr[4];   // slot << 16 | rank within the slot
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = tid + u * NT;
        sr[u] = 0;
        if (e < cnt) {
            const uint32_t row = rowv[u];
            uint32_t s = mix_hash(row) & (uint32_t)(T - 1);
            for (;;) {
                const uint32_t prev = atomicCAS(&L.hkey[s], kNoRow, row);
                if (prev == kNoRow || prev == row) break;
                s = (s + 1) & (uint32_t)(T - 1);
            }
            sr[u] = (s << 16) | atomicAdd(&L.hcnt[s], 1u);
        }
    }
    __syncthreads();
    // packed (count << 16 | pieces) per slot, then one exclusive scan
    for (int i = tid; i < T; i += NT) {
        const uint32_t c = L.hcnt[i];
        L.hcnt[i] = (c << 16) | ((c + kPiece - 1) / kPiece);
    }
    __syncthreads();
    block_scan_lds(L.hcnt, T, NT, wsum);
    if (tid == 0) {
        // totals: elements = cnt; pieces = prefix of the last slot plus its own pieces
        const uint32_t pl = L.hcnt[T - 1] & 0xFFFFu;
        const uint32_t el = L.hcnt[T - 1] >> 16;
        const uint32_t own = (uint32_t)cnt - el;
        L.hcnt[T] = ((uint32_t)cnt << 16) | (pl + (own + kPiece - 1) / kPiece);
    }
    if (SCATTER || pos_out) {
        const int nm = a.nmodes, mode = a.mode;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + u * NT;
            if (e < cnt) {
                const int pos = (int)(L.hcnt[sr[u] >> 16] >> 16) + (int)(sr[u] & 0xFFFFu);
                if constexpr (SCATTER) {
                    L.valg[pos] = v[u];
#pragma unroll
                    for (int k = 0; k < NMAX; ++k)
                        if (k < nm && k != mode) L.crdg[(k - (k > mode)) * T + pos] = xc[k][u];
                } else {
                    pos_out[base + e] = (uint16_t)pos;
                }
            }
        }
        __syncthreads();  // totals visible
        for (int i = tid; i < T; i += NT) {
            const uint32_t pk = L.hcnt[i];
            const uint32_t nx = i + 1 < T ? L.hcnt[i + 1] : L.hcnt[T];
            const uint32_t c = (nx >> 16) - (pk >> 16);
            const uint32_t p0 = pk & 0xFFFFu, np = (c + kPiece - 1) / kPiece;
            for (uint32_t q = 0; q < np; ++q) L.ptab[p0 + q] = (uint16_t)i;
        }
    }
    __syncthreads();
}

// Walk the staged tile: every piece (nonzeros [p0, p1) of the row-grouped
// tile, one output row) becomes one record of ld floats (columns R..ld-1
// zero) at the position the piece source gives, with row row_base + its row.
// EXACT: the lane groups cover exactly R columns (no column mask).
// With at most 4 modes every nonzero slot of an unrolled step reads all its
// coordinates from LDS first, then issues every factor-row gather, then waits
// once; with more modes the gathers go mode by mode.  NFIX > 0: the tensor has
// exactly NFIX modes (no run-time mode test between the gathers, which would
// otherwise make the compiler wait for one mode's rows before the next
// mode's gathers are issued).
// DICT: a crdg entry is either the byte offset in `ldsb` of a row held in
// the LDS row cache (at most lim, the offset of the cache's last row) or, with
// kDictMiss set, a global row.  Every lane reads its step's rows from LDS
// first, then the lanes whose row is global load it over the LDS value.
template <int NT, int T, int G, int VEC, int NB, int NMAX, int NFIX, bool EXACT, class Pieces, bool DICT = false>
__device__ __forceinline__ void seg_walk(const MttkrpArgs &a, const uint32_t *__restrict__ crdg,
                                         const float *__restrict__ valg, int npieces, const Pieces &pieces,
                                         uint64_t *__restrict__ rec_row, float *__restrict__ rec_val, int ld,
                                         int64_t row_base, const char *__restrict__ ldsb = nullptr, uint32_t lim = 0) {
    constexpr int UB = DICT ? kUnrollDict : kUnroll;
    constexpr int NO = NMAX - 1;  // non-output modes at most
    const int j = threadIdx.x % G;
    static_assert(NFIX == 0 || NFIX == NMAX, "a fixed mode count is the maximum");
    static_assert(!DICT || NMAX <= 4, "the row cache serves at most 3 non-output modes");
    const int R = a.rank, mode = a.mode, no = NFIX ? NFIX - 1 : a.nmodes - 1;
    // factor of the o-th non-output mode as a row buffer
    spt_i4 fb[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        const int k = o + (o >= mode);
        fb[o] = o < no ? row_rsrc(a.f[k], R, a.frows[k]) : row_rsrc(nullptr, R, 0u);
    }
    constexpr int NG = NT / G;
    if (npieces <= 0) return;
    // pieces are dealt in snake order (round r: group g, then NG - 1 - g),
    // which balances the groups when the plan lists the pieces longest first
    const int g = threadIdx.x / G;
    const int nr = (npieces + NG - 1) / NG;
    auto kof = [&](int r) { return min(r * NG + ((r & 1) ? NG - 1 - g : g), npieces - 1); };
    typename Pieces::Raw cur = pieces.fetch(kof(0));
    for (int r = 0; r < nr; ++r) {
        const int k = r * NG + ((r & 1) ? NG - 1 - g : g);
        // the next piece's descriptor is fetched while this one is walked
        const typename Pieces::Raw nxt = pieces.fetch(kof(r + 1));
        int p0, p1;
        uint32_t prow;
        int64_t pos;
        const bool live = k < npieces && pieces.decode(k, cur, p0, p1, prow, pos);
        cur = nxt;
        if (!live) continue;
        float acc[NB][VEC];
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[b][v] = 0.f;
        for (int q = p0; q < p1; q += UB) {
            int pp[UB];
            float x[UB];
#pragma unroll
            for (int u = 0; u < UB; ++u) {
                const bool ok = q + u < p1;
                pp[u] = ok ? q + u : p1 - 1;  // in range either way; the value is zeroed
                const float v = valg[pp[u]];
                x[u] = ok ? v : 0.f;
            }
            float p[UB][NB][VEC];
#pragma unroll
            for (int u = 0; u < UB; ++u)
#pragma unroll
                for (int b = 0; b < NB; ++b)
#pragma unroll
                    for (int v = 0; v < VEC; ++v) p[u][b][v] = x[u];
            if constexpr (NO <= 3) {
                uint32_t row[NO][UB];
#pragma unroll
                for (int o = 0; o < NO; ++o)
                    if (o < no)
#pragma unroll
                        for (int u = 0; u < UB; ++u) row[o][u] = crdg[o * T + pp[u]];
                float xv[NO][UB][NB][VEC];
                if constexpr (DICT) {
                    // every index read of the step is issued before anything
                    // waits for one (the scheduler may not hoist a use between them)
                    __builtin_amdgcn_sched_barrier(0);
                    // Every lane first reads LDS (a miss reads the last cached
                    // row: its entry, flag set, clamps to lim), then the misses
                    // load their rows globally into the same registers.  A global
                    // load into the registers of an LDS read waits for that read;
                    // with all LDS reads of the step issued first the loads wait
                    // for one LDS round trip, and no branch splits hits from misses.
#pragma unroll
                    for (int o = 0; o < NO; ++o) {
#pragma unroll
                        for (int u = 0; u < UB; ++u) {
                            const uint32_t off = min(row[o][u], lim);
#pragma unroll
                            for (int b = 0; b < NB; ++b) {
                                const int c = (b * G + j) * VEC;
                                if (o < no && (EXACT || c < R)) {
                                    const float *cp = reinterpret_cast<const float *>(ldsb + off) + c;
                                    if constexpr (VEC == 4) {
                                        const float4 t4 = *reinterpret_cast<const float4 *>(cp);
                                        xv[o][u][b][0] = t4.x;
                                        xv[o][u][b][1] = t4.y;
                                        xv[o][u][b][2] = t4.z;
                                        xv[o][u][b][3] = t4.w;
                                    } else {
#pragma unroll
                                        for (int v = 0; v < VEC; ++v) xv[o][u][b][v] = cp[v];
                                    }
                                }
                            }
                        }
                    }
#pragma unroll
                    for (int o = 0; o < NO; ++o) {
                        if (o < no) {
#pragma unroll
                            for (int u = 0; u < UB; ++u) {
                                const uint32_t rv = row[o][u];
#pragma unroll
                                for (int b = 0; b < NB; ++b) {
                                    const int c = (b * G + j) * VEC;
                                    if (EXACT || c < R) {
                                        if (rv & kDictMiss) load_row_vec<VEC>(fb[o], rv & ~kDictMiss, c, xv[o][u][b]);
                                    } else {
#pragma unroll
                                        for (int v = 0; v < VEC; ++v) xv[o][u][b][v] = 0.f;
                                    }
                                }
                            }
                        }
                    }
                } else {
#pragma unroll
                    for (int o = 0; o < NO; ++o) {
                        if (o < no) {
#pragma unroll
                            for (int u = 0; u < UB; ++u) {
#pragma unroll
                                for (int b = 0; b < NB; ++b) {
                                    const int c = (b * G + j) * VEC;
                                    if (EXACT || c < R) {
                                        load_row_vec<VEC>(fb[o], row[o][u], c, xv[o][u][b]);
                                    } else {
#pragma unroll
                                        for (int v = 0; v < VEC; ++v) xv[o][u][b][v] = 0.f;
                                    }
                                }
                            }
                        }
                    }
                }
#pragma unroll
                for (int o = 0; o < NO; ++o)
                    if (o < no)
#pragma unroll
                        for (int u = 0; u < UB; ++u)
#pragma unroll
                            for (int b = 0; b < NB; ++b)
#pragma unroll
                                for (int v = 0; v < VEC; ++v) p[u][b][v] *= xv[o][u][b][v];
            } else {
#pragma unroll
                for (int o = 0; o < NO; ++o) {
                    if (o < no) {
                        float xv[UB][NB][VEC];
#pragma unroll
                        for (int u = 0; u < UB; ++u) {
                            const uint32_t rw = crdg[o * T + pp[u]];
#pragma unroll
                            for (int b = 0; b < NB; ++b) {
                                const int c = (b * G + j) * VEC;
                                if (EXACT || c < R) {
                                    load_row_vec<VEC>(fb[o], rw, c, xv[u][b]);
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
            }
#pragma unroll
            for (int u = 0; u < UB; ++u)
#pragma unroll
                for (int b = 0; b < NB; ++b)
#pragma unroll
                    for (int v = 0; v < VEC; ++v) acc[b][v] += p[u][b][v];
        }
        if (j == 0) rec_row[pos] = (uint64_t)(row_base + prow);
        float *o = rec_val + pos * ld;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int c = (b * G + j) * VEC;
            if (EXACT || c < ld) {
                if constexpr (VEC == 4) {
                    // columns at or beyond R were loaded as zero factors, so acc is 0 there
                    *reinterpret_cast<float4 *>(o + c) = make_float4(acc[b][0], acc[b][1], acc[b][2], acc[b][3]);
                } else {
#pragma unroll
                    for (int v = 0; v < VEC; ++v) o[c + v] = acc[b][v];
                }
            }
        }
    }
}

// Pieces given by the plan, read from global memory (the tile's range
// starts at k0).  Reads stay inside the tile and a record outside the plan's
// range is never written, whatever the plan holds.
template <int T>
struct PlanPieces {
    const uint32_t *__restrict__ pdesc, *__restrict__ prow, *__restrict__ pdst;
    int64_t k0, cap, rec_base;
    struct Raw {
        uint32_t d, r, x;
    };
    __device__ __forceinline__ Raw fetch(int k) const { return Raw{pdesc[k0 + k], prow[k0 + k], pdst[k0 + k]}; }
    __device__ __forceinline__ bool decode(int, const Raw &q, int &p0, int &p1, uint32_t &row, int64_t &pos) const {
        p0 = (int)(q.d & 0xFFFFu);
        p1 = min(p0 + (int)(q.d >> 16), T);
        row = q.r;
        pos = rec_base + q.x;
        return q.x < cap && p0 < p1;
    }
};

// The same from the packed plan of one tensor: one 16-byte load per piece.
template <int T>
struct PackedPieces {
    const spt_u4 *__restrict__ pk;
    int64_t k0, cap;
    using Raw = spt_u4;
    __device__ __forceinline__ Raw fetch(int k) const { return pk[k0 + k]; }
    __device__ __forceinline__ bool decode(int, const Raw &q, int &p0, int &p1, uint32_t &row, int64_t &pos) const {
        p0 = (int)(q.x & 0xFFFFu);
        p1 = min(p0 + (int)(q.x >> 16), T);
        row = q.y;
        pos = q.z;
        return q.z < cap && p0 < p1;
    }
};

// Planned SEGMENT kernel.  The plan holds, per nonzero, its position in the
// tile's row-grouped order (u16) and, per piece, (start | length << 16, row,
// record), with the records of one row contiguous.  A tile is staged by one
// scatter of values and non-output coordinates to their positions; there is
// no hashing, no atomic and no scan at run time.
// PACKED: the pieces come from a.pl_piece (one tensor, records from 0);
// otherwise from a.pl_desc / pl_row / pl_dest with records from rec_base
// (a batched member).
template <int NT, int T, int G, int VEC, int NB, int NMAX, int NFIX, bool EXACT, bool PACKED>
__device__ __forceinline__ void segp_tile(const MttkrpArgs &a, int64_t tile, char *lds, uint64_t *__restrict__ rec_row,
                                          float *__restrict__ rec_val, int ld, int64_t rec_base, int64_t row_base) {
    constexpr int PER = T / NT;  // nonzeros staged per thread
    static_assert(PER * NT == T && PER >= 1 && PER <= 8, "tile must be 1..8 nonzeros per thread");
    const int nm = NFIX ? NFIX : a.nmodes, mode = a.mode, tid = threadIdx.x;
    uint32_t *crdg = (uint32_t *)lds;
    float *valg = (float *)(crdg + (size_t)(nm - 1) * T);
    const CodecRegs cr = load_codec_regs(a.codec);
    const int64_t k0 = a.pl_off[tile], k1 = min(a.pl_off[tile + 1], k0 + T);  // a tile has at most T pieces
    const int npieces = (int)(k1 - k0);
    const int64_t base = tile * (int64_t)T;
    const int64_t rem = a.nnz - base;
    const int cnt = rem < T ? (int)rem : T;
    const int nwords = 2 * a.codec.key_words;
    uint32_t w[PER][4];
    float v[PER];
    int ps[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int e = tid + u * NT;
        uint64_t klo = 0, khi = 0;
        float x = 0.f;
        int q = 0;
        if (e < cnt) {
            klo = __builtin_nontemporal_load(a.lo + base + e);
            if (nwords == 4) khi = __builtin_nontemporal_load(a.hi + base + e);
            x = __builtin_nontemporal_load(a.vals + base + e);
            q = a.pl_pos[base + e] & (T - 1);  // a position inside the tile
        }
        w[u][0] = (uint32_t)klo;
        w[u][1] = (uint32_t)(klo >> 32);
        w[u][2] = (uint32_t)khi;
        w[u][3] = (uint32_t)(khi >> 32);
        v[u] = x;
        ps[u] = q;
    }
    // decode the non-output coordinates and scatter them with the values
#pragma unroll
    for (int k = 0; k < NMAX; ++k) {
        if (k < nm && k != mode) {
            uint32_t x[PER];
#pragma unroll
            for (int u = 0; u < PER; ++u) x[u] = 0;
#pragma unroll
            for (int word = 0; word < 4; ++word) {
                if (word < nwords) {
                    const int r0 = __builtin_amdgcn_readlane(cr.rb, k * 5 + word);
                    const int r1 = __builtin_amdgcn_readlane(cr.rb, k * 5 + word + 1);
                    for (int r = r0; r < r1; ++r) {
                        const uint32_t d = run_desc(cr, r);
                        const uint32_t kpos = (d >> 8) & 31u, cpos = (d >> 16) & 31u, len = d >> 24;
#pragma unroll
                        for (int u = 0; u < PER; ++u) x[u] |= __builtin_amdgcn_ubfe(w[u][word], kpos, len) << cpos;
                    }
                }
            }
            const int o = k - (k > mode);
#pragma unroll
            for (int u = 0; u < PER; ++u)
                if (tid + u * NT < cnt) crdg[o * T + ps[u]] = x[u];
        }
    }
#pragma unroll
    for (int u = 0; u < PER; ++u)
        if (tid + u * NT < cnt) valg[ps[u]] = v[u];
    __syncthreads();
    if constexpr (PACKED)
        seg_walk<NT, T, G, VEC, NB, NMAX, NFIX, EXACT>(
            a, crdg, valg, npieces, PackedPieces<T>{reinterpret_cast<const spt_u4 *>(a.pl_piece), k0, a.rec_cap},
            rec_row, rec_val, ld, row_base);
    else
        seg_walk<NT, T, G, VEC, NB, NMAX, NFIX, EXACT>(
            a, crdg, valg, npieces, PlanPieces<T>{a.pl_desc, a.pl_row, a.pl_dest, k0, a.rec_cap, rec_base}, rec_row,
            rec_val, ld, row_base);
}

template <int NT, int T, int G, int VEC, int NB, int NMAX, int NFIX, bool EXACT>
__global__ __launch_bounds__(NT) void k_mttkrp_segp(MttkrpArgs a, int64_t ntiles) {
    extern __shared__ __align__(16) char lds[];
    const int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    segp_tile<NT, T, G, VEC, NB, NMAX, NFIX, EXACT, true>(a, tile, lds, a.rec_row, a.rec_val, a.rank, 0, 0);
}

// ---------------------------------------------------------------- row cache
// Tile dictionary (mode-agnostic, tiles of kDictTile nonzeros in key order):
// for every mode k, a tile's distinct mode-k rows, most frequent first, and
// per nonzero the index of its row in that list.  The linearized order keeps
// a tile inside a small sub-box of the index space, so a tile touches few
// distinct rows of every mode (a few hundred per 4096 nonzeros on the ratings
// tensor) and each of them many times.

// Build one mode's dictionary: one workgroup per tile hashes the tile's
// mode-a.mode rows, buckets them by count (64 buckets, counts >= 63 in the
// first), and writes row[off[tile] + i] (i-th most frequent row) and
// slot[e] = i for every nonzero e.  off comes from the counting pass (its
// distinct rows per tile).
template <int NT, int NMAX>
__global__ __launch_bounds__(NT) void k_emit_dict(MttkrpArgs a, const int64_t *__restrict__ off,
                                                  uint32_t *__restrict__ row_out, uint16_t *__restrict__ slot_out) {
    constexpr int T = 4 * NT;
    constexpr int NBK = 64;
    extern __shared__ __align__(16) char lds[];
    __shared__ uint32_t bucket[NBK];
    uint32_t *hkey = (uint32_t *)lds;
    uint32_t *hcnt = hkey + T;
    const int tid = threadIdx.x;
    const int64_t tile = blockIdx.x;
    const int64_t base = tile * (int64_t)T;
    const int64_t rem = a.nnz - base;
    const int cnt = rem < T ? (int)rem : T;
    const int64_t d0 = off[tile], d1 = off[tile + 1];
    for (int i = tid; i < T; i += NT) {
        hkey[i] = kNoRow;
        hcnt[i] = 0;
    }
    if (tid < NBK) bucket[tid] = 0;
    const CodecRegs cr = load_codec_regs(a.codec);
    const int nwords = 2 * a.codec.key_words;
    uint32_t rowv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = tid + u * NT;
        uint32_t w[4] = {0, 0, 0, 0};
        if (e < cnt) {
            const uint64_t klo = a.lo[base + e];
            const uint64_t khi = nwords == 4 ? a.hi[base + e] : 0ull;
            w[0] = (uint32_t)klo;
            w[1] = (uint32_t)(klo >> 32);
            w[2] = (uint32_t)khi;
            w[3] = (uint32_t)(khi >> 32);
        }
        rowv[u] = decode_mode(cr, a.mode, nwords, w);
    }
    __syncthreads();  // hash cleared
    uint32_t hs[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = tid + u * NT;
        hs[u] = 0;
        if (e < cnt) {
            const uint32_t r = rowv[u];
            uint32_t h = mix_hash(r) & (uint32_t)(T - 1);
            for (;;) {
                const uint32_t prev = atomicCAS(&hkey[h], kNoRow, r);
                if (prev == kNoRow || prev == r) break;
                h = (h + 1) & (uint32_t)(T - 1);
            }
            atomicAdd(&hcnt[h], 1u);
            hs[u] = h;
        }
    }
    __syncthreads();
    auto bucket_of = [](uint32_t c) { return c >= (uint32_t)(NBK - 1) ? 0u : (uint32_t)(NBK - 1) - c; };
    for (int i = tid; i < T; i += NT)
        if (hkey[i] != kNoRow) atomicAdd(&bucket[bucket_of(hcnt[i])], 1u);
    __syncthreads();
    if (tid == 0) {
        uint32_t run = 0;
        for (int b = 0; b < NBK; ++b) {
            const uint32_t c = bucket[b];
            bucket[b] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int i = tid; i < T; i += NT) {
        if (hkey[i] != kNoRow) {
            const uint32_t d = atomicAdd(&bucket[bucket_of(hcnt[i])], 1u);
            if (d0 + d < d1) row_out[d0 + d] = hkey[i];
            hcnt[i] = d;  // the slot now holds its row's dictionary index
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = tid + u * NT;
        if (e < cnt) slot_out[base + e] = (uint16_t)hcnt[hs[u]];
    }
}

// LDS of the row-cached kernel: crdg[nm - 1][T], valg[T], then the cache of
// cap rows of R floats per non-output mode.
__host__ __device__ inline size_t segd_lds_bytes(int T, int nmodes, int cap, int R) {
    return segp_lds_bytes(T, nmodes) + (size_t)(nmodes - 1) * cap * R * 4;
}

// Row-cached form of segp_tile (tiles of kDictTile nonzeros).  Staging reads
// no keys: per nonzero the value, its plan position and its dictionary index
// in every non-output mode.  The first cap rows of each non-output mode's
// tile dictionary are copied to LDS; a nonzero whose index is below cap
// reads its factor row there, any other reads it from HBM/L2 by its global
// row.
template <int NT, int T, int G, int VEC, int NB, int NMAX, int NFIX, bool EXACT>
__device__ __forceinline__ void segd_tile(const MttkrpArgs &a, int64_t tile, char *lds) {
    constexpr int PER = T / NT;
    constexpr int NO = NMAX - 1;
    static_assert(PER * NT == T && NMAX <= 4, "row cache: 4 modes at most");
    const int nm = NFIX ? NFIX : a.nmodes, mode = a.mode, tid = threadIdx.x, no = nm - 1;
    const int R = a.rank, cap = a.d_cap;
    uint32_t *crdg = (uint32_t *)lds;
    float *valg = (float *)(crdg + (size_t)no * T);
    float *cache = valg + T;
    const int64_t k0 = a.pl_off[tile], k1 = min(a.pl_off[tile + 1], k0 + T);
    const int64_t base = tile * (int64_t)T;
    const int64_t rem = a.nnz - base;
    const int cnt = rem < T ? (int)rem : T;
    // every thread stages PER consecutive nonzeros: one 16-byte load of
    // values and one 8-byte load per u16 stream (tiles start at multiples of
    // T, so the vectors are aligned); the last tile's ragged end goes element
    // by element
    static_assert(PER == 4, "row-cached staging loads 4 nonzeros per thread");
    const int e0 = tid * PER;
    float v[PER];
    uint32_t q[PER];
    uint32_t sl[NO][PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        v[u] = 0.f;
        q[u] = 0;
#pragma unroll
        for (int o = 0; o < NO; ++o) sl[o][u] = 0;
    }
    if (e0 + PER <= cnt) {
        const spt_f4 x = __builtin_nontemporal_load(reinterpret_cast<const spt_f4 *>(a.vals + base + e0));
        const spt_u2 w = __builtin_nontemporal_load(reinterpret_cast<const spt_u2 *>(a.pl_pos + base + e0));
        v[0] = x.x;
        v[1] = x.y;
        v[2] = x.z;
        v[3] = x.w;
        q[0] = w.x & 0xFFFFu;
        q[1] = w.x >> 16;
        q[2] = w.y & 0xFFFFu;
        q[3] = w.y >> 16;
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            if (o < no) {
                const spt_u2 d = __builtin_nontemporal_load(reinterpret_cast<const spt_u2 *>(a.d_slot[o] + base + e0));
                sl[o][0] = d.x & 0xFFFFu;
                sl[o][1] = d.x >> 16;
                sl[o][2] = d.y & 0xFFFFu;
                sl[o][3] = d.y >> 16;
            }
        }
    } else {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = e0 + u;
            if (e < cnt) {
                v[u] = a.vals[base + e];
                q[u] = a.pl_pos[base + e];
#pragma unroll
                for (int o = 0; o < NO; ++o)
                    if (o < no) sl[o][u] = a.d_slot[o][base + e];
            }
        }
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) q[u] &= (uint32_t)(T - 1);  // a position inside the tile
    // copy the cached rows: the first min(distinct, cap) of each dictionary
    int64_t dbase[NO];
    int dn[NO], dlast[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        dbase[o] = 0;
        dn[o] = 0;
        dlast[o] = 0;
        if (o < no) {
            dbase[o] = a.d_off[o][tile];
            const int64_t d = a.d_off[o][tile + 1] - dbase[o];  // distinct rows of the tile
            dn[o] = (int)min<int64_t>(d, (int64_t)cap);
            dlast[o] = (int)max<int64_t>(d - 1, 0);
        }
    }
    if ((R & 3) == 0) {
        const int r4 = R >> 2;
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            if (o < no) {
                const float *f = a.f[o + (o >= mode)];
                const uint32_t *dr = a.d_row[o] + dbase[o];
                float *cb = cache + (size_t)o * cap * R;
                for (int i = tid; i < dn[o] * r4; i += NT) {
                    const int sidx = i / r4, c = i - sidx * r4;
                    const float4 x = *reinterpret_cast<const float4 *>(f + (size_t)dr[sidx] * R + 4 * c);
                    *reinterpret_cast<float4 *>(cb + (size_t)sidx * R + 4 * c) = x;
                }
            }
        }
    } else {
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            if (o < no) {
                const float *f = a.f[o + (o >= mode)];
                const uint32_t *dr = a.d_row[o] + dbase[o];
                float *cb = cache + (size_t)o * cap * R;
                for (int i = tid; i < dn[o] * R; i += NT) {
                    const int sidx = i / R, c = i - sidx * R;
                    cb[(size_t)sidx * R + c] = f[(size_t)dr[sidx] * R + c];
                }
            }
        }
    }
    // scatter: cached rows by their byte offset in LDS, the others by global
    // row with kDictMiss set.  The global rows of all PER nonzeros are loaded
    // before the first LDS store, so the thread waits for them once.
    const uint32_t cache_off = (uint32_t)(reinterpret_cast<const char *>(cache) - lds);
    uint32_t grow[NO][PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            grow[o][u] = 0;
            if (o < no && e0 + u < cnt) grow[o][u] = a.d_row[o][dbase[o] + min(sl[o][u], (uint32_t)dlast[o])];
        }
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        if (e0 + u < cnt) {
            valg[q[u]] = v[u];
#pragma unroll
            for (int o = 0; o < NO; ++o) {
                if (o < no) {
                    const uint32_t si = min(sl[o][u], (uint32_t)dlast[o]);
                    crdg[o * T + q[u]] = (int)si < dn[o] ? cache_off + ((uint32_t)(o * cap) + si) * (uint32_t)(R * 4)
                                                         : (grow[o][u] | kDictMiss);
                }
            }
        }
    }
    __syncthreads();
    // the largest entry a cached row can have: the last slot of the last mode
    const uint32_t lim = cache_off + ((uint32_t)(no * cap) - 1u) * (uint32_t)(R * 4);
    seg_walk<NT, T, G, VEC, NB, NMAX, NFIX, EXACT, PackedPieces<T>, true>(
        a, crdg, valg, (int)(k1 - k0), PackedPieces<T>{reinterpret_cast<const spt_u4 *>(a.pl_piece), k0, a.rec_cap},
        a.rec_row, a.rec_val, a.rank, 0, lds, lim);
}

template <int NT, int T, int G, int VEC, int NB, int NMAX, int NFIX, bool EXACT>
__global__ __launch_bounds__(NT) void k_mttkrp_segd(MttkrpArgs a, int64_t ntiles) {
    extern __shared__ __align__(16) char lds[];
    const int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    segd_tile<NT, T, G, VEC, NB, NMAX, NFIX, EXACT>(a, tile, lds);
}

// Batched: tile `it` of the whole batch belongs to the last item whose
// first_tile <= it.
__device__ __forceinline__ int seg_item_of(const SegItem *__restrict__ items, int count, int64_t it) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].first_tile <= it) lo = mid;
        else hi = mid - 1;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

// Every tensor's records start at its rec_base in the batch's record array,
// its rows at row_base of the concatenated output (records of the whole batch
// stay grouped by row: tensors are laid out in order).
// Persistent: a grid sized to the resident workgroups pulls the batch's tiles
// (T = 4 NT nonzeros each, over all tensors in order) from the counter
// *next_tile, zero at launch, until the counter passes total_tiles.  A
// workgroup's tiles only increase, so it finds each tile's tensor by moving
// forward from the last one.
template <int NT, int G, int VEC, int NB, int NMAX, int NFIX>
__global__ __launch_bounds__(NT) void k_mttkrp_segp_batched(const SegItem *__restrict__ items, int count,
                                                            int64_t total_tiles, uint64_t *__restrict__ rec_row,
                                                            float *__restrict__ rec_val, int ld,
                                                            unsigned long long *__restrict__ next_tile) {
    extern __shared__ __align__(16) char lds[];
    __shared__ int64_t s_tile;
    int b = 0;
    for (;;) {
        if (threadIdx.x == 0) s_tile = (int64_t)atomicAdd(next_tile, 1ull);
        __syncthreads();  // also: every wave is done with the previous tile's LDS
        const int64_t it = s_tile;
        __syncthreads();  // every thread has read s_tile before it is replaced
        if (it >= total_tiles) break;
        while (b + 1 < count && items[b + 1].first_tile <= it) ++b;
        const SegItem &item = items[b];
        segp_tile<NT, 4 * NT, G, VEC, NB, NMAX, NFIX, false, false>(item.a, it - item.first_tile, lds, rec_row, rec_val,
                                                                    ld, item.rec_base, item.row_base);
    }
}

// The plan of one mode: positions of every nonzero, and per piece its
// (start | length << 16), row, and (for the record layout) its pair and index
// within the pair; per distinct (tile, row) pair its row (sort key) and pieces.
// Emission of one tile: positions to pos (the tensor's), piece start/length
// and row to desc/prow at a.pl_off[tile]; piece pair and index to
// ppair/psub at gpiece; pair (row_base + row, pieces) to pair_key/pair_np at
// gpair (pair indices are global, gpair-based).
template <int NT, int NMAX>
__device__ __forceinline__ void emit_tile(const MttkrpArgs &a, int64_t tile, char *lds, uint32_t *wsum,
                                          uint16_t *__restrict__ pos, uint32_t *__restrict__ desc,
                                          uint32_t *__restrict__ prow, int64_t gpiece, int64_t gpair, int64_t row_base,
                                          uint32_t *__restrict__ ppair, uint32_t *__restrict__ psub,
                                          uint64_t *__restrict__ pair_key, uint32_t *__restrict__ pair_np) {
    constexpr int T = 4 * NT;
    const SegLds L = seg_carve_plan(lds, T);
    const CodecRegs cr = load_codec_regs(a.codec);
    seg_stage<NT, NMAX, false>(a, tile, L, cr, wsum, pos);
    // pair index of every occupied slot: exclusive count of occupied slots before it
    uint32_t *occ = (uint32_t *)L.valg;  // free in counting mode; T entries
    for (int i = threadIdx.x; i < T; i += NT) {
        const uint32_t nx = i + 1 < T ? L.hcnt[i + 1] : L.hcnt[T];
        occ[i] = (nx >> 16) != (L.hcnt[i] >> 16) ? 1u : 0u;
    }
    __syncthreads();
    block_scan_lds(occ, T, NT, wsum);
    const int64_t pbase = a.pl_off[tile], qbase = gpair;
    for (int i = threadIdx.x; i < T; i += NT) {
        const uint32_t pk = L.hcnt[i];
        const uint32_t nx = i + 1 < T ? L.hcnt[i + 1] : L.hcnt[T];
        const uint32_t c = (nx >> 16) - (pk >> 16);
        if (c > 0) {
            pair_key[qbase + occ[i]] = (uint64_t)(row_base + L.hkey[i]);
            pair_np[qbase + occ[i]] = (c + kPiece - 1) / kPiece;
        }
    }
    // the tile's pieces are stored longest first (a counting sort on the
    // length): dealt to lane groups in snake order they balance the walk
    __shared__ uint32_t lstart[kPiece + 1];
    const int npieces = (int)(L.hcnt[T] & 0xFFFFu);
    auto piece = [&](int k, int &s, int &i, int &p0, int &p1) {
        s = L.ptab[k];
        const uint32_t pk = L.hcnt[s];
        const uint32_t pn = (s + 1 < T) ? L.hcnt[s + 1] : L.hcnt[T];
        const int first = (int)(pk >> 16), last = (int)(pn >> 16);
        i = k - (int)(pk & 0xFFFFu);
        p0 = first + i * kPiece;
        p1 = min(p0 + kPiece, last);
    };
    for (int b = threadIdx.x; b <= kPiece; b += NT) lstart[b] = 0;
    __syncthreads();
    for (int k = threadIdx.x; k < npieces; k += NT) {
        int sl, i, p0, p1;
        piece(k, sl, i, p0, p1);
        atomicAdd(&lstart[kPiece - (p1 - p0)], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int b = 0; b <= kPiece; ++b) {
            const uint32_t c = lstart[b];
            lstart[b] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < npieces; k += NT) {
        int sl, i, p0, p1;
        piece(k, sl, i, p0, p1);
        const uint32_t q = atomicAdd(&lstart[kPiece - (p1 - p0)], 1u);
        desc[pbase + q] = (uint32_t)p0 | ((uint32_t)(p1 - p0) << 16);
        prow[pbase + q] = L.hkey[sl];
        ppair[gpiece + q] = (uint32_t)(qbase + occ[sl]);
        psub[gpiece + q] = (uint32_t)i;
    }
}

template <int NT, int NMAX>
__global__ __launch_bounds__(NT) void k_emit_plan(MttkrpArgs a, int64_t ntiles, const int64_t *__restrict__ pair_off,
                                                  uint16_t *__restrict__ pos, uint32_t *__restrict__ desc,
                                                  uint32_t *__restrict__ prow, uint32_t *__restrict__ ppair,
                                                  uint32_t *__restrict__ psub, uint64_t *__restrict__ pair_key,
                                                  uint32_t *__restrict__ pair_np) {
    extern __shared__ __align__(16) char lds[];
    __shared__ uint32_t wsum[NT / 64];
    const int64_t tile = blockIdx.x;
    emit_tile<NT, NMAX>(a, tile, lds, wsum, pos, desc, prow, a.pl_off[tile], pair_off[tile], 0, ppair, psub, pair_key,
                        pair_np);
}

// Batched emission: item b's plan arrays come in its args (pl_pos, pl_desc,
// pl_row, pl_off); gpiece_off / gpair_off give each global tile's first
// piece and pair in the batch-wide arrays; pair keys are rows of the
// concatenated output (row_base + row).
template <int NT, int NMAX>
__global__ __launch_bounds__(NT) void k_emit_plan_batched(const SegItem *__restrict__ items, int count,
                                                          const int64_t *__restrict__ gpiece_off,
                                                          const int64_t *__restrict__ gpair_off,
                                                          uint32_t *__restrict__ ppair, uint32_t *__restrict__ psub,
                                                          uint64_t *__restrict__ pair_key,
                                                          uint32_t *__restrict__ pair_np) {
    extern __shared__ __align__(16) char lds[];
    __shared__ uint32_t wsum[NT / 64];
    const int64_t it = blockIdx.x;
    const int b = seg_item_of(items, count, it);
    const SegItem &item = items[b];
    const MttkrpArgs &a = item.a;
    emit_tile<NT, NMAX>(a, it - item.first_tile, lds, wsum, const_cast<uint16_t *>(a.pl_pos),
                        const_cast<uint32_t *>(a.pl_desc), const_cast<uint32_t *>(a.pl_row), gpiece_off[it],
                        gpair_off[it], item.row_base, ppair, psub, pair_key, pair_np);
}

// Batched piece records: global piece g of item b (pieces from
// items[b].rec_base) gets its first pair record plus its index, made local
// to the item (the item's records start at its rec_base).
__global__ __launch_bounds__(256) void k_piece_dest_batched(const SegItem *__restrict__ items, int count,
                                                            const int64_t *__restrict__ piece_base,
                                                            const uint32_t *__restrict__ ppair,
                                                            const uint32_t *__restrict__ psub,
                                                            const uint32_t *__restrict__ pair_first, int64_t n) {
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < n; g += (int64_t)gridDim.x * 256) {
        int lo = 0, hi = count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (piece_base[mid] <= g) lo = mid;
            else hi = mid - 1;
        }
        const uint32_t d = pair_first[ppair[g]] + psub[g];
        const_cast<uint32_t *>(items[lo].a.pl_dest)[g - piece_base[lo]] = d - (uint32_t)piece_base[lo];
    }
}

// packed[k] = {desc[k], prow[k], first record of piece k's pair + its index within the pair, 0}
__global__ __launch_bounds__(256) void k_piece_pack(const uint32_t *__restrict__ ppair, const uint32_t *__restrict__ psub,
                                                    const uint32_t *__restrict__ pair_first,
                                                    const uint32_t *__restrict__ desc, const uint32_t *__restrict__ prow,
                                                    spt_u4 *__restrict__ packed, int64_t n) {
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) {
        spt_u4 q;
        q.x = desc[k];
        q.y = prow[k];
        q.z = pair_first[ppair[k]] + psub[k];
        q.w = 0u;
        packed[k] = q;
    }
}

// pieces | distinct rows << 32 of a tile after the hashing stage
template <int T>
__device__ __forceinline__ int64_t tile_counts(const SegLds &L) {
    __shared__ uint32_t s_distinct;
    if (threadIdx.x == 0) s_distinct = 0;
    __syncthreads();
    uint32_t d = 0;
    for (int i = threadIdx.x; i < T; i += blockDim.x) {
        const uint32_t nx = i + 1 < T ? L.hcnt[i + 1] : L.hcnt[T];
        d += (nx >> 16) != (L.hcnt[i] >> 16);
    }
    atomicAdd(&s_distinct, d);
    __syncthreads();
    return (int64_t)(L.hcnt[T] & 0xFFFFu) | ((int64_t)s_distinct << 32);
}

// Pieces and distinct rows of every tile (the plan's counting pass).
template <int NT, int NMAX>
__global__ __launch_bounds__(NT) void k_count_pieces(MttkrpArgs a, int64_t ntiles, int64_t *__restrict__ out) {
    constexpr int T = 4 * NT;
    extern __shared__ __align__(16) char lds[];
    __shared__ uint32_t wsum[NT / 64];
    const int64_t tile = blockIdx.x;
    const SegLds L = seg_carve_plan(lds, T);
    const CodecRegs cr = load_codec_regs(a.codec);
    seg_stage<NT, NMAX, false>(a, tile, L, cr, wsum);
    const int64_t c = tile_counts<T>(L);
    if (threadIdx.x == 0) out[tile] = c;
}

template <int NT, int NMAX>
__global__ __launch_bounds__(NT) void k_count_pieces_batched(const SegItem *__restrict__ items, int count,
                                                             int64_t total_tiles, int64_t *__restrict__ out) {
    constexpr int T = 4 * NT;
    extern __shared__ __align__(16) char lds[];
    __shared__ uint32_t wsum[NT / 64];
    const int64_t it = blockIdx.x;
    const int b = seg_item_of(items, count, it);
    const MttkrpArgs &a = items[b].a;
    const SegLds L = seg_carve_plan(lds, T);
    const CodecRegs cr = load_codec_regs(a.codec);
    seg_stage<NT, NMAX, false>(a, it - items[b].first_tile, L, cr, wsum);
    const int64_t c = tile_counts<T>(L);
    if (threadIdx.x == 0) out[it] = c;
}

template <int NT, int T, int NMAX, int NFIX, int G, int VEC, int NB>
spt_status launch_seg_k(const MttkrpArgs &a, int64_t ntiles, hipStream_t s) {
    if constexpr (T == kDictTile && NMAX <= 4) {
        if (a.d_cap > 0) {
            const size_t lds = segd_lds_bytes(T, a.nmodes, a.d_cap, a.rank);
            if (a.rank == G * VEC * NB)
                hipLaunchKernelGGL((k_mttkrp_segd<NT, T, G, VEC, NB, NMAX, NFIX, true>), dim3((unsigned)ntiles),
                                   dim3(NT), lds, s, a, ntiles);
            else
                hipLaunchKernelGGL((k_mttkrp_segd<NT, T, G, VEC, NB, NMAX, NFIX, false>), dim3((unsigned)ntiles),
                                   dim3(NT), lds, s, a, ntiles);
            SPT_HIP(hipGetLastError());
            return SPT_OK;
        }
    }
    const size_t lds = segp_lds_bytes(T, a.nmodes);
    if (a.rank == G * VEC * NB)
        hipLaunchKernelGGL((k_mttkrp_segp<NT, T, G, VEC, NB, NMAX, NFIX, true>), dim3((unsigned)ntiles), dim3(NT), lds, s,
                           a, ntiles);
    else
        hipLaunchKernelGGL((k_mttkrp_segp<NT, T, G, VEC, NB, NMAX, NFIX, false>), dim3((unsigned)ntiles), dim3(NT), lds,
                           s, a, ntiles);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

template <int NT, int T, int NMAX, int NFIX>
spt_status launch_seg_nt(const MttkrpArgs &a, int64_t ntiles, hipStream_t s) {
    const int R = a.rank;
    if ((R & 3) == 0) {
        const int r4 = R >> 2;
        if (r4 <= 1) return launch_seg_k<NT, T, NMAX, NFIX, 1, 4, 1>(a, ntiles, s);
        if (r4 <= 2) return launch_seg_k<NT, T, NMAX, NFIX, 2, 4, 1>(a, ntiles, s);
        if (r4 <= 4) return launch_seg_k<NT, T, NMAX, NFIX, 4, 4, 1>(a, ntiles, s);
        if (r4 <= 8) return launch_seg_k<NT, T, NMAX, NFIX, 8, 4, 1>(a, ntiles, s);
        if (r4 <= 16) return launch_seg_k<NT, T, NMAX, NFIX, 16, 4, 1>(a, ntiles, s);
        if (r4 <= 32) return launch_seg_k<NT, T, NMAX, NFIX, 32, 4, 1>(a, ntiles, s);
        return launch_seg_k<NT, T, NMAX, NFIX, 64, 4, 1>(a, ntiles, s);
    }
    if (R <= 64) return launch_seg_k<NT, T, NMAX, NFIX, 64, 1, 1>(a, ntiles, s);
    if (R <= 128) return launch_seg_k<NT, T, NMAX, NFIX, 64, 1, 2>(a, ntiles, s);
    if (R <= 192) return launch_seg_k<NT, T, NMAX, NFIX, 64, 1, 3>(a, ntiles, s);
    return launch_seg_k<NT, T, NMAX, NFIX, 64, 1, 4>(a, ntiles, s);
}

template <int NT>
spt_status launch_emit_nt(const MttkrpArgs &a, int64_t ntiles, const PlanOut &o, hipStream_t s) {
    const size_t lds = seg_plan_lds_bytes(4 * NT);
    if (a.nmodes <= 4)
        hipLaunchKernelGGL((k_emit_plan<NT, 4>), dim3((unsigned)ntiles), dim3(NT), lds, s, a, ntiles, o.pair_off, o.pos,
                           o.desc, o.prow, o.ppair, o.psub, o.pair_key, o.pair_np);
    else
        hipLaunchKernelGGL((k_emit_plan<NT, 8>), dim3((unsigned)ntiles), dim3(NT), lds, s, a, ntiles, o.pair_off, o.pos,
                           o.desc, o.prow, o.ppair, o.psub, o.pair_key, o.pair_np);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

template <int NT>
spt_status launch_count_nt(const MttkrpArgs &a, int64_t ntiles, int64_t *out, hipStream_t s) {
    const size_t lds = seg_plan_lds_bytes(4 * NT);
    if (a.nmodes <= 4)
        hipLaunchKernelGGL((k_count_pieces<NT, 4>), dim3((unsigned)ntiles), dim3(NT), lds, s, a, ntiles, out);
    else
        hipLaunchKernelGGL((k_count_pieces<NT, 8>), dim3((unsigned)ntiles), dim3(NT), lds, s, a, ntiles, out);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

}  // namespace

// tile sizes served: 1024 (256 threads), 2048 (512), 4096 (1024 threads)
bool seg_tile_ok(int tile, int nmodes) {
    if (tile != 1024 && tile != 2048 && tile != 4096) return false;
    return seg_lds_bytes(tile, nmodes) <= 160 * 1024 - 1024 && segp_lds_bytes(tile, nmodes) <= 160 * 1024 - 1024;
}

spt_status launch_emit_plan(const MttkrpArgs &a, const PlanOut &o, hipStream_t s) {
    const int64_t ntiles = (a.nnz + a.tile - 1) / a.tile;
    if (ntiles == 0) return SPT_OK;
    if (!seg_tile_ok(a.tile, a.nmodes)) return fail(SPT_E_INVALID_ARG, "segment: tile does not fit LDS");
    if (a.tile == 1024) return launch_emit_nt<256>(a, ntiles, o, s);
    if (a.tile == 2048) return launch_emit_nt<512>(a, ntiles, o, s);
    return launch_emit_nt<1024>(a, ntiles, o, s);
}

spt_status launch_piece_pack(const uint32_t *ppair, const uint32_t *psub, const uint32_t *pair_first,
                             const uint32_t *desc, const uint32_t *prow, uint32_t *packed, int64_t n, hipStream_t s) {
    if (n == 0) return SPT_OK;
    const int64_t g = std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_piece_pack, dim3((unsigned)g), dim3(256), 0, s, ppair, psub, pair_first, desc, prow,
                       reinterpret_cast<spt_u4 *>(packed), n);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

spt_status launch_count_pieces(const MttkrpArgs &a, int64_t *counts, hipStream_t s) {
    const int64_t ntiles = (a.nnz + a.tile - 1) / a.tile;
    if (ntiles == 0) return SPT_OK;
    if (!seg_tile_ok(a.tile, a.nmodes)) return fail(SPT_E_INVALID_ARG, "segment: tile does not fit LDS");
    if (a.tile == 1024) return launch_count_nt<256>(a, ntiles, counts, s);
    if (a.tile == 2048) return launch_count_nt<512>(a, ntiles, counts, s);
    return launch_count_nt<1024>(a, ntiles, counts, s);
}

namespace {
// 3 and 4 modes get a kernel with the mode count fixed; others the general one
template <int NT, int T>
spt_status launch_seg_tile(const MttkrpArgs &a, int64_t ntiles, hipStream_t s) {
    const int nm = a.nmodes;
    if (nm == 3) return launch_seg_nt<NT, T, 3, 3>(a, ntiles, s);
    if (nm == 4) return launch_seg_nt<NT, T, 4, 4>(a, ntiles, s);
    return nm < 3 ? launch_seg_nt<NT, T, 3, 0>(a, ntiles, s) : launch_seg_nt<NT, T, 8, 0>(a, ntiles, s);
}
}  // namespace

spt_status launch_emit_dict(const MttkrpArgs &a, const int64_t *off, uint32_t *rows, uint16_t *slots, hipStream_t s) {
    const int64_t ntiles = (a.nnz + kDictTile - 1) / kDictTile;
    if (ntiles == 0) return SPT_OK;
    constexpr int NT = kDictTile / 4;
    const size_t lds = (size_t)kDictTile * 8;
    hipLaunchKernelGGL((k_emit_dict<NT, 8>), dim3((unsigned)ntiles), dim3(NT), lds, s, a, off, rows, slots);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

int dict_cap(int nmodes, int rank) {
    if (nmodes < 2 || nmodes > 4) return 0;
    const size_t fixed = segp_lds_bytes(kDictTile, nmodes);
    if (fixed >= kDictLdsBudget) return 0;
    const size_t cap = (kDictLdsBudget - fixed) / ((size_t)(nmodes - 1) * rank * 4);
    return cap >= (size_t)kDictMinCap ? (int)std::min<size_t>(cap, kDictTile) : 0;
}

spt_status launch_mttkrp_seg(const MttkrpArgs &a, hipStream_t s) {
    const int64_t ntiles = (a.nnz + a.tile - 1) / a.tile;
    if (ntiles == 0) return SPT_OK;
    if (!seg_tile_ok(a.tile, a.nmodes)) return fail(SPT_E_INVALID_ARG, "segment: tile does not fit LDS");
    if (!a.pl_pos || !a.pl_off || !a.pl_piece) return fail(SPT_E_INVALID_ARG, "segment: no plan");
    if (a.tile == 1024) return launch_seg_tile<256, 1024>(a, ntiles, s);
    if (a.tile == 2048) return launch_seg_tile<512, 2048>(a, ntiles, s);
    return launch_seg_tile<kSegpThreads4096, 4096>(a, ntiles, s);
}

namespace {
template <int NT, int NMAX, int NFIX, int G, int VEC, int NB>
spt_status launch_segb_k(const SegItem *items, int count, int64_t total_tiles, uint64_t *rec_row, float *rec_val,
                         int ld, unsigned long long *next_tile, hipStream_t s) {
    const size_t lds = segp_lds_bytes(4 * NT, NMAX);
    static std::atomic<int> per_cu{0};  // resident workgroups per CU (fixed per instantiation: its LDS is)
    int pc = per_cu.load(std::memory_order_relaxed);
    if (pc == 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &pc, reinterpret_cast<const void *>(&k_mttkrp_segp_batched<NT, G, VEC, NB, NMAX, NFIX>), NT, lds) !=
                hipSuccess ||
            pc < 1) {
            (void)hipGetLastError();  // not a failure of this call: one resident workgroup per CU is assumed
            pc = 1;
        }
        per_cu.store(pc, std::memory_order_relaxed);
    }
    const int64_t grid = std::min<int64_t>(total_tiles, (int64_t)pc * device_cus());
    spt_status st = launch_fill_zero(reinterpret_cast<float *>(next_tile), 2, s);  // the tile counter
    if (st != SPT_OK) return st;
    hipLaunchKernelGGL((k_mttkrp_segp_batched<NT, G, VEC, NB, NMAX, NFIX>), dim3((unsigned)grid), dim3(NT), lds, s, items,
                       count, total_tiles, rec_row, rec_val, ld, next_tile);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

template <int NT, int NMAX, int NFIX>
spt_status launch_segb_n(const SegItem *items, int count, int64_t total_tiles, uint64_t *rec_row, float *rec_val,
                         int ld, bool vec4, unsigned long long *next_tile, hipStream_t s) {
    if (vec4) {
        const int r4 = ld >> 2;
        if (r4 <= 1) return launch_segb_k<NT, NMAX, NFIX, 1, 4, 1>(items, count, total_tiles, rec_row, rec_val, ld, next_tile, s);
        if (r4 <= 2) return launch_segb_k<NT, NMAX, NFIX, 2, 4, 1>(items, count, total_tiles, rec_row, rec_val, ld, next_tile, s);
        if (r4 <= 4) return launch_segb_k<NT, NMAX, NFIX, 4, 4, 1>(items, count, total_tiles, rec_row, rec_val, ld, next_tile, s);
        if (r4 <= 8) return launch_segb_k<NT, NMAX, NFIX, 8, 4, 1>(items, count, total_tiles, rec_row, rec_val, ld, next_tile, s);
        return launch_segb_k<NT, NMAX, NFIX, 16, 4, 1>(items, count, total_tiles, rec_row, rec_val, ld, next_tile, s);
    }
    return launch_segb_k<NT, NMAX, NFIX, 64, 1, 1>(items, count, total_tiles, rec_row, rec_val, ld, next_tile, s);
}

template <int NT>
spt_status launch_segb_t(const SegItem *items, int count, int64_t total_tiles, int nmodes_min, int nmodes_max, int ld,
                         bool vec4, uint64_t *rec_row, float *rec_val, unsigned long long *next_tile, hipStream_t s) {
    if (nmodes_min == 3 && nmodes_max == 3)
        return launch_segb_n<NT, 3, 3>(items, count, total_tiles, rec_row, rec_val, ld, vec4, next_tile, s);
    if (nmodes_max <= 4) return launch_segb_n<NT, 4, 0>(items, count, total_tiles, rec_row, rec_val, ld, vec4, next_tile, s);
    return launch_segb_n<NT, 8, 0>(items, count, total_tiles, rec_row, rec_val, ld, vec4, next_tile, s);
}

template <int NT>
void launch_emit_b(const SegItem *items, int count, int64_t total_tiles, int nmodes_max, const int64_t *gpiece_off,
                   const int64_t *gpair_off, uint32_t *ppair, uint32_t *psub, uint64_t *pair_key, uint32_t *pair_np,
                   hipStream_t s) {
    constexpr int T = 4 * NT;
    if (nmodes_max <= 4)
        hipLaunchKernelGGL((k_emit_plan_batched<NT, 4>), dim3((unsigned)total_tiles), dim3(NT), seg_plan_lds_bytes(T), s,
                           items, count, gpiece_off, gpair_off, ppair, psub, pair_key, pair_np);
    else
        hipLaunchKernelGGL((k_emit_plan_batched<NT, 8>), dim3((unsigned)total_tiles), dim3(NT),
                           seg_plan_lds_bytes(T), s,
                           items, count, gpiece_off, gpair_off, ppair, psub, pair_key, pair_np);
}

template <int NT>
void launch_count_b(const SegItem *items, int count, int64_t total_tiles, int nmodes_max, int64_t *counts,
                    hipStream_t s) {
    constexpr int T = 4 * NT;
    if (nmodes_max <= 4)
        hipLaunchKernelGGL((k_count_pieces_batched<NT, 4>), dim3((unsigned)total_tiles), dim3(NT), seg_plan_lds_bytes(T), s,
                           items, count, total_tiles, counts);
    else
        hipLaunchKernelGGL((k_count_pieces_batched<NT, 8>), dim3((unsigned)total_tiles), dim3(NT),
                           seg_plan_lds_bytes(T), s,
                           items, count, total_tiles, counts);
}
}  // namespace

bool seg_batch_fits(int nmodes_max, int tile) { return seg_tile_ok(tile, nmodes_max); }

spt_status launch_emit_plan_batched(const SegItem *items, int count, int64_t total_tiles, int nmodes_max, int tile,
                                    const int64_t *gpiece_off, const int64_t *gpair_off, uint32_t *ppair,
                                    uint32_t *psub, uint64_t *pair_key, uint32_t *pair_np, hipStream_t s) {
    if (total_tiles == 0) return SPT_OK;
    if (!seg_batch_fits(nmodes_max, tile)) return fail(SPT_E_INVALID_ARG, "batch plan: tile does not fit LDS");
    if (tile == 1024) launch_emit_b<256>(items, count, total_tiles, nmodes_max, gpiece_off, gpair_off, ppair, psub, pair_key, pair_np, s);
    else if (tile == 2048) launch_emit_b<512>(items, count, total_tiles, nmodes_max, gpiece_off, gpair_off, ppair, psub, pair_key, pair_np, s);
    else launch_emit_b<1024>(items, count, total_tiles, nmodes_max, gpiece_off, gpair_off, ppair, psub, pair_key, pair_np, s);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

spt_status launch_piece_dest_batched(const SegItem *items, int count, const int64_t *piece_base, const uint32_t *ppair,
                                     const uint32_t *psub, const uint32_t *pair_first, int64_t n, hipStream_t s) {
    if (n == 0) return SPT_OK;
    const int64_t g = std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_piece_dest_batched, dim3((unsigned)g), dim3(256), 0, s, items, count, piece_base, ppair, psub,
                       pair_first, n);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

spt_status launch_count_pieces_batched(const SegItem *items, int count, int64_t total_tiles, int nmodes_max, int tile,
                                       int64_t *counts, hipStream_t s) {
    if (total_tiles == 0) return SPT_OK;
    if (!seg_batch_fits(nmodes_max, tile)) return fail(SPT_E_INVALID_ARG, "batch plan: tile does not fit LDS");
    if (tile == 1024) launch_count_b<256>(items, count, total_tiles, nmodes_max, counts, s);
    else if (tile == 2048) launch_count_b<512>(items, count, total_tiles, nmodes_max, counts, s);
    else launch_count_b<1024>(items, count, total_tiles, nmodes_max, counts, s);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

spt_status launch_mttkrp_seg_batched(const SegItem *items, int count, int64_t total_tiles, int nmodes_min,
                                     int nmodes_max, int tile, int ld, bool vec4, uint64_t *rec_row, float *rec_val,
                                     unsigned long long *next_tile, hipStream_t s) {
    if (total_tiles == 0) return SPT_OK;
    if (ld > 64 || (vec4 && (ld & 3))) return fail(SPT_E_INVALID_ARG, "batched MTTKRP: rank above 64");
    if (!seg_batch_fits(nmodes_max, tile)) return fail(SPT_E_INVALID_ARG, "batched MTTKRP: tile does not fit LDS");
    if (!next_tile) return fail(SPT_E_INVALID_ARG, "batched MTTKRP: no tile counter");
    if (tile == 1024)
        return launch_segb_t<256>(items, count, total_tiles, nmodes_min, nmodes_max, ld, vec4, rec_row, rec_val, next_tile, s);
    if (tile == 2048)
        return launch_segb_t<512>(items, count, total_tiles, nmodes_min, nmodes_max, ld, vec4, rec_row, rec_val, next_tile, s);
    return launch_segb_t<1024>(items, count, total_tiles, nmodes_min, nmodes_max, ld, vec4, rec_row, rec_val, next_tile, s);
}

}  // namespace spt
