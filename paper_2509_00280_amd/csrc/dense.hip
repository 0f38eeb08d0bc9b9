// Dense FP64 steps of CP-ALS on gfx950 (the ALS update that Section II-B
// defers to Kolda and Bader):
//   gram        G = C^T C for an I x R FP32 matrix: FP32 values widened to FP64
//               (products exact) and accumulated by v_mfma_f64_16x16x4_f64;
//               only the upper block triangle is computed and mirrored.
//   solve_prep  one workgroup: V = Hadamard product of the other Grams,
//               Cholesky V = L L^T with a ridge retry, W = V^-1, column norms of
//               M W from the quadratic form lambda_r^2 = (W (M^T M) W)_rr,
//               S = W diag(1/lambda).
//   apply       C = fp32(M S) row block by row block (FP64 FMAs), with the
//               fit's inner product sum M .* C * lambda fused in.
//   fit         |Xhat|^2 = lambda^T (Hadamard of all Grams) lambda and the fit.
#include <algorithm>

#include "spt_internal.h"

namespace spt {

namespace {

constexpr int kThreads = 256;
constexpr int kGramSliceRows1 = 512;   // rows of a Gram slice (one workgroup, 8 waves)
constexpr int kGramSThreads = 512;

typedef double double4_t __attribute__((ext_vector_type(4)));

int gram_nb(int R) { return (R + 15) / 16; }
// row slices (workgroups, one partial each) of the Gram kernel
int gram_chunks(int64_t rows, int R) {
    const int ld = gram_nb(R) * 16;
    int64_t slices = (rows + kGramSliceRows1 - 1) / kGramSliceRows1;
    const int64_t cap = std::max<int64_t>(4, (int64_t)(32u << 20) / ((int64_t)ld * ld * 8));  // ~32 MB of partials
    slices = std::min<int64_t>(slices, cap);
    return (int)std::max<int64_t>(1, slices);
}

// Partial Grams of row slices, one slice per workgroup of 8 waves (so
// enough waves keep the row loads in flight while the number of partials
// stays bounded).  Wave w takes the slice's row groups of 4 rows
// w UNR + 8 UNR j, ..., accumulates every 16x16 block tile (pb <= qb) of R
// with FP64 MFMA into independent accumulators, and the waves add their
// tiles in LDS in wave order (deterministic).  Lane layout of
// v_mfma_f64_16x16x4_f64: A[m][k] from lane m + 16k, B[k][n] from lane
// n + 16k, D[m][n] in lane n + 16*(m%4), element m/4.
template <int NB, int UNR>
__global__ __launch_bounds__(kGramSThreads) void k_gram_partial(const float *__restrict__ C, int64_t rows, int R,
                                                                double *__restrict__ work) {
    constexpr int NT = NB * (NB + 1) / 2, LDP = NB * 16, NWAVE = kGramSThreads / 64;
    __shared__ double red[LDP * LDP];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t slice = blockIdx.x;
    const int64_t nslices = gridDim.x;
    const int64_t r_per = ((rows + nslices - 1) / nslices + 3) / 4 * 4;
    const int64_t r0 = slice * r_per;
    const int64_t r1 = min(r0 + r_per, rows);
    const int kr = lane >> 4, cc = lane & 15;
    double4_t acc[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) acc[i] = (double4_t){0.0, 0.0, 0.0, 0.0};
    for (int64_t g0 = r0 / 4 + (int64_t)wave * UNR; g0 * 4 < r1; g0 += (int64_t)NWAVE * UNR) {
        double v[UNR][NB];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int64_t row = (g0 + u) * 4 + kr;
            const bool rok = row < r1;
            const float *rp = C + row * R;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int c = b * 16 + cc;
                v[u][b] = (rok && c < R) ? (double)rp[c] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            int t = 0;
#pragma unroll
            for (int pb = 0; pb < NB; ++pb)
#pragma unroll
                for (int qb = pb; qb < NB; ++qb, ++t)
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[u][pb], v[u][qb], acc[t], 0, 0, 0);
        }
    }
    for (int w = 0; w < NWAVE; ++w) {
        if (wave == w) {
            int t = 0;
#pragma unroll
            for (int pb = 0; pb < NB; ++pb)
#pragma unroll
                for (int qb = pb; qb < NB; ++qb, ++t)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int m = 4 * e + (lane >> 4), n = lane & 15;
                        double &d = red[(pb * 16 + m) * LDP + qb * 16 + n];
                        d = (w == 0) ? acc[t][e] : d + acc[t][e];
                    }
        }
        __syncthreads();
    }
    double *wb = work + (size_t)slice * LDP * LDP;
    for (int e = threadIdx.x; e < LDP * LDP; e += kGramSThreads) wb[e] = red[e];
}

// Batched Gram in two launches.  (1) One workgroup of 8 waves per row slice
// of kGramSliceRows rows of an item: wave w takes row groups of 4 rows
// [4 (w UNR + 8 UNR j), ...) of the slice, accumulates every 16x16 block tile
// (pb <= qb) with FP64 MFMA, the waves add their tiles in LDS in wave order,
// and the slice's partial goes to work[first_slice + slice].  (2) One
// workgroup per item sums its slices in order (deterministic).  Columns at or
// beyond the item's rank read as 0.
constexpr int kGramBThreads = 512;
template <int NB, int UNR>
__global__ __launch_bounds__(kGramBThreads) void k_gram_batched_partial(const GramItem *__restrict__ items, int count,
                                                                       double *__restrict__ work) {
    constexpr int NT = NB * (NB + 1) / 2, LDP = NB * 16, NWAVE = kGramBThreads / 64;
    __shared__ double red[LDP * LDP];
    const int64_t gs = blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].first_slice <= gs) lo = mid;
        else hi = mid - 1;
    }
    const GramItem &it = items[__builtin_amdgcn_readfirstlane(lo)];
    const float *__restrict__ C = it.C;
    const int64_t r0 = (gs - it.first_slice) * kGramSliceRows;
    const int64_t rows = min(it.rows, r0 + kGramSliceRows);
    const int ld = it.ld, R = it.rank;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int kr = lane >> 4, cc = lane & 15;
    double4_t acc[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) acc[i] = (double4_t){0.0, 0.0, 0.0, 0.0};
    for (int64_t g0 = r0 / 4 + (int64_t)wave * UNR; g0 * 4 < rows; g0 += (int64_t)NWAVE * UNR) {
        double v[UNR][NB];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int64_t row = (g0 + u) * 4 + kr;
            const bool rok = row < rows;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int c = b * 16 + cc;
                v[u][b] = (rok && c < R) ? (double)C[row * ld + c] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            int t = 0;
#pragma unroll
            for (int pb = 0; pb < NB; ++pb)
#pragma unroll
                for (int qb = pb; qb < NB; ++qb, ++t)
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[u][pb], v[u][qb], acc[t], 0, 0, 0);
        }
    }
    for (int w = 0; w < NWAVE; ++w) {
        if (wave == w) {
            int t = 0;
#pragma unroll
            for (int pb = 0; pb < NB; ++pb)
#pragma unroll
                for (int qb = pb; qb < NB; ++qb, ++t)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int m = 4 * e + (lane >> 4), n = lane & 15;
                        double &d = red[(pb * 16 + m) * LDP + qb * 16 + n];
                        d = (w == 0) ? acc[t][e] : d + acc[t][e];
                    }
        }
        __syncthreads();
    }
    double *wb = work + (size_t)gs * LDP * LDP;
    for (int e = threadIdx.x; e < LDP * LDP; e += kGramBThreads) wb[e] = red[e];
}

template <int NB>
__global__ __launch_bounds__(256) void k_gram_batched_reduce(const GramItem *__restrict__ items,
                                                             const double *__restrict__ work) {
    constexpr int LDP = NB * 16;
    const GramItem &it = items[blockIdx.x];
    const int R = it.rank;
    for (int e = threadIdx.x; e < R * R; e += 256) {
        const int p = e / R, q = e % R;
        const int a = (p / 16 <= q / 16) ? p : q, b = (p / 16 <= q / 16) ? q : p;
        double s = 0.0;
        for (int64_t k = 0; k < it.nslices; ++k) s += work[(size_t)(it.first_slice + k) * LDP * LDP + a * LDP + b];
        it.G[e] = s;
    }
}

// G[p][q] = sum over slices (upper block triangle mirrored), in two
// deterministic stages: kGramSplit groups of slices, then the groups.
constexpr int kGramSplit = 64;

__device__ __forceinline__ size_t gram_upper(int e, int R, int ld) {
    const int p = e / R, q = e % R;
    const int a = (p / 16 <= q / 16) ? p : q, b = (p / 16 <= q / 16) ? q : p;
    return (size_t)a * ld + b;
}

__global__ __launch_bounds__(kThreads) void k_gram_reduce1(const double *__restrict__ work, int nslices, int R,
                                                           double *__restrict__ w2) {
    const int nb = (R + 15) / 16, ld = nb * 16;
    const int e = blockIdx.x * kThreads + threadIdx.x;
    if (e >= R * R) return;
    const int y = blockIdx.y, S = gridDim.y;
    const int c0 = (int)((int64_t)nslices * y / S), c1 = (int)((int64_t)nslices * (y + 1) / S);
    const size_t off = gram_upper(e, R, ld), stride = (size_t)ld * ld;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int c = c0;
    for (; c + 4 <= c1; c += 4) {
        s0 += work[(size_t)c * stride + off];
        s1 += work[(size_t)(c + 1) * stride + off];
        s2 += work[(size_t)(c + 2) * stride + off];
        s3 += work[(size_t)(c + 3) * stride + off];
    }
    for (; c < c1; ++c) s0 += work[(size_t)c * stride + off];
    w2[(size_t)y * R * R + e] = (s0 + s1) + (s2 + s3);
}

__global__ __launch_bounds__(kThreads) void k_gram_reduce2(const double *__restrict__ w2, int S, int R,
                                                           double *__restrict__ G) {
    const int e = blockIdx.x * kThreads + threadIdx.x;
    if (e >= R * R) return;
    double s = 0.0;
    for (int y = 0; y < S; ++y) s += w2[(size_t)y * R * R + e];
    G[e] = s;
}

// ------------------------------------------------------------------ solve preparation
// One workgroup; R <= 64.  LDS: three R x R FP64 matrices.  W = V^-1 from
// the Cholesky factor: a right-looking factorisation V = L L^T and, in the
// same sweep, a right-looking forward substitution X = L^-1 (step j of the
// substitution needs only column j of L, which step j of the factorisation
// forms), then W = X^T X.  Every thread updates the same matrix elements in
// place at every step; the only values a step reads from other threads (the
// pivot column, the pivot row of X) are staged in double-buffered vectors by
// their owners during the step before: one barrier per step.  The pivot's
// reciprocal square root comes from the hardware estimate and two Newton
// steps, which gives l, 1/l and 1/l^2 without a square root or a divide.
// One 16 x 16 tile (ti, tj) of X^T Y for R x R row-major LDS matrices (R <=
// 64) on v_mfma_f64_16x16x4_f64 (A[m][k] from lane m + 16 k, B[k][n] from
// lane n + 16 k; D[m][n] in lane n + 16 (m % 4), element m / 4).  Indices at
// or beyond R read as 0.  Every lane of the wave must be active.
__device__ __forceinline__ double4_t solve_mfma_tile(const double *X, const double *Y, int R, int ti, int tj,
                                                     int lane) {
    double4_t acc = {0.0, 0.0, 0.0, 0.0};
    const int kq = lane >> 4, row = ti * 16 + (lane & 15), col = tj * 16 + (lane & 15);
    for (int k0 = 0; k0 < R; k0 += 4) {
        const int k = k0 + kq;
        const double a = (k < R && row < R) ? X[k * R + row] : 0.0;
        const double b = (k < R && col < R) ? Y[k * R + col] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    return acc;
}

constexpr int kSolveThreads = 1024;  // 16 waves: 4 matrix elements per thread at R = 64
__device__ __forceinline__ void solve_prep_body(const double *__restrict__ grams, int nmodes, int mode, int R,
                                                const double *__restrict__ gram_m, double *__restrict__ S,
                                                double *__restrict__ lambda, int *__restrict__ status,
                                                double *__restrict__ gram_new) {
    __shared__ double A[64 * 64];
    __shared__ double B[64 * 64];
    __shared__ double Xs[64 * 64];
    __shared__ double vec[2][64];   // staged pivot column of the factorisation
    __shared__ double vecx[2][64];  // staged pivot row of X
    const int tid = threadIdx.x;
    const int RR = R * R;
    // V = Hadamard product of the Grams of every mode except `mode` -> A
    for (int e = tid; e < RR; e += kSolveThreads) {
        double v = 1.0;
        for (int k = 0; k < nmodes; ++k)
            if (k != mode) v *= grams[(size_t)k * RR + e];
        A[e] = v;
    }
    __syncthreads();
    double trace = 0.0;
    for (int i = 0; i < R; ++i) trace += A[i * R + i];
    const double ridge0 = 1e-12 * trace / R;
    // The sweep below changes only lower triangles (of the working matrix and
    // of X): each thread owns up to PT of their R (R + 1) / 2 elements, the
    // t-th in row i = largest with i (i + 1) / 2 <= t, column t - i (i + 1) / 2.
    constexpr int PT = (64 * 65 / 2 + kSolveThreads - 1) / kSolveThreads;
    const int RT = R * (R + 1) / 2;
    int ei[PT], ek[PT];  // row and column of each owned element (t < RT)
#pragma unroll
    for (int m = 0; m < PT; ++m) {
        const int t = tid + m * kSolveThreads;
        int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
        while ((i + 1) * (i + 2) / 2 <= t) ++i;
        while (i > 0 && i * (i + 1) / 2 > t) --i;
        ei[m] = i;
        ek[m] = t - i * (i + 1) / 2;
    }
    int attempt = 0;
    for (; attempt < 4; ++attempt) {
        const double ridge = attempt == 0 ? 0.0 : ridge0 * pow(1e3, (double)(attempt - 1));
        for (int e = tid; e < RR; e += kSolveThreads) {
            const int i = e / R, j = e % R;
            B[e] = A[e] + (i == j ? ridge : 0.0);
            Xs[e] = i == j ? 1.0 : 0.0;
            if (j == 0) vec[0][i] = B[e];
            if (i == 0) vecx[0][j] = Xs[e];
        }
        __syncthreads();
        // Step j: with column j of the working matrix as it was before the
        // step (cj) and l = L[j][j], the factorisation scales column j and
        // updates the trailing matrix (lower triangle of B), and the
        // substitution scales row j of X and subtracts L[i][j] X[j][:] / l
        // (= cj[i] X[j][:] / d) from the rows below, X[j][:] as it was before
        // the step (rj).  The owners of column j + 1 and of row j + 1 of X
        // stage them for the next step.  All threads read the same pivot, so
        // they leave the loop together.
        bool ok = true;
        for (int j = 0; j < R; ++j) {
            const double *cj = vec[j & 1];
            double *cn = vec[(j + 1) & 1];
            const double *rj = vecx[j & 1];
            double *rn = vecx[(j + 1) & 1];
            const double d = cj[j];
            if (!(d > 0.0) || !isfinite(d)) {
                ok = false;
                break;
            }
            double r = __builtin_amdgcn_rsq(d);
            r = r * (1.5 - 0.5 * d * r * r);
            r = r * (1.5 - 0.5 * d * r * r);
            const double l = d * r, il = r, id = r * r;
#pragma unroll
            for (int m = 0; m < PT; ++m) {
                // rows above the pivot are final in both matrices
                if (tid + m * kSolveThreads < RT && ei[m] >= j) {
                    const int i = ei[m], k = ek[m], e = i * R + k;
                    double x = B[e];
                    if (k == j) {
                        x = i == j ? l : (i > j ? x * il : x);
                        B[e] = x;
                    } else if (i > j && k > j && k <= i) {
                        x -= cj[i] * cj[k] * id;
                        B[e] = x;
                    }
                    if (k == j + 1 && i > j) cn[i] = x;
                    double y = Xs[e];
                    if (i == j) {
                        y *= il;
                        Xs[e] = y;
                    } else if (i > j && k <= j) {
                        y -= cj[i] * rj[k] * id;
                        Xs[e] = y;
                    }
                    if (i == j + 1) rn[k] = y;
                }
            }
            __syncthreads();
        }
        if (ok) break;
        __syncthreads();
    }
    if (attempt == 4) {
        if (tid == 0) *status = -1;
        return;
    }
    // The three R x R products below run on FP64 MFMA, one 16 x 16 output
    // tile per wave.  Every left operand is read transposed (X^T, and the
    // symmetric Gm and W), so a wave's reads of either operand run along a
    // row of LDS.
    const int wave = tid >> 6, lane = tid & 63, nt = (R + 15) / 16;
    const bool tile_wave = wave < nt * nt;
    const int ti = tile_wave ? wave / nt : 0, tj = tile_wave ? wave % nt : 0;
    auto store_tile = [&](const double4_t &acc, double *dst) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = ti * 16 + 4 * e + (lane >> 4), c = tj * 16 + (lane & 15);
            if (r < R && c < R) dst[r * R + c] = acc[e];
        }
    };
    // W = X^T X = V^-1 into B (L is no longer needed)
    if (tile_wave) store_tile(solve_mfma_tile(Xs, Xs, R, ti, tj, lane), B);
    for (int e = tid; e < RR; e += kSolveThreads) A[e] = gram_m[e];
    __syncthreads();
    // Tm = Gm W into Xs
    if (tile_wave) store_tile(solve_mfma_tile(A, B, R, ti, tj, lane), Xs);
    __syncthreads();
    // P = W Tm = W Gm W into A (every read of Gm is done)
    if (tile_wave) store_tile(solve_mfma_tile(B, Xs, R, ti, tj, lane), A);
    __syncthreads();
    // lambda_r^2 = P[r][r]
    __shared__ double lam_s[64];
    for (int r = tid; r < R; r += kSolveThreads) {
        const double s2 = A[r * R + r];
        const double l = s2 > 0.0 ? sqrt(s2) : 0.0;
        lam_s[r] = l > 0.0 ? l : 1.0;
        lambda[r] = lam_s[r];
    }
    __syncthreads();
    // The Gram of the new factor C = M S without reading C: C^T C = S^T Gm S,
    // and with S = W diag(1/lambda), W symmetric, its (p, q) entry is
    // P[p][q] / (lambda_p lambda_q).  FP64 throughout, so it is the Gram of
    // the exact product rather than of C rounded to FP32.  Only the other
    // modes' Grams were read above, so the slot of `mode` may be overwritten.
    if (gram_new)
        for (int e = tid; e < RR; e += kSolveThreads) gram_new[e] = A[e] / (lam_s[e / R] * lam_s[e % R]);
    for (int e = tid; e < RR; e += kSolveThreads) S[e] = B[e] / lam_s[e % R];
    if (tid == 0) *status = attempt;
}

__global__ __launch_bounds__(kSolveThreads) void k_solve_prep(const double *__restrict__ grams, int nmodes, int mode, int R,
                                                         const double *__restrict__ gram_m, double *__restrict__ S,
                                                         double *__restrict__ lambda, int *__restrict__ status,
                                                         double *__restrict__ gram_new) {
    solve_prep_body(grams, nmodes, mode, R, gram_m, S, lambda, status, gram_new);
}

__global__ __launch_bounds__(kSolveThreads) void k_solve_prep_batched(const SolveItem *__restrict__ items, int mode) {
    const SolveItem &it = items[blockIdx.x];
    solve_prep_body(it.grams, it.nmodes, mode, it.rank, it.gram_m, it.S, it.lambda, it.status + mode,
                    it.gram_new);
}

// ------------------------------------------------------------------ apply
// RP = R padded to 16/32/64; CG = RP/4 column groups of 4; RG = 256/CG row groups of 4 rows.
template <int RP>
__device__ __forceinline__ void apply_body(const float *__restrict__ M, int ldm, int64_t rows, int R,
                                           const double *__restrict__ S, float *__restrict__ C,
                                           const double *__restrict__ lambda, double *__restrict__ inner_partials,
                                           int64_t blk) {
    constexpr int CG = RP / 4, RG = kThreads / CG, RW = RG * 4;
    __shared__ double sS[RP * RP];
    __shared__ float sM[RW * RP];
    __shared__ double red[4];
    const int tid = threadIdx.x;
    for (int e = tid; e < RP * RP; e += kThreads) {
        const int p = e / RP, q = e % RP;
        sS[e] = (p < R && q < R) ? S[p * R + q] : 0.0;
    }
    const int64_t row0 = blk * RW;
    for (int e = tid; e < RW * RP; e += kThreads) {
        const int r = e / RP, c = e % RP;
        const int64_t row = row0 + r;
        sM[e] = (row < rows && c < R) ? M[row * ldm + c] : 0.f;
    }
    __syncthreads();
    const int cg = tid % CG, rg = tid / CG;
    const int c0 = cg * 4, rl = rg * 4;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[i][q] = 0.0;
    for (int k = 0; k < R; ++k) {
        double m[4], s[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) m[i] = (double)sM[(rl + i) * RP + k];
#pragma unroll
        for (int q = 0; q < 4; ++q) s[q] = sS[k * RP + c0 + q];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[i][q] = fma(m[i], s[q], acc[i][q]);
    }
    double inner = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t row = row0 + rl + i;
        if (row < rows) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int c = c0 + q;
                if (c < R) {
                    const float v = (float)acc[i][q];
                    C[row * R + c] = v;
                    if (inner_partials) inner += (double)sM[(rl + i) * RP + c] * (double)v * lambda[c];
                }
            }
        }
    }
    if (inner_partials) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) inner += __shfl_down(inner, off, 64);
        if ((tid & 63) == 0) red[tid >> 6] = inner;
        __syncthreads();
        if (tid == 0) inner_partials[blk] = red[0] + red[1] + red[2] + red[3];
    }
}


// Single-tensor apply on FP64 MFMA: C = M S for 16-row tiles, one tile per
// wave at a time (tiles strided over the grid), S (RP x RP) in LDS.  The k
// index of v_mfma_f64_16x16x4_f64 is only summed over, so step j takes
// columns kq KS + j (KS = RP / 4) for lane quarter kq: every lane then holds
// 16 (or RP / 4) contiguous values of its row of M, loaded once per tile.
// Also the fit's inner product sum_rc M[r][c] C[r][c] lambda[c] per block.
template <int NB>
__global__ __launch_bounds__(kThreads) void k_apply_mfma(const float *__restrict__ M, int64_t rows, int R,
                                                         const double *__restrict__ S, float *__restrict__ C,
                                                         const double *__restrict__ lambda,
                                                         double *__restrict__ inner_partials) {
    constexpr int RP = NB * 16, KS = RP / 4;
    __shared__ double sS[RP * RP];
    __shared__ double red[kThreads / 64];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int e = tid; e < RP * RP; e += kThreads) {
        const int p = e / RP, q = e % RP;
        sS[e] = (p < R && q < R) ? S[p * R + q] : 0.0;
    }
    __syncthreads();
    const int mrow = lane & 15, kq = lane >> 4;
    const int64_t ntile = (rows + 15) / 16;
    const bool vec_ok = R == RP && ((uintptr_t)M & 15u) == 0;
    double inner = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * (kThreads / 64) + wave; t < ntile;
         t += (int64_t)gridDim.x * (kThreads / 64)) {
        const int64_t r0 = t * 16;
        const int64_t arow = r0 + mrow;
        float a[KS];
        if (vec_ok && arow < rows) {
            // the lane's KS values are contiguous and 16-byte aligned: vector loads
            const float4 *mp = reinterpret_cast<const float4 *>(M + arow * R + kq * KS);
#pragma unroll
            for (int j4 = 0; j4 < KS / 4; ++j4) {
                const float4 v = mp[j4];
                a[4 * j4] = v.x;
                a[4 * j4 + 1] = v.y;
                a[4 * j4 + 2] = v.z;
                a[4 * j4 + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int j = 0; j < KS; ++j) {
                const int c = kq * KS + j;
                a[j] = (arow < rows && c < R) ? M[arow * R + c] : 0.f;
            }
        }
        double4_t acc[NB];
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) acc[cb] = (double4_t){0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int j = 0; j < KS; ++j) {
            const double av = (double)a[j];
            const double *srow = sS + (kq * KS + j) * RP + mrow;  // B[k][n] = S[k][cb 16 + n], n = lane & 15
#pragma unroll
            for (int cb = 0; cb < NB; ++cb)
                acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, srow[cb * 16], acc[cb], 0, 0, 0);
        }
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = 4 * e + (lane >> 4), n = lane & 15;
                const int64_t row = r0 + m;
                const int c = cb * 16 + n;
                if (row < rows && c < R) {
                    const float v = (float)acc[cb][e];
                    C[row * R + c] = v;
                    if (inner_partials) inner += (double)M[row * R + c] * (double)v * lambda[c];
                }
            }
        }
    }
    if (inner_partials) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) inner += __shfl_down(inner, off, 64);
        if (lane == 0) red[wave] = inner;
        __syncthreads();
        if (tid == 0) {
            double sum = 0.0;
            for (int w = 0; w < kThreads / 64; ++w) sum += red[w];
            inner_partials[blockIdx.x] = sum;
        }
    }
}

// Batched: block `g` belongs to the last item whose first_block <= g.
template <int RP>
__global__ __launch_bounds__(kThreads) void k_apply_batched(const ApplyItem *__restrict__ items, int count) {
    const int64_t g = blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].first_block <= g) lo = mid;
        else hi = mid - 1;
    }
    const ApplyItem &it = items[__builtin_amdgcn_readfirstlane(lo)];
    apply_body<RP>(it.M, it.ldm, it.rows, it.rank, it.S, it.C, it.lambda, it.inner, g - it.first_block);
}

template <int RP>
int apply_rows_per_block() { return (kThreads / (RP / 4)) * 4; }

int apply_rp(int R) { return R <= 16 ? 16 : (R <= 32 ? 32 : 64); }

// ------------------------------------------------------------------ fit
__device__ __forceinline__ void fit_body(const double *__restrict__ grams, int nmodes, int R,
                                         const double *__restrict__ lambda,
                                         const double *__restrict__ inner_partials, int nparts, double norm_x2,
                                         double *__restrict__ out) {
    __shared__ double red[2][4];
    const int tid = threadIdx.x;
    const int RR = R * R;
    double xh = 0.0;
    for (int e = tid; e < RR; e += kThreads) {
        double v = 1.0;
        for (int k = 0; k < nmodes; ++k) v *= grams[(size_t)k * RR + e];
        xh += lambda[e / R] * v * lambda[e % R];
    }
    double in = 0.0;
    for (int i = tid; i < nparts; i += kThreads) in += inner_partials[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        xh += __shfl_down(xh, off, 64);
        in += __shfl_down(in, off, 64);
    }
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = xh;
        red[1][tid >> 6] = in;
    }
    __syncthreads();
    if (tid == 0) {
        const double nxh = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        const double inner = red[1][0] + red[1][1] + red[1][2] + red[1][3];
        double r2 = norm_x2 + nxh - 2.0 * inner;
        if (r2 < 0.0) r2 = 0.0;
        out[0] = 1.0 - sqrt(r2) / sqrt(norm_x2);
        out[1] = nxh;
        out[2] = inner;
    }
}

__global__ __launch_bounds__(kThreads) void k_fit(const double *__restrict__ grams, int nmodes, int R,
                                                  const double *__restrict__ lambda,
                                                  const double *__restrict__ inner_partials, int nparts,
                                                  double norm_x2, double *__restrict__ out) {
    fit_body(grams, nmodes, R, lambda, inner_partials, nparts, norm_x2, out);
}

__global__ __launch_bounds__(kThreads) void k_fit_batched(const FitItem *__restrict__ items) {
    const FitItem &it = items[blockIdx.x];
    fit_body(it.grams, it.nmodes, it.rank, it.lambda, it.inner, it.nparts, it.norm_x2, it.out);
}

// out[1] must hold |Xhat|^2 from k_fit; writes out[0] (fit) and out[3] (residual^2).
__device__ __forceinline__ void fit_direct_body(const double *__restrict__ parts, int64_t nparts, double norm_x2,
                                                double *__restrict__ out) {
    __shared__ double red[2][4];
    const int tid = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (int64_t i = tid; i < nparts; i += kThreads) {
        a += parts[2 * i];
        b += parts[2 * i + 1];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
    }
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = a;
        red[1][tid >> 6] = b;
    }
    __syncthreads();
    if (tid == 0) {
        const double res = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        const double hat = red[1][0] + red[1][1] + red[1][2] + red[1][3];
        double off_support = out[1] - hat;  // model mass on the zero cells
        if (off_support < 0.0) off_support = 0.0;
        const double r2 = res + off_support;
        out[0] = 1.0 - sqrt(r2) / sqrt(norm_x2);
        out[3] = r2;
    }
}

__global__ __launch_bounds__(kThreads) void k_fit_direct(const double *__restrict__ parts, int nparts, double norm_x2,
                                                         double *__restrict__ out) {
    fit_direct_body(parts, nparts, norm_x2, out);
}

__global__ __launch_bounds__(kThreads) void k_fit_direct_batched(const FitDirectItem *__restrict__ items) {
    const FitDirectItem &it = items[blockIdx.x];
    fit_direct_body(it.parts, it.nparts, it.norm_x2, it.out);
}

}  // namespace

size_t gram_work_bytes(int64_t rows, int rank) {
    const int ld = gram_nb(rank) * 16;
    return (size_t)gram_chunks(rows, rank) * ld * ld * sizeof(double) + (size_t)kGramSplit * rank * rank * sizeof(double);
}

spt_status launch_gram(const float *C, int64_t rows, int rank, double *G, double *work, size_t work_bytes,
                       hipStream_t s) {
    if (rank > 64) return fail(SPT_E_INVALID_ARG, "gram: rank above 64");
    const int chunks = gram_chunks(rows, rank);
    if (gram_work_bytes(rows, rank) > work_bytes) return fail(SPT_E_INVALID_ARG, "gram: workspace too small");
    const int nb = gram_nb(rank), ld = nb * 16;
    const dim3 g((unsigned)chunks), b(kGramSThreads);
    if (nb == 1) hipLaunchKernelGGL((k_gram_partial<1, 4>), g, b, 0, s, C, rows, rank, work);
    else if (nb == 2) hipLaunchKernelGGL((k_gram_partial<2, 4>), g, b, 0, s, C, rows, rank, work);
    else if (nb == 3) hipLaunchKernelGGL((k_gram_partial<3, 2>), g, b, 0, s, C, rows, rank, work);
    else hipLaunchKernelGGL((k_gram_partial<4, 1>), g, b, 0, s, C, rows, rank, work);
    const int nslices = chunks;
    const int S = std::min(kGramSplit, nslices);
    double *w2 = work + (size_t)nslices * ld * ld;
    const int rb = (rank * rank + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_gram_reduce1, dim3(rb, S), dim3(kThreads), 0, s, work, nslices, rank, w2);
    hipLaunchKernelGGL(k_gram_reduce2, dim3(rb), dim3(kThreads), 0, s, w2, S, rank, G);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

spt_status launch_solve_prep(const double *grams, int nmodes, int mode, int rank, const double *gram_m, double *S,
                             double *lambda, int *status_out, double *gram_new, hipStream_t s) {
    if (rank > 64) return fail(SPT_E_INVALID_ARG, "solve: rank above 64");
    hipLaunchKernelGGL(k_solve_prep, dim3(1), dim3(kSolveThreads), 0, s, grams, nmodes, mode, rank, gram_m, S, lambda,
                       status_out, gram_new);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

constexpr int64_t kApplyMaxBlocks = 2048;
int apply_blocks(int64_t rows, int rank) {
    (void)rank;
    const int64_t tiles = (rows + 15) / 16;  // 16-row MFMA tiles, 4 per block at a time
    return (int)std::max<int64_t>(1, std::min<int64_t>((tiles + 3) / 4, kApplyMaxBlocks));
}


spt_status launch_apply(const float *M, int64_t rows, int rank, const double *S, float *C, const double *lambda,
                        double *inner_partials, int *nparts_out, hipStream_t s) {
    const int blocks = apply_blocks(rows, rank);
    const int rp = apply_rp(rank);
    if (rp == 16)
        hipLaunchKernelGGL(k_apply_mfma<1>, dim3(blocks), dim3(kThreads), 0, s, M, rows, rank, S, C, lambda,
                           inner_partials);
    else if (rp == 32)
        hipLaunchKernelGGL(k_apply_mfma<2>, dim3(blocks), dim3(kThreads), 0, s, M, rows, rank, S, C, lambda,
                           inner_partials);
    else
        hipLaunchKernelGGL(k_apply_mfma<4>, dim3(blocks), dim3(kThreads), 0, s, M, rows, rank, S, C, lambda,
                           inner_partials);
    SPT_HIP(hipGetLastError());
    if (nparts_out) *nparts_out = blocks;
    return SPT_OK;
}

spt_status launch_fit(const double *grams, int nmodes, int rank, const double *lambda, const double *inner_partials,
                      int nparts, double norm_x2, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_fit, dim3(1), dim3(kThreads), 0, s, grams, nmodes, rank, lambda, inner_partials, nparts, norm_x2,
                       out);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

spt_status launch_fit_direct_batched(const FitDirectItem *items, int count, hipStream_t s) {
    if (count <= 0) return SPT_OK;
    hipLaunchKernelGGL(k_fit_direct_batched, dim3((unsigned)count), dim3(kThreads), 0, s, items);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

spt_status launch_fit_direct(const double *resid_partials, int nparts, double norm_x2, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_fit_direct, dim3(1), dim3(kThreads), 0, s, resid_partials, nparts, norm_x2, out);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

int64_t gram_slices(int64_t rows) { return std::max<int64_t>(1, (rows + kGramSliceRows - 1) / kGramSliceRows); }

size_t gram_batched_ws_bytes(int64_t total_slices, int rmax) {
    const size_t ldp = (size_t)gram_nb(rmax) * 16;
    return (size_t)std::max<int64_t>(total_slices, 1) * ldp * ldp * sizeof(double);
}

spt_status launch_gram_batched(const GramItem *items, int count, int64_t total_slices, int rmax, double *work,
                               hipStream_t s) {
    if (count == 0 || total_slices == 0) return SPT_OK;
    if (rmax > 64) return fail(SPT_E_INVALID_ARG, "gram: rank above 64");
    const int nb = gram_nb(rmax);
    const dim3 g((unsigned)total_slices), b(kGramBThreads);
    if (nb == 1) {
        hipLaunchKernelGGL((k_gram_batched_partial<1, 4>), g, b, 0, s, items, count, work);
        hipLaunchKernelGGL(k_gram_batched_reduce<1>, dim3(count), dim3(256), 0, s, items, work);
    } else if (nb == 2) {
        hipLaunchKernelGGL((k_gram_batched_partial<2, 4>), g, b, 0, s, items, count, work);
        hipLaunchKernelGGL(k_gram_batched_reduce<2>, dim3(count), dim3(256), 0, s, items, work);
    } else if (nb == 3) {
        hipLaunchKernelGGL((k_gram_batched_partial<3, 2>), g, b, 0, s, items, count, work);
        hipLaunchKernelGGL(k_gram_batched_reduce<3>, dim3(count), dim3(256), 0, s, items, work);
    } else {
        hipLaunchKernelGGL((k_gram_batched_partial<4, 2>), g, b, 0, s, items, count, work);
        hipLaunchKernelGGL(k_gram_batched_reduce<4>, dim3(count), dim3(256), 0, s, items, work);
    }
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

spt_status launch_solve_prep_batched(const SolveItem *items, int count, int mode, hipStream_t s) {
    if (count == 0) return SPT_OK;
    hipLaunchKernelGGL(k_solve_prep_batched, dim3(count), dim3(kSolveThreads), 0, s, items, mode);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

int apply_rows_per_launch_block(int rmax) {
    const int rp = apply_rp(rmax);
    return rp == 16 ? apply_rows_per_block<16>() : (rp == 32 ? apply_rows_per_block<32>() : apply_rows_per_block<64>());
}

spt_status launch_apply_batched(const ApplyItem *items, int count, int64_t total_blocks, int rmax, hipStream_t s) {
    if (total_blocks == 0) return SPT_OK;
    const int rp = apply_rp(rmax);
    if (rp == 16) hipLaunchKernelGGL(k_apply_batched<16>, dim3((unsigned)total_blocks), dim3(kThreads), 0, s, items, count);
    else if (rp == 32) hipLaunchKernelGGL(k_apply_batched<32>, dim3((unsigned)total_blocks), dim3(kThreads), 0, s, items, count);
    else hipLaunchKernelGGL(k_apply_batched<64>, dim3((unsigned)total_blocks), dim3(kThreads), 0, s, items, count);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

spt_status launch_fit_batched(const FitItem *items, int count, hipStream_t s) {
    if (count == 0) return SPT_OK;
    hipLaunchKernelGGL(k_fit_batched, dim3(count), dim3(kThreads), 0, s, items);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

}  // namespace spt
