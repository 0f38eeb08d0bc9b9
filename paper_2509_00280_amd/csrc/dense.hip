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
#include "spt_internal.h"

namespace spt {

namespace {

constexpr int kThreads = 256;
constexpr int kGramRowsPerChunk = 4096;
constexpr int kGramMaxChunks = 512;
constexpr int kTilesPerWave = 4;

typedef double double4_t __attribute__((ext_vector_type(4)));

int gram_nb(int R) { return (R + 15) / 16; }
int gram_ntiles(int R) { const int nb = gram_nb(R); return nb * (nb + 1) / 2; }
int gram_chunks(int64_t rows) {
    int64_t c = (rows + kGramRowsPerChunk - 1) / kGramRowsPerChunk;
    if (c < 1) c = 1;
    if (c > kGramMaxChunks) c = kGramMaxChunks;
    return (int)c;
}

// Partial Grams of row chunks.  Tile t (pb <= qb) of R in 16x16 blocks; the
// wave's lane layout for v_mfma_f64_16x16x4_f64: A[m][k] from lane m + 16k,
// B[k][n] from lane n + 16k, D[m][n] in lane n + 16*(m%4), element m/4.
__global__ __launch_bounds__(kThreads) void k_gram_partial(const float *__restrict__ C, int64_t rows, int R,
                                                           double *__restrict__ work) {
    const int nb = (R + 15) / 16;
    const int ntiles = nb * (nb + 1) / 2;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int t_base = blockIdx.y * (4 * kTilesPerWave) + wave;
    int pb[kTilesPerWave], qb[kTilesPerWave];
    bool act[kTilesPerWave];
#pragma unroll
    for (int i = 0; i < kTilesPerWave; ++i) {
        int t = t_base + 4 * i;
        act[i] = t < ntiles;
        if (!act[i]) t = 0;
        // decode t -> (p, q) with p <= q, row-major over the upper triangle
        int p = 0, rem = t;
        while (rem >= nb - p) {
            rem -= nb - p;
            ++p;
        }
        pb[i] = p;
        qb[i] = p + rem;
    }
    double4_t acc[kTilesPerWave];
#pragma unroll
    for (int i = 0; i < kTilesPerWave; ++i) acc[i] = (double4_t){0.0, 0.0, 0.0, 0.0};
    const int kr = lane >> 4, cc = lane & 15;
    const int64_t r_per = ((rows + gridDim.x - 1) / gridDim.x + 3) & ~3LL;
    const int64_t r0 = (int64_t)blockIdx.x * r_per;
    const int64_t r1 = r0 + r_per < rows ? r0 + r_per : rows;
    for (int64_t i0 = r0; i0 < r1; i0 += 4) {
        const int64_t row = i0 + kr;
        const float *rp = C + row * R;
        const bool rok = row < r1;
#pragma unroll
        for (int i = 0; i < kTilesPerWave; ++i) {
            if (act[i]) {
                const int ca = pb[i] * 16 + cc, cb = qb[i] * 16 + cc;
                const double a = (rok && ca < R) ? (double)rp[ca] : 0.0;
                const double b = (rok && cb < R) ? (double)rp[cb] : 0.0;
                acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
            }
        }
    }
    const int ld = nb * 16;
    double *wb = work + (size_t)blockIdx.x * ld * ld;
#pragma unroll
    for (int i = 0; i < kTilesPerWave; ++i) {
        if (act[i]) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int m = 4 * v + (lane >> 4), n = lane & 15;
                wb[(size_t)(pb[i] * 16 + m) * ld + qb[i] * 16 + n] = acc[i][v];
            }
        }
    }
}

// G[p][q] = sum over chunks (upper block triangle mirrored), deterministic order.
__global__ __launch_bounds__(kThreads) void k_gram_reduce(const double *__restrict__ work, int nchunks, int R,
                                                          double *__restrict__ G) {
    const int nb = (R + 15) / 16, ld = nb * 16;
    for (int e = blockIdx.x * kThreads + threadIdx.x; e < R * R; e += gridDim.x * kThreads) {
        const int p = e / R, q = e % R;
        const int a = (p / 16 <= q / 16) ? p : q, b = (p / 16 <= q / 16) ? q : p;
        double s = 0.0;
        for (int c = 0; c < nchunks; ++c) s += work[(size_t)c * ld * ld + (size_t)a * ld + b];
        G[e] = s;
    }
}

// ------------------------------------------------------------------ solve preparation
// One workgroup; R <= 64.  LDS: two R x R FP64 matrices.
__global__ __launch_bounds__(kThreads) void k_solve_prep(const double *__restrict__ grams, int nmodes, int mode, int R,
                                                         const double *__restrict__ gram_m, double *__restrict__ S,
                                                         double *__restrict__ lambda, int *__restrict__ status) {
    __shared__ double A[64 * 64];
    __shared__ double B[64 * 64];
    __shared__ double sdiag;
    __shared__ int sfail;
    const int tid = threadIdx.x;
    const int RR = R * R;
    // V = Hadamard product of the Grams of every mode except `mode` -> A
    for (int e = tid; e < RR; e += kThreads) {
        double v = 1.0;
        for (int k = 0; k < nmodes; ++k)
            if (k != mode) v *= grams[(size_t)k * RR + e];
        A[e] = v;
    }
    __syncthreads();
    double trace = 0.0;
    for (int i = 0; i < R; ++i) trace += A[i * R + i];
    const double ridge0 = 1e-12 * trace / R;
    int attempt = 0;
    for (; attempt < 4; ++attempt) {
        const double ridge = attempt == 0 ? 0.0 : ridge0 * pow(1e3, (double)(attempt - 1));
        for (int e = tid; e < RR; e += kThreads) {
            const int i = e / R, j = e % R;
            B[e] = (i >= j) ? A[e] + (i == j ? ridge : 0.0) : 0.0;
        }
        if (tid == 0) sfail = 0;
        __syncthreads();
        // left-looking Cholesky in B (lower triangle), column by column
        for (int j = 0; j < R; ++j) {
            double s = 0.0;
            const int i = j + tid;
            if (i < R) {
                s = B[i * R + j];
                for (int k = 0; k < j; ++k) s -= B[i * R + k] * B[j * R + k];
            }
            if (tid == 0) {
                if (!(s > 0.0) || !isfinite(s)) sfail = 1;
                sdiag = sqrt(s > 0.0 ? s : 1.0);
            }
            __syncthreads();
            if (i < R) B[i * R + j] = (tid == 0) ? sdiag : s / sdiag;
            __syncthreads();
        }
        if (!sfail) break;
        __syncthreads();
    }
    if (attempt == 4) {
        if (tid == 0) *status = -1;
        return;
    }
    // Linv (lower) into A: thread c solves L x = e_c by forward substitution
    for (int c = tid; c < R; c += kThreads) {
        for (int i = 0; i < R; ++i) {
            if (i < c) {
                A[i * R + c] = 0.0;
                continue;
            }
            double s = (i == c) ? 1.0 : 0.0;
            for (int k = c; k < i; ++k) s -= B[i * R + k] * A[k * R + c];
            A[i * R + c] = s / B[i * R + i];
        }
    }
    __syncthreads();
    // W = Linv^T Linv into B
    for (int e = tid; e < RR; e += kThreads) {
        const int p = e / R, q = e % R;
        const int i0 = p > q ? p : q;
        double s = 0.0;
        for (int i = i0; i < R; ++i) s += A[i * R + p] * A[i * R + q];
        B[e] = s;
    }
    __syncthreads();
    // Tm = gram_m W into A
    for (int e = tid; e < RR; e += kThreads) {
        const int a = e / R, r = e % R;
        double s = 0.0;
        for (int b = 0; b < R; ++b) s += gram_m[a * R + b] * B[b * R + r];
        A[e] = s;
    }
    __syncthreads();
    // lambda_r^2 = sum_a W[r][a] Tm[a][r]
    __shared__ double lam_s[64];
    for (int r = tid; r < R; r += kThreads) {
        double s = 0.0;
        for (int a = 0; a < R; ++a) s += B[r * R + a] * A[a * R + r];
        const double l = s > 0.0 ? sqrt(s) : 0.0;
        lam_s[r] = l > 0.0 ? l : 1.0;
        lambda[r] = lam_s[r];
    }
    __syncthreads();
    for (int e = tid; e < RR; e += kThreads) S[e] = B[e] / lam_s[e % R];
    if (tid == 0) *status = attempt;
}

// ------------------------------------------------------------------ apply
// RP = R padded to 16/32/64; CG = RP/4 column groups of 4; RG = 256/CG row groups of 4 rows.
template <int RP>
__global__ __launch_bounds__(kThreads) void k_apply(const float *__restrict__ M, int64_t rows, int R,
                                                    const double *__restrict__ S, float *__restrict__ C,
                                                    const double *__restrict__ lambda,
                                                    double *__restrict__ inner_partials) {
    constexpr int CG = RP / 4, RG = kThreads / CG, RW = RG * 4;
    __shared__ double sS[RP * RP];
    __shared__ float sM[RW * RP];
    __shared__ double red[4];
    const int tid = threadIdx.x;
    for (int e = tid; e < RP * RP; e += kThreads) {
        const int p = e / RP, q = e % RP;
        sS[e] = (p < R && q < R) ? S[p * R + q] : 0.0;
    }
    const int64_t row0 = (int64_t)blockIdx.x * RW;
    for (int e = tid; e < RW * RP; e += kThreads) {
        const int r = e / RP, c = e % RP;
        const int64_t row = row0 + r;
        sM[e] = (row < rows && c < R) ? M[row * R + c] : 0.f;
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
        if (tid == 0) inner_partials[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    }
}

template <int RP>
int apply_rows_per_block() { return (kThreads / (RP / 4)) * 4; }

int apply_rp(int R) { return R <= 16 ? 16 : (R <= 32 ? 32 : 64); }

// ------------------------------------------------------------------ fit
__global__ __launch_bounds__(kThreads) void k_fit(const double *__restrict__ grams, int nmodes, int R,
                                                  const double *__restrict__ lambda,
                                                  const double *__restrict__ inner_partials, int nparts,
                                                  double norm_x2, double *__restrict__ out) {
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

// out[1] must hold |Xhat|^2 from k_fit; writes out[0] (fit) and out[3] (residual^2).
__global__ __launch_bounds__(kThreads) void k_fit_direct(const double *__restrict__ parts, int nparts, double norm_x2,
                                                         double *__restrict__ out) {
    __shared__ double red[2][4];
    const int tid = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (int i = tid; i < nparts; i += kThreads) {
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

}  // namespace

size_t gram_work_bytes(int64_t rows, int rank) {
    const int ld = gram_nb(rank) * 16;
    return (size_t)gram_chunks(rows) * ld * ld * sizeof(double);
}

spt_status launch_gram(const float *C, int64_t rows, int rank, double *G, double *work, size_t work_bytes,
                       hipStream_t s) {
    const int chunks = gram_chunks(rows);
    if (gram_work_bytes(rows, rank) > work_bytes) return fail(SPT_E_INVALID_ARG, "gram: workspace too small");
    const int ty = (gram_ntiles(rank) + 4 * kTilesPerWave - 1) / (4 * kTilesPerWave);
    hipLaunchKernelGGL(k_gram_partial, dim3(chunks, ty), dim3(kThreads), 0, s, C, rows, rank, work);
    int rb = (rank * rank + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_gram_reduce, dim3(rb), dim3(kThreads), 0, s, work, chunks, rank, G);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

spt_status launch_solve_prep(const double *grams, int nmodes, int mode, int rank, const double *gram_m, double *S,
                             double *lambda, int *status_out, hipStream_t s) {
    if (rank > 64) return fail(SPT_E_INVALID_ARG, "solve: rank above 64");
    hipLaunchKernelGGL(k_solve_prep, dim3(1), dim3(kThreads), 0, s, grams, nmodes, mode, rank, gram_m, S, lambda,
                       status_out);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

int apply_blocks(int64_t rows, int rank) {
    const int rp = apply_rp(rank);
    const int rw = rp == 16 ? apply_rows_per_block<16>() : (rp == 32 ? apply_rows_per_block<32>() : apply_rows_per_block<64>());
    int64_t b = (rows + rw - 1) / rw;
    return (int)(b < 1 ? 1 : b);
}

spt_status launch_apply(const float *M, int64_t rows, int rank, const double *S, float *C, const double *lambda,
                        double *inner_partials, int *nparts_out, hipStream_t s) {
    const int blocks = apply_blocks(rows, rank);
    const int rp = apply_rp(rank);
    if (rp == 16)
        hipLaunchKernelGGL(k_apply<16>, dim3(blocks), dim3(kThreads), 0, s, M, rows, rank, S, C, lambda, inner_partials);
    else if (rp == 32)
        hipLaunchKernelGGL(k_apply<32>, dim3(blocks), dim3(kThreads), 0, s, M, rows, rank, S, C, lambda, inner_partials);
    else
        hipLaunchKernelGGL(k_apply<64>, dim3(blocks), dim3(kThreads), 0, s, M, rows, rank, S, C, lambda, inner_partials);
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

spt_status launch_fit_direct(const double *resid_partials, int nparts, double norm_x2, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_fit_direct, dim3(1), dim3(kThreads), 0, s, resid_partials, nparts, norm_x2, out);
    SPT_HIP(hipGetLastError());
    return SPT_OK;
}

}  // namespace spt
