/*
 * Oracle (test infrastructure only): plain, single-threaded FP64 sparse MTTKRP
 * over a coordinate-list (COO) tensor.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark load this file's library; the
 * product path never does.  It shares no code with the GPU library.
 *
 * Definition followed (Section II-B, MTTKRP paragraph and Fig. 2): the
 * mode-n MTTKRP of an N-way tensor X with factor matrices C^(k) is
 * X_(n) (KRP over k != n of C^(k)).  Element-wise, every nonzero v at
 * coordinates (i_1..i_N) reads row i_k of every C^(k), k != n, multiplies
 * those rows element-wise (the Hadamard product that forms its Khatri-Rao
 * row), scales by v and adds the result into row i_n of the output.
 *
 * Reading taken where the paper is silent: the output is a separate
 * I_n x R matrix, zeroed first (the paper says the nonzero "updates row
 * i_n" of the factor; CP-ALS needs the product itself).
 *
 * Layout: coords is structure-of-arrays, coords[k * nnz + e] = i_k of
 * nonzero e (0-based); factors[k] is row-major I_k x rank; out is row-major
 * I_mode x rank.  Accumulation is FP64 in input order.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int oracle_mttkrp(int nmodes, const int64_t *dims, int64_t nnz,
                  const uint32_t *coords, const float *vals,
                  const double *const *factors, int rank, int mode,
                  double *out)
{
    if (nmodes < 1 || mode < 0 || mode >= nmodes || rank < 1)
        return -1;
    memset(out, 0, sizeof(double) * (size_t)dims[mode] * (size_t)rank);
    double *row = (double *)malloc(sizeof(double) * (size_t)rank);
    if (!row)
        return -2;
    for (int64_t e = 0; e < nnz; ++e) {
        /* start from the nonzero's value */
        for (int r = 0; r < rank; ++r)
            row[r] = (double)vals[e];
        /* Hadamard product of the rows i_k of every other factor */
        for (int k = 0; k < nmodes; ++k) {
            if (k == mode)
                continue;
            const double *f = factors[k] + (int64_t)coords[(int64_t)k * nnz + e] * rank;
            for (int r = 0; r < rank; ++r)
                row[r] *= f[r];
        }
        /* accumulate into row i_mode of the output */
        double *o = out + (int64_t)coords[(int64_t)mode * nnz + e] * rank;
        for (int r = 0; r < rank; ++r)
            o[r] += row[r];
    }
    free(row);
    return 0;
}

/*
 * The same definition with FP64 values (the paper's precision, Section IV-A:
 * FP64 values and factors).  Identical loops; only the value type differs.
 */
int oracle_mttkrp_f64vals(int nmodes, const int64_t *dims, int64_t nnz,
                          const uint32_t *coords, const double *vals,
                          const double *const *factors, int rank, int mode,
                          double *out)
{
    if (nmodes < 1 || mode < 0 || mode >= nmodes || rank < 1)
        return -1;
    memset(out, 0, sizeof(double) * (size_t)dims[mode] * (size_t)rank);
    double *row = (double *)malloc(sizeof(double) * (size_t)rank);
    if (!row)
        return -2;
    for (int64_t e = 0; e < nnz; ++e) {
        for (int r = 0; r < rank; ++r)
            row[r] = vals[e];
        for (int k = 0; k < nmodes; ++k) {
            if (k == mode)
                continue;
            const double *f = factors[k] + (int64_t)coords[(int64_t)k * nnz + e] * rank;
            for (int r = 0; r < rank; ++r)
                row[r] *= f[r];
        }
        double *o = out + (int64_t)coords[(int64_t)mode * nnz + e] * rank;
        for (int r = 0; r < rank; ++r)
            o[r] += row[r];
    }
    free(row);
    return 0;
}
