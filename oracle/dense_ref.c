/*
 * Brute-force FCS of a dense or COO tensor in plain C, float64 accumulators.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by tests/ and by the CPU-baseline leg of
 * bench.py through ctypes.  The product library never links or calls it.
 *
 * It is the general-tensor formula of Section 3.2 of the paper written out:
 * every element T[i_0..i_{N-1}] is added, with sign S = prod_n s_n(i_n), to
 * bin H = sum_n h_n(i_n) (0-based) of each of the D sketches.  It exists only
 * because the NumPy form of the same loop is too slow and too large in memory
 * for a 2^30-element tensor; tests check it against the NumPy oracle.
 *
 * Layout: T is vec(T), mode 0 fastest.  Hash tables are h[d][off_n + i] and
 * s[d][off_n + i] with off_n = I_0 + ... + I_{n-1}.  out is D x Jt, row-major,
 * and is accumulated into (the caller zeroes it).
 */
#include <stdint.h>

#define ORACLE_MAX_N 16

/* Rows are the fibres along mode 0: row r enumerates (i_1, ..., i_{N-1}) with
 * i_1 fastest.  Only rows [row_begin, row_end) are visited, so a caller can
 * sketch a sample of the tensor; T points at the start of the full tensor. */
int oracle_fcs_dense_rows(int N, const int64_t *I, const float *T, int D,
                          const int32_t *h, const int8_t *s, int64_t Jt,
                          int64_t row_begin, int64_t row_end, double *out)
{
    if (N < 1 || N > ORACLE_MAX_N || D < 1) return 1;
    int64_t off[ORACLE_MAX_N], sumI = 0;
    for (int n = 0; n < N; ++n) { off[n] = sumI; sumI += I[n]; }
    const int64_t I0 = I[0];

    for (int64_t r = row_begin; r < row_end; ++r) {
        /* decode the row index into (i_1, ..., i_{N-1}) */
        int64_t idx[ORACLE_MAX_N], rem = r;
        for (int n = 1; n < N; ++n) { idx[n] = rem % I[n]; rem /= I[n]; }
        const float *row = T + r * I0;
        for (int d = 0; d < D; ++d) {
            const int32_t *hd = h + (int64_t)d * sumI;
            const int8_t *sd = s + (int64_t)d * sumI;
            int64_t c = 0;
            double sign = 1.0;
            for (int n = 1; n < N; ++n) {
                c += hd[off[n] + idx[n]];
                sign *= (double)sd[off[n] + idx[n]];
            }
            double *o = out + (int64_t)d * Jt;
            for (int64_t i0 = 0; i0 < I0; ++i0) {
                int64_t H = c + hd[i0];
                double S = sign * (double)sd[i0];
                o[H] += S * (double)row[i0];
            }
        }
    }
    return 0;
}

/* COO form: coordinate k is (idx[0][k], ..., idx[N-1][k]) with value val[k];
 * idx is stored mode-major, idx[n * nnz + k]. */
int oracle_fcs_coo(int N, const int64_t *I, int64_t nnz, const int32_t *idx,
                   const float *val, int D, const int32_t *h, const int8_t *s,
                   int64_t Jt, double *out)
{
    if (N < 1 || N > ORACLE_MAX_N || D < 1) return 1;
    int64_t off[ORACLE_MAX_N], sumI = 0;
    for (int n = 0; n < N; ++n) { off[n] = sumI; sumI += I[n]; }
    for (int d = 0; d < D; ++d) {
        const int32_t *hd = h + (int64_t)d * sumI;
        const int8_t *sd = s + (int64_t)d * sumI;
        double *o = out + (int64_t)d * Jt;
        for (int64_t k = 0; k < nnz; ++k) {
            int64_t H = 0;
            double S = 1.0;
            for (int n = 0; n < N; ++n) {
                int64_t i = idx[(int64_t)n * nnz + k];
                H += hd[off[n] + i];
                S *= (double)sd[off[n] + i];
            }
            o[H] += S * (double)val[k];
        }
    }
    return 0;
}
