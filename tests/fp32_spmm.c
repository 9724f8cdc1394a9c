/* Test helper for the CGLS rounding envelopes: a CSR matrix times a batch
 * of vectors in FP32 arithmetic, each row summed with one fused multiply-add
 * per entry (one correct FP32 implementation of the product, for comparison
 * with the GPU's, which sums in another order).  `order` picks the summation
 * order: 0 the stored order; otherwise each row's entries are taken
 * cyclically from a start drawn from (row, order) by a hash, forwards for odd
 * `order` and backwards for even.
 *   out[b][r] = sum over n in [ptr[r], ptr[r+1]) of val[n] * x[b][idx[n]]
 */
#include <math.h>
#include <stdint.h>

static uint64_t mix(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

void fp32_csr_spmm(int64_t nrows, const int64_t *ptr, const int32_t *idx, const float *val, int64_t ncols,
                   int batch, const float *x, float *out, int64_t order)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t n0 = ptr[r], len = ptr[r + 1] - ptr[r];
        const int64_t start = (order && len) ? (int64_t)(mix((uint64_t)r * 0x100000001b3ull ^ (uint64_t)order) %
                                                        (uint64_t)len)
                                            : 0;
        const int64_t step = (order & 1) || !order ? 1 : len - 1;  /* len - 1 == -1 modulo len */
        for (int b = 0; b < batch; ++b) {
            const float *xb = x + (int64_t)b * ncols;
            float acc = 0.0f;
            int64_t j = start;
            for (int64_t t = 0; t < len; ++t) {
                const int64_t n = n0 + j;
                acc = fmaf(val[n], xb[idx[n]], acc);
                j += step;
                if (j >= len) j -= len;
            }
            out[(int64_t)b * nrows + r] = acc;
        }
    }
}
