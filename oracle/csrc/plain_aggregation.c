/* Oracle helper (TEST INFRASTRUCTURE ONLY): the three aggregation passes of
 * oracle/_aggregate.py:aggregate_py transcribed to C for large graphs.
 * Plain aggregation, Vanek, Mandel & Brezina (1996); see that module for the
 * statement of the passes.  Not part of the GPU library, which has its own
 * independent implementation. */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int64_t oracle_plain_aggregation(int64_t n, const int64_t *ptr, const int64_t *col,
                                 const double *w, const uint8_t *strong, int64_t *agg)
{
    int64_t nagg = 0;
    for (int64_t i = 0; i < n; ++i) agg[i] = -1;

    /* pass 1 */
    for (int64_t i = 0; i < n; ++i) {
        if (agg[i] != -1) continue;
        int has = 0, all_free = 1;
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
            if (!strong[k]) continue;
            has = 1;
            if (agg[col[k]] != -1) { all_free = 0; break; }
        }
        if (!has || !all_free) continue;
        agg[i] = nagg;
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k)
            if (strong[k]) agg[col[k]] = nagg;
        ++nagg;
    }

    /* pass 2, against the pass-1 snapshot */
    int64_t *snap = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!snap) return -1;
    memcpy(snap, agg, (size_t)n * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        if (snap[i] != -1) continue;
        int64_t best = -1;
        double bestw = 0.0;
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
            if (!strong[k]) continue;
            int64_t j = col[k];
            if (snap[j] != -1 && (best < 0 || w[k] > bestw)) { best = j; bestw = w[k]; }
        }
        if (best >= 0) agg[i] = snap[best];
    }
    free(snap);

    /* pass 3 */
    for (int64_t i = 0; i < n; ++i) {
        if (agg[i] != -1) continue;
        int has = 0;
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k)
            if (strong[k]) { has = 1; break; }
        if (!has) continue;
        agg[i] = nagg;
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k)
            if (strong[k] && agg[col[k]] == -1) agg[col[k]] = nagg;
        ++nagg;
    }
    return nagg;
}
