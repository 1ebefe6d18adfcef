/* Runs the C oracle's entry points on graphs read from a binary file, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer.  Input file:
 *   int32 n, int64 nnz, int32 weighted, double alpha, uint64 seed,
 *   uint32 stream, uint32 t_begin, uint32 count,
 *   int32 row_ptr[n+1], int32 col_idx[nnz], (weighted) double weights[nnz]
 * Output (text): one line per tree "digest steps roots", then "R <sum of R>",
 * "visits <sum>", "parents <sum of parents>", "est <sum of diag bits>". */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_sample_w(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                 const double *weights, double alpha, uint64_t seed, uint32_t stream,
                 uint32_t t_begin, uint32_t count, const int32_t *order, uint32_t *R,
                 uint64_t *visits, int32_t *parents, uint32_t *tree_visits, uint64_t *digests,
                 uint64_t *steps, uint32_t *roots);
void orc_estimate(int32_t n, const uint32_t *R, uint32_t tau, int literal, double *diag,
                  double *farness, double *closeness);
uint32_t orc_tau(int64_t m, int64_t n, double eps, double delta, double kappa);

static void *must(size_t bytes) {
    void *p = calloc(bytes ? bytes : 1, 1);
    if (!p) exit(3);
    return p;
}

int main(int argc, char **argv) {
    if (argc != 2) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t n, weighted;
    int64_t nnz;
    double alpha;
    uint64_t seed;
    uint32_t stream, t0, count;
    if (fread(&n, 4, 1, f) != 1 || fread(&nnz, 8, 1, f) != 1 || fread(&weighted, 4, 1, f) != 1 ||
        fread(&alpha, 8, 1, f) != 1 || fread(&seed, 8, 1, f) != 1 || fread(&stream, 4, 1, f) != 1 ||
        fread(&t0, 4, 1, f) != 1 || fread(&count, 4, 1, f) != 1)
        return 2;
    int32_t *rp = must(4u * ((size_t)n + 1));
    int32_t *ci = must(4u * (size_t)nnz);
    double *w = weighted ? must(8u * (size_t)nnz) : NULL;
    if (fread(rp, 4, (size_t)n + 1, f) != (size_t)n + 1) return 2;
    if (nnz && fread(ci, 4, (size_t)nnz, f) != (size_t)nnz) return 2;
    if (w && nnz && fread(w, 8, (size_t)nnz, f) != (size_t)nnz) return 2;
    fclose(f);
    uint32_t *R = must(4u * (size_t)n);
    uint64_t *visits = must(8u * (size_t)n);
    int32_t *parents = must(4u * (size_t)n * count);
    uint32_t *tvis = must(4u * (size_t)n * count);
    uint64_t *dig = must(8u * count), *steps = must(8u * count);
    uint32_t *roots = must(4u * count);
    if (orc_sample_w(n, rp, ci, w, alpha, seed, stream, t0, count, NULL, R, visits, parents, tvis,
                     dig, steps, roots) != 0)
        return 4;
    for (uint32_t i = 0; i < count; ++i)
        printf("%llu %llu %u\n", (unsigned long long)dig[i], (unsigned long long)steps[i], roots[i]);
    unsigned long long sr = 0, sv = 0, sp = 0, se = 0;
    for (int32_t v = 0; v < n; ++v) {
        sr += R[v];
        sv += visits[v];
    }
    for (size_t i = 0; i < (size_t)n * count; ++i) sp += (unsigned long long)(uint32_t)parents[i];
    double *d = must(8u * (size_t)n), *fa = must(8u * (size_t)n), *cl = must(8u * (size_t)n);
    orc_estimate(n, R, count ? count : 1, 0, d, fa, cl);
    for (int32_t v = 0; v < n; ++v) {
        uint64_t b;
        memcpy(&b, &d[v], 8);
        se += b;
    }
    printf("R %llu\nvisits %llu\nparents %llu\nest %llu\ntau %u\n", sr, sv, sp, se,
           orc_tau(nnz / 2, n, 0.1, 0.1, 0.0));
    free(rp); free(ci); free(w); free(R); free(visits); free(parents); free(tvis);
    free(dig); free(steps); free(roots); free(d); free(fa); free(cl);
    return 0;
}
