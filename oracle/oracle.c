/*
 * oracle.c -- plain, slow FP64 CPU reference for the TCUDB join-aggregate
 * operator (Hu, Li, Tseng, "TCUDB: Accelerating Database with Tensor
 * Processors", SIGMOD 2022).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker, not the product: only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it.  It shares no code, header, table or helper with the HIP library.
 *
 * What it computes is the SQL definition of the operator, not the matrix
 * method.  For relation A with records (group g, key k, value v) and relation B
 * with records (key k, group h, value w), the operator of Section 3.3
 * (group-by aggregate over a join, Lemma Q3) in the form of the matrix
 * multiplication query of Section 2.3 / Fig. "matrix multiplication query" is
 *
 *     C[g,h] = sum over pairs (a in A, b in B) with a.key == b.key,
 *              a.group == g, b.group == h  of  a.val * b.val      (bag semantics)
 *
 * evaluated here as a hash join: B is bucketed by key, and every A record is
 * paired with every B record of its bucket.  Every sum is accumulated with the
 * compensated dot product Dot2 of Ogita, Rump and Oishi ("Accurate sum and dot
 * product", SIAM J. Sci. Comput. 26(6), 2005): TwoProduct through an FMA plus
 * Knuth's TwoSum, so the oracle's own error is about one rounding of the result
 * plus a term of order (n u)^2 sum |a.val * b.val|.
 *
 * Records whose key or group falls outside [0,K) x [0,M) (resp. [0,K) x [0,N))
 * take part in nothing: they are the records the operator skips and reports.
 * A NULL value column stands for COUNT (every value is 1), Section 3.3.
 *
 * Build: gcc -O2 -std=c11 -fopenmp -fPIC -shared -ffp-contract=off.
 * -ffp-contract=off is required: a contracted a*b+c inside TwoSum/TwoProduct
 * would break the error-free transformations.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* ---------------------------------------------------------------- Dot2 --- */

typedef struct { double hi, lo; } acc2;

/* Knuth's TwoSum: s + e == a + b exactly. */
static inline void two_sum(double a, double b, double *s, double *e) {
    double x = a + b;
    double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

/* TwoProduct with an FMA: p + e == a * b exactly (barring underflow). */
static inline void two_prod(double a, double b, double *p, double *e) {
    double x = a * b;
    *e = fma(a, b, -x);
    *p = x;
}

static inline void acc2_add(acc2 *acc, double a, double b) {
    double p, ep, s, es;
    two_prod(a, b, &p, &ep);
    two_sum(acc->hi, p, &s, &es);
    acc->hi = s;
    acc->lo += es + ep;
}

static inline double acc2_value(acc2 a) { return a.hi + a.lo; }

/* ------------------------------------------------------------- buckets --- */

static inline int in_range(int32_t x, int32_t n) { return x >= 0 && x < n; }

/*
 * Stable counting sort of the valid records of a relation by `primary`.
 * A record is valid when primary in [0,np) and secondary in [0,ns).
 * On return off[0..np] are bucket offsets into order[], which lists record
 * indices in increasing index order inside each bucket.  If `secondary_sorted`
 * is set, each bucket is additionally ordered by the secondary column
 * (stable), which the per-cell queries use for binary search.
 */
static int bucket_records(int64_t n, const int32_t *primary, int32_t np,
                          const int32_t *secondary, int32_t ns,
                          int secondary_sorted, int64_t **off_out, int64_t **order_out) {
    int64_t *off = (int64_t *)calloc((size_t)np + 1, sizeof(int64_t));
    int64_t *order = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!off || !order) { free(off); free(order); return -1; }
    for (int64_t i = 0; i < n; ++i)
        if (in_range(primary[i], np) && in_range(secondary[i], ns)) off[primary[i] + 1]++;
    for (int32_t b = 0; b < np; ++b) off[b + 1] += off[b];
    if (!secondary_sorted) {
        int64_t *pos = (int64_t *)malloc((size_t)np * sizeof(int64_t));
        if (!pos) { free(off); free(order); return -1; }
        memcpy(pos, off, (size_t)np * sizeof(int64_t));
        for (int64_t i = 0; i < n; ++i)
            if (in_range(primary[i], np) && in_range(secondary[i], ns)) order[pos[primary[i]]++] = i;
        free(pos);
    } else {
        /* first a stable sort by secondary, then a stable sort by primary */
        int64_t *soff = (int64_t *)calloc((size_t)ns + 1, sizeof(int64_t));
        int64_t *tmp = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
        int64_t *pos = (int64_t *)malloc((size_t)(np > ns ? np : ns) * sizeof(int64_t));
        if (!soff || !tmp || !pos) { free(soff); free(tmp); free(pos); free(off); free(order); return -1; }
        for (int64_t i = 0; i < n; ++i)
            if (in_range(primary[i], np) && in_range(secondary[i], ns)) soff[secondary[i] + 1]++;
        for (int32_t b = 0; b < ns; ++b) soff[b + 1] += soff[b];
        memcpy(pos, soff, (size_t)ns * sizeof(int64_t));
        for (int64_t i = 0; i < n; ++i)
            if (in_range(primary[i], np) && in_range(secondary[i], ns)) tmp[pos[secondary[i]]++] = i;
        memcpy(pos, off, (size_t)np * sizeof(int64_t));
        int64_t nvalid = off[np];
        for (int64_t t = 0; t < nvalid; ++t) {
            int64_t i = tmp[t];
            order[pos[primary[i]]++] = i;
        }
        free(soff); free(tmp); free(pos);
    }
    *off_out = off;
    *order_out = order;
    return 0;
}

static inline double value_of(const double *val, int64_t i) { return val ? val[i] : 1.0; }

static int set_threads(int nthreads) {
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int used = 1;
#pragma omp parallel
    {
#pragma omp single
        used = omp_get_num_threads();
    }
    return used;
}

/* -------------------------------------------------------------- encode --- */

/*
 * Value-filled encoding of one relation into a dense R x Ccols row-major
 * matrix (Section 3.1 for 0/1 entries, Section 3.3 for value entries):
 * out[row, col] = sum of val over the records with that (row, col).
 * Duplicate coordinates add up (bag semantics); the sum runs in record order.
 * Returns the number of records skipped because a coordinate is out of range.
 */
int64_t orc_encode(int64_t n, const int32_t *row, const int32_t *col, const double *val,
                   int32_t R, int32_t Ccols, double *out) {
    memset(out, 0, (size_t)R * (size_t)Ccols * sizeof(double));
    int64_t skipped = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!in_range(row[i], R) || !in_range(col[i], Ccols)) { skipped++; continue; }
        out[(int64_t)row[i] * Ccols + col[i]] += value_of(val, i);
    }
    return skipped;
}

/* ------------------------------------------------------------- forward --- */

/*
 * C for a set of groups g of A (all of [0,M) when rows == NULL):
 *   C[r, h] = sum_{a: a.group == rows[r]} sum_{b: b.key == a.key, b.group == h} a.val * b.val
 *   cnt[r, h] = number of such pairs (optional, exact).
 * C (and cnt) are nrows x N row-major (M x N when rows == NULL).
 * Returns the number of OpenMP threads used, or -1 on allocation failure.
 */
int orc_join_agg_rows(int64_t nA, const int32_t *ag, const int32_t *ak, const double *av,
                      int64_t nB, const int32_t *bk, const int32_t *bh, const double *bw,
                      int32_t M, int32_t K, int32_t N,
                      int64_t nrows, const int32_t *rows, double *C, int64_t *cnt, int nthreads) {
    int used = set_threads(nthreads);
    int64_t *boff, *border, *aoff, *aorder;
    if (bucket_records(nB, bk, K, bh, N, 0, &boff, &border)) return -1;
    if (bucket_records(nA, ag, M, ak, K, 0, &aoff, &aorder)) { free(boff); free(border); return -1; }
    int64_t R = rows ? nrows : M;
    int failed = 0;
#pragma omp parallel
    {
        acc2 *acc = (acc2 *)malloc((size_t)N * sizeof(acc2));
        int64_t *pc = (int64_t *)malloc((size_t)N * sizeof(int64_t));
        if (!acc || !pc) {
#pragma omp atomic write
            failed = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t r = 0; r < R; ++r) {
                int32_t g = rows ? rows[r] : (int32_t)r;
                memset(acc, 0, (size_t)N * sizeof(acc2));
                memset(pc, 0, (size_t)N * sizeof(int64_t));
                if (in_range(g, M)) {
                    for (int64_t t = aoff[g]; t < aoff[g + 1]; ++t) {
                        int64_t i = aorder[t];
                        double v = value_of(av, i);
                        int32_t k = ak[i];
                        for (int64_t u = boff[k]; u < boff[k + 1]; ++u) {
                            int64_t j = border[u];
                            acc2_add(&acc[bh[j]], v, value_of(bw, j));
                            pc[bh[j]]++;
                        }
                    }
                }
                for (int32_t h = 0; h < N; ++h) {
                    C[r * N + h] = acc2_value(acc[h]);
                    if (cnt) cnt[r * N + h] = pc[h];
                }
            }
        }
        free(acc);
        free(pc);
    }
    free(boff); free(border); free(aoff); free(aorder);
    return failed ? -1 : used;
}

/*
 * C and the pair count at individual cells (cg[c], ch[c]): the same sum as
 * above restricted to one (g, h).  B is bucketed by key and ordered by group
 * inside each bucket, so each A record finds its partners with a binary search.
 * Cells outside [0,M) x [0,N) give 0.
 */
int orc_join_agg_cells(int64_t nA, const int32_t *ag, const int32_t *ak, const double *av,
                       int64_t nB, const int32_t *bk, const int32_t *bh, const double *bw,
                       int32_t M, int32_t K, int32_t N,
                       int64_t ncells, const int32_t *cg, const int32_t *ch,
                       double *out, int64_t *cnt, int nthreads) {
    int used = set_threads(nthreads);
    int64_t *boff, *border, *aoff, *aorder;
    if (bucket_records(nB, bk, K, bh, N, 1, &boff, &border)) return -1;
    if (bucket_records(nA, ag, M, ak, K, 0, &aoff, &aorder)) { free(boff); free(border); return -1; }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t c = 0; c < ncells; ++c) {
        int32_t g = cg[c], h = ch[c];
        acc2 acc = {0.0, 0.0};
        int64_t pairs = 0;
        if (in_range(g, M) && in_range(h, N)) {
            for (int64_t t = aoff[g]; t < aoff[g + 1]; ++t) {
                int64_t i = aorder[t];
                int32_t k = ak[i];
                /* lower bound of group h inside bucket k */
                int64_t lo = boff[k], hi = boff[k + 1];
                while (lo < hi) {
                    int64_t mid = lo + (hi - lo) / 2;
                    if (bh[border[mid]] < h) lo = mid + 1; else hi = mid;
                }
                for (int64_t u = lo; u < boff[k + 1] && bh[border[u]] == h; ++u) {
                    acc2_add(&acc, value_of(av, i), value_of(bw, border[u]));
                    pairs++;
                }
            }
        }
        out[c] = acc2_value(acc);
        if (cnt) cnt[c] = pairs;
    }
    free(boff); free(border); free(aoff); free(aorder);
    return used;
}

/*
 * Right-hand side of Freivalds' check: out[g] = sum_h C[g,h] r[h], evaluated
 * from the records in O(nA + nB) by regrouping the defining double sum
 * (distributivity):
 *   t[k]   = sum_{b: b.key == k} b.val * r[b.group]
 *   out[g] = sum_{a: a.group == g} a.val * t[a.key]
 * (R. Freivalds, "Probabilistic machines can use less running time", IFIP 1977.)
 * Both sums stream over the records: a fixed number of record chunks keep
 * Dot2 partial sums per key (per group), which are then combined in chunk
 * order with TwoSum, so the result does not depend on the thread count and
 * no relation-sized buffer is allocated.
 */
#define ORC_CHUNKS 64

static int stream_dot2(int64_t n, const int32_t *idx, int32_t nidx, const int32_t *other,
                       int32_t nother, const double *val, const double *factor_by_other,
                       const int32_t *factor_index, double *out) {
    /* out[idx[i]] = sum_i val[i] * factor_by_other[factor_index[i]] over valid i */
    acc2 *part = (acc2 *)calloc((size_t)ORC_CHUNKS * (size_t)nidx, sizeof(acc2));
    if (!part) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < ORC_CHUNKS; ++c) {
        const int64_t i0 = n * c / ORC_CHUNKS, i1 = n * (c + 1) / ORC_CHUNKS;
        acc2 *pc = part + (size_t)c * nidx;
        for (int64_t i = i0; i < i1; ++i) {
            if (!in_range(idx[i], nidx) || !in_range(other[i], nother)) continue;
            acc2_add(&pc[idx[i]], value_of(val, i), factor_by_other[factor_index[i]]);
        }
    }
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < nidx; ++j) {
        acc2 tot = {0.0, 0.0};
        for (int c = 0; c < ORC_CHUNKS; ++c) {
            const acc2 pc = part[(size_t)c * nidx + j];
            double s, e;
            two_sum(tot.hi, pc.hi, &s, &e);
            tot.hi = s;
            tot.lo += e + pc.lo;
        }
        out[j] = acc2_value(tot);
    }
    free(part);
    return 0;
}

int orc_freivalds(int64_t nA, const int32_t *ag, const int32_t *ak, const double *av,
                  int64_t nB, const int32_t *bk, const int32_t *bh, const double *bw,
                  int32_t M, int32_t K, int32_t N, const double *r, double *out, int nthreads) {
    int used = set_threads(nthreads);
    double *t = (double *)malloc((size_t)K * sizeof(double));
    if (!t) return -1;
    /* t[k] over B: index = key, factor r[group]; out[g] over A: index = group, factor t[key] */
    int bad = stream_dot2(nB, bk, K, bh, N, bw, r, bh, t);
    if (!bad) bad = stream_dot2(nA, ag, M, ak, K, av, t, ak, out);
    free(t);
    return bad ? -1 : used;
}

/* ------------------------------------------------------------ gradient --- */

/*
 * Gradient of L = sum_{g,h} W[g,h] C[g,h] with respect to the value columns,
 * by differentiating the defining sum term by term:
 *   dL/d a_i.val = sum_{b: b.key == a_i.key} W[a_i.group, b.group] * b.val
 *   dL/d b_j.val = sum_{a: a.key == b_j.key} W[a.group, b_j.group] * a.val
 * For records idx[0..nidx) of the chosen relation (all records when idx ==
 * NULL).  which == 0 selects A, which == 1 selects B.  Records that take part
 * in nothing (out-of-range coordinates) get 0.
 */
int orc_grad(int64_t nA, const int32_t *ag, const int32_t *ak, const double *av,
             int64_t nB, const int32_t *bk, const int32_t *bh, const double *bw,
             int32_t M, int32_t K, int32_t N, const double *W,
             int which, int64_t nidx, const int64_t *idx, double *out, int nthreads) {
    int used = set_threads(nthreads);
    int64_t *off, *order;
    if (which == 0) {
        if (bucket_records(nB, bk, K, bh, N, 0, &off, &order)) return -1;
        int64_t R = idx ? nidx : nA;
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t r = 0; r < R; ++r) {
            int64_t i = idx ? idx[r] : r;
            acc2 acc = {0.0, 0.0};
            if (i >= 0 && i < nA && in_range(ag[i], M) && in_range(ak[i], K)) {
                int32_t k = ak[i];
                const double *wrow = W + (int64_t)ag[i] * N;
                for (int64_t u = off[k]; u < off[k + 1]; ++u) {
                    int64_t j = order[u];
                    acc2_add(&acc, wrow[bh[j]], value_of(bw, j));
                }
            }
            out[r] = acc2_value(acc);
        }
    } else {
        if (bucket_records(nA, ak, K, ag, M, 0, &off, &order)) return -1;
        int64_t R = idx ? nidx : nB;
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t r = 0; r < R; ++r) {
            int64_t j = idx ? idx[r] : r;
            acc2 acc = {0.0, 0.0};
            if (j >= 0 && j < nB && in_range(bk[j], K) && in_range(bh[j], N)) {
                int32_t k = bk[j], h = bh[j];
                for (int64_t u = off[k]; u < off[k + 1]; ++u) {
                    int64_t i = order[u];
                    acc2_add(&acc, W[(int64_t)ag[i] * N + h], value_of(av, i));
                }
            }
            out[r] = acc2_value(acc);
        }
    }
    free(off); free(order);
    return used;
}

/* --------------------------------------------------------------- split --- */

/*
 * Fixed-point slicing of a dense R x L row-major matrix, used by the
 * mixed-precision form of the contraction (the paper's feasibility test of
 * Section 4.2.1 picks a narrow matrix-unit type from per-column min/max
 * metadata; the mixed form generalises that to several narrow slices).
 *
 * axis == 0: one scale per row; axis == 1: one scale per column.  For a line
 * (row or column) with largest magnitude mx:
 *   e = the exponent with 2^(e-1) <= mx < 2^e   (e = 0 when mx == 0),
 *   r_0 = x / 2^e  (so |r_0| < 1),
 *   for p = 1..nslices:  t = r_{p-1} * 2^bits,  d_p = trunc(t),  r_p = t - d_p,
 * so that x = 2^e * (sum_p d_p 2^(-bits p) + r_s 2^(-bits s)) exactly, every
 * d_p an integer with |d_p| < 2^bits and the sign of x.  Every step is exact in
 * FP64 (power-of-two scalings and the removal of an integer part).
 * slices[p][row][col] holds d_(p+1); exps[line] holds e.
 * Returns 0, or the 1-based index of the first line holding a NaN or infinity
 * (that line's outputs are then undefined).
 */
int64_t orc_split(int32_t R, int32_t L, const double *X, int axis, int nslices, int bits,
                  int32_t *exps, double *slices) {
    int64_t nlines = axis == 0 ? R : L;
    int64_t len = axis == 0 ? L : R;
    int64_t bad = 0;
    for (int64_t line = 0; line < nlines; ++line) {
        double mx = 0.0;
        for (int64_t t = 0; t < len; ++t) {
            double x = axis == 0 ? X[line * L + t] : X[t * L + line];
            if (!isfinite(x)) { if (!bad) bad = line + 1; mx = 0.0; break; }
            if (fabs(x) > mx) mx = fabs(x);
        }
        int e = 0;
        if (mx > 0.0) frexp(mx, &e);
        exps[line] = e;
        for (int64_t t = 0; t < len; ++t) {
            int64_t at = axis == 0 ? line * L + t : t * L + line;
            double r = ldexp(X[at], -e);
            for (int p = 0; p < nslices; ++p) {
                double tt = ldexp(r, bits);
                double d = trunc(tt);
                slices[(int64_t)p * R * L + at] = d;
                r = tt - d;
            }
        }
    }
    return bad;
}

/* ---------------------------------------------------------- dictionary --- */

static int cmp_i64(const void *x, const void *y) {
    const int64_t a = *(const int64_t *)x, b = *(const int64_t *)y;
    return (a > b) - (a < b);
}

static int32_t rank_of(const int64_t *dict, int64_t k, int64_t v) {
    int64_t lo = 0, hi = k;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (dict[mid] < v) lo = mid + 1; else hi = mid;
    }
    return (int32_t)lo;
}

/*
 * dom(ID) of Section 3.1: the union of two columns' values, sorted, with
 * duplicates removed (dict[0..k)); every value's code is its 0-based rank.
 * Returns k, or -1 on allocation failure.
 */
int64_t orc_dict(int64_t na, const int64_t *a, int64_t nb, const int64_t *b, int32_t *ca,
                 int32_t *cb, int64_t *dict) {
    int64_t n = na + nb;
    int64_t *all = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!all) return -1;
    memcpy(all, a, (size_t)na * sizeof(int64_t));
    memcpy(all + na, b, (size_t)nb * sizeof(int64_t));
    qsort(all, (size_t)n, sizeof(int64_t), cmp_i64);
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i)
        if (k == 0 || all[i] != dict[k - 1]) dict[k++] = all[i];
    free(all);
    for (int64_t i = 0; i < na; ++i) ca[i] = rank_of(dict, k, a[i]);
    for (int64_t i = 0; i < nb; ++i) cb[i] = rank_of(dict, k, b[i]);
    return k;
}

/*
 * The product of integer truncations, the quantity the CRT mixed form
 * computes exactly before its final scaling (the error model of that form:
 * Section 4.2.1's feasibility bound, retargeted, as for orc_split).
 *
 * X is M x K and Y is K x N, row-major FP64.  Every row g of X gets
 *   e_g = the exponent with 2^(e_g - 1) <= max_k |X[g,k]| < 2^e_g (0 if zero),
 *   Xi[g,k] = trunc(X[g,k] * 2^(bits - e_g))            (|Xi| < 2^bits),
 * every column h of Y likewise f_h and Yi[k,h]; then
 *   out[g,h] = (sum_k Xi[g,k] Yi[k,h]) * 2^(e_g + f_h - 2 bits)
 * with the sum exact in 128-bit integers and one rounding to FP64 at the end
 * (the scaling by a power of two is exact).  bits in [1, 53]; non-finite
 * inputs give -1 (returned), else the number of threads used.
 */
int orc_trunc_product(int32_t M, int32_t K, int32_t N, const double *X, const double *Y, int bits,
                      double *out, int threads) {
    if (bits < 1 || bits > 53) return -1;
    int *ex = (int *)malloc(sizeof(int) * (size_t)(M > 0 ? M : 1));
    int *ey = (int *)malloc(sizeof(int) * (size_t)(N > 0 ? N : 1));
    int64_t *xi = (int64_t *)malloc(sizeof(int64_t) * ((size_t)M * (size_t)K + 1));
    int64_t *yt = (int64_t *)malloc(sizeof(int64_t) * ((size_t)K * (size_t)N + 1));
    if (!ex || !ey || !xi || !yt) {
        free(ex); free(ey); free(xi); free(yt);
        return -2;
    }
    int bad = 0;
    for (int32_t g = 0; g < M; ++g) {
        double mx = 0.0;
        for (int32_t k = 0; k < K; ++k) {
            const double v = X[(size_t)g * K + k];
            if (!isfinite(v)) bad = 1;
            else if (fabs(v) > mx) mx = fabs(v);
        }
        int e = 0;
        if (mx > 0.0) frexp(mx, &e);
        ex[g] = e;
        for (int32_t k = 0; k < K; ++k)
            xi[(size_t)g * K + k] = (int64_t)trunc(ldexp(X[(size_t)g * K + k], bits - e));
    }
    for (int32_t h = 0; h < N; ++h) {
        double mx = 0.0;
        for (int32_t k = 0; k < K; ++k) {
            const double v = Y[(size_t)k * N + h];
            if (!isfinite(v)) bad = 1;
            else if (fabs(v) > mx) mx = fabs(v);
        }
        int f = 0;
        if (mx > 0.0) frexp(mx, &f);
        ey[h] = f;
        /* column h of Y, transposed so the inner loop runs over contiguous k */
        for (int32_t k = 0; k < K; ++k)
            yt[(size_t)h * K + k] = (int64_t)trunc(ldexp(Y[(size_t)k * N + h], bits - f));
    }
    if (bad) {
        free(ex); free(ey); free(xi); free(yt);
        return -1;
    }
    int used = 1;
#pragma omp parallel num_threads(threads)
    {
#pragma omp single
        used = omp_get_num_threads();
#pragma omp for schedule(dynamic, 4)
        for (int32_t g = 0; g < M; ++g) {
            const int64_t *a = xi + (size_t)g * K;
            for (int32_t h = 0; h < N; ++h) {
                const int64_t *b = yt + (size_t)h * K;
                __int128 p = 0;
                for (int32_t k = 0; k < K; ++k) p += (__int128)a[k] * (__int128)b[k];
                out[(size_t)g * N + h] = ldexp((double)p, ex[g] + ey[h] - 2 * bits);
            }
        }
    }
    free(ex); free(ey); free(xi); free(yt);
    return used;
}

/*
 * The certificate of a mixed-form product C = X Y: the plan of step a0
 * (Section 4.2.1's feasibility test, which reads the operands' magnitudes to
 * choose the narrow type, retargeted), written from its definition and
 * without the rounding margins a device evaluation adds.
 * X is M x K and Y is K x N, row-major FP64.  Per line (row g of X, column h
 * of Y):
 *   e = the exponent with 2^(e - 1) <= max |z| < 2^e (0 for a zero line),
 *   q = floor(|z| 2^(7 - e)) for every entry, 0 <= q <= 127,
 *   s = sum over the line of |z| 2^-e (compensated sum, one final rounding);
 * per cell:
 *   T[g,h] = sum_k qX[g,k] qY[k,h] (exact), r = 2^14 (s_g + s_h), or r = 0
 *   when s_g or s_h is 0 (an all-zero line: every term of the cell is 0).
 * need_bits = max over cells of the smallest b >= 1 with r <= 2^b tcrt T,
 * need_slices = max over cells of the smallest S in 1..8 with
 *   r + (S - 1) 2^14 K <= 2^(7S) tdig[S] T  (255 when no S meets it);
 * a cell with T = 0 needs 0 when r = 0 and 255 of each otherwise.
 * umax[0], umax[1]: the largest s over the rows of X and the columns of Y.
 * T_out (M x N) and s_out (M + N: rows, then columns) may be NULL.
 * Returns -1 for non-finite inputs, else the number of threads used.
 */
static double line_sum_scaled(const double *z, int64_t n, int64_t stride, int e) {
    double hi = 0.0, lo = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double s, err;
        two_sum(hi, fabs(z[i * stride]), &s, &err);
        hi = s;
        lo += err;
    }
    return ldexp(hi + lo, -e);
}

static int line_exponent_of(const double *z, int64_t n, int64_t stride, int *bad) {
    double mx = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double v = z[i * stride];
        if (!isfinite(v)) *bad = 1;
        else if (fabs(v) > mx) mx = fabs(v);
    }
    int e = 0;
    if (mx > 0.0) frexp(mx, &e);
    return e;
}

int orc_certificate(int32_t M, int32_t K, int32_t N, const double *X, const double *Y,
                    double tcrt, const double *tdig, uint32_t *need_bits, uint32_t *need_slices,
                    double *umax, int64_t *T_out, double *s_out, int threads) {
    int *ex = (int *)malloc(sizeof(int) * (size_t)(M > 0 ? M : 1));
    int *ey = (int *)malloc(sizeof(int) * (size_t)(N > 0 ? N : 1));
    double *sx = (double *)malloc(sizeof(double) * (size_t)(M > 0 ? M : 1));
    double *sy = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    int32_t *qx = (int32_t *)malloc(sizeof(int32_t) * ((size_t)M * (size_t)K + 1));
    int32_t *qyt = (int32_t *)malloc(sizeof(int32_t) * ((size_t)K * (size_t)N + 1));
    if (!ex || !ey || !sx || !sy || !qx || !qyt) {
        free(ex); free(ey); free(sx); free(sy); free(qx); free(qyt);
        return -2;
    }
    int bad = 0;
    umax[0] = umax[1] = 0.0;
    for (int32_t g = 0; g < M; ++g) {
        const double *row = X + (size_t)g * K;
        ex[g] = line_exponent_of(row, K, 1, &bad);
        sx[g] = line_sum_scaled(row, K, 1, ex[g]);
        if (sx[g] > umax[0]) umax[0] = sx[g];
        for (int32_t k = 0; k < K; ++k)
            qx[(size_t)g * K + k] = (int32_t)floor(ldexp(fabs(row[k]), 7 - ex[g]));
    }
    for (int32_t h = 0; h < N; ++h) {
        ey[h] = line_exponent_of(Y + h, K, N, &bad);
        sy[h] = line_sum_scaled(Y + h, K, N, ey[h]);
        if (sy[h] > umax[1]) umax[1] = sy[h];
        for (int32_t k = 0; k < K; ++k)
            qyt[(size_t)h * K + k] = (int32_t)floor(ldexp(fabs(Y[(size_t)k * N + h]), 7 - ey[h]));
    }
    if (bad) {
        free(ex); free(ey); free(sx); free(sy); free(qx); free(qyt);
        return -1;
    }
    if (s_out != NULL) {
        memcpy(s_out, sx, sizeof(double) * (size_t)M);
        memcpy(s_out + M, sy, sizeof(double) * (size_t)N);
    }
    uint32_t nb = 0, ns = 0;
    int used = 1;
#pragma omp parallel num_threads(threads) reduction(max : nb, ns)
    {
#pragma omp single
        used = omp_get_num_threads();
#pragma omp for schedule(dynamic, 4)
        for (int32_t g = 0; g < M; ++g) {
            for (int32_t h = 0; h < N; ++h) {
                int64_t T = 0;
                for (int32_t k = 0; k < K; ++k)
                    T += (int64_t)qx[(size_t)g * K + k] * (int64_t)qyt[(size_t)h * K + k];
                if (T_out != NULL) T_out[(size_t)g * N + h] = T;
                const long double r = (sx[g] > 0.0 && sy[h] > 0.0)
                                          ? 16384.0L * ((long double)sx[g] + (long double)sy[h])
                                          : 0.0L;
                uint32_t cb, cs;
                if (T == 0) {
                    cb = cs = r > 0.0L ? 255u : 0u;
                } else {
                    const long double tT = (long double)tcrt * (long double)T;
                    cb = 1;
                    while (cb < 254 && r > ldexpl(tT, (int)cb)) ++cb;
                    cs = 255;
                    for (int S = 1; S <= 8; ++S) {
                        const long double lhs = r + (long double)(S - 1) * 16384.0L * K;
                        if (lhs <= ldexpl((long double)tdig[S] * (long double)T, 7 * S)) {
                            cs = (uint32_t)S;
                            break;
                        }
                    }
                }
                if (cb > nb) nb = cb;
                if (cs > ns) ns = cs;
            }
        }
    }
    *need_bits = nb;
    *need_slices = ns;
    free(ex); free(ey); free(sx); free(sy); free(qx); free(qyt);
    return used;
}
