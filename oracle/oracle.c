/*
 * CPU oracle for the neighbourhood-graph step (test infrastructure only).
 *
 * Only the test suite, the package smoke check and the benchmark's CPU
 * baseline leg call this code.  It shares nothing with the HIP library: no
 * headers, helpers or tables.  It is deliberately plain and slow: float64
 * everywhere, brute force, no blocking, no algebraic rewriting.
 *
 * What it computes (the paper's neighbourhood-graph step, Methods:
 * "Dimensionality reduction and graph analysis", which stores the kNN graph
 * and the connectivities built the way scanpy builds them, i.e. the UMAP
 * fuzzy simplicial set; UMAP is the method the Technical architecture
 * section names for the embedding):
 *
 *   knn            exact k nearest neighbours by Euclidean distance, the
 *                  squared distance summed from direct differences
 *                  (Methods, Custom GPU kernels: d_ij = ||x_i - x_j||^2),
 *                  ties broken towards the lower index, the query itself
 *                  forced into slot 0 when queries and references coincide.
 *   smooth_knn     per row: rho = smallest strictly positive neighbour
 *                  distance; sigma > 0 solving
 *                      sum_{j=1..k-1} exp(-max(0, d_ij - rho) / sigma) = log2 k
 *                  by bisection; directed weights
 *                      a_ij = exp(-max(0, d_ij - rho) / sigma).
 *   fuzzy_union    symmetric weights w = a + b - a*b over every pair joined
 *                  by an edge in either direction (a missing direction counts
 *                  as 0), stored as CSR (Methods, Implementation: CSR for
 *                  row-wise access) with ascending unique columns, no
 *                  diagonal, no stored zeros.
 *
 *   edistance_sums the group-pair sums of Euclidean distances behind the
 *                  energy distance (Methods, "Perturbation distance
 *                  computation"); see the function's comment.
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   - k counts the query itself: k slots, slot 0 = self, k-1 neighbours,
 *     target log2(k).
 *   - rows with m >= log2 k slots at distance <= rho have no positive root;
 *     they get sigma = 0 and a = 1 where d <= rho, a = 0 elsewhere.
 *   - bisection: start at sigma = 1 with the bracket (0, inf); double until
 *     the bracket closes above, then halve; stop when |f - log2 k| <=
 *     1e-12 log2 k, when the bracket is below one ulp, or after 200 steps.
 *   - no lower floor on sigma.
 *
 * Compiled with -ffp-contract=off so that every product and sum is rounded
 * on its own, in the order written.
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_ABI 1

int oracle_abi_version(void) { return ORACLE_ABI; }

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Squared Euclidean distance of two float32 rows, in float64, dims in order. */
static double sq_dist(const float *x, const float *y, int d) {
    double s = 0.0;
    for (int t = 0; t < d; ++t) {
        double diff = (double)x[t] - (double)y[t];
        s = s + diff * diff;
    }
    return s;
}

/* (d2, j) lexicographic order: smaller distance first, lower index on ties. */
static int before(double da, int64_t ja, double db, int64_t jb) {
    return da < db || (da == db && ja < jb);
}

/*
 * Exact kNN by brute force.
 *
 * Q: nq x d float32 row-major queries; R: nr x d float32 references.
 * self_ids: NULL, or per query the reference row that is the query itself.
 *   When given (>= 0), that row is excluded from the candidates and placed in
 *   slot 0 with distance 0, and the remaining k-1 slots hold the nearest
 *   other rows.  When NULL (or < 0 for a query) all k slots come from the
 *   references.
 * out_idx: nq x k int32; out_d2: nq x k float64 squared distances (may be
 * NULL); out_dist: nq x k float32 = float32(sqrt(d2)) (may be NULL).
 * Rows are sorted by (d2, index).  Returns 0, or -1 on bad arguments.
 */
int oracle_knn(const float *Q, int64_t nq, const int64_t *self_ids, const float *R, int64_t nr,
               int d, int k, int32_t *out_idx, double *out_d2, float *out_dist) {
    if (nq < 0 || nr < 1 || d < 1 || k < 1 || k > nr) return -1;
    int fail = 0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < nq; ++q) {
        const float *x = Q + q * (int64_t)d;
        int64_t self = self_ids ? self_ids[q] : -1;
        int start = 0;
        double *bd = (double *)malloc(sizeof(double) * (size_t)k);
        int64_t *bj = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
        if (!bd || !bj) {
            fail = 1;
            free(bd);
            free(bj);
            continue;
        }
        if (self >= 0) {
            bd[0] = 0.0;
            bj[0] = self;
            start = 1;
        }
        int cnt = start; /* filled slots; slots [start, cnt) sorted ascending */
        for (int64_t j = 0; j < nr; ++j) {
            if (j == self) continue;
            double v = sq_dist(x, R + j * (int64_t)d, d);
            if (cnt < k) {
                int p = cnt++;
                while (p > start && before(v, j, bd[p - 1], bj[p - 1])) {
                    bd[p] = bd[p - 1];
                    bj[p] = bj[p - 1];
                    --p;
                }
                bd[p] = v;
                bj[p] = j;
            } else if (k > start && before(v, j, bd[k - 1], bj[k - 1])) {
                int p = k - 1;
                while (p > start && before(v, j, bd[p - 1], bj[p - 1])) {
                    bd[p] = bd[p - 1];
                    bj[p] = bj[p - 1];
                    --p;
                }
                bd[p] = v;
                bj[p] = j;
            }
        }
        for (int s = 0; s < k; ++s) {
            int64_t o = q * (int64_t)k + s;
            out_idx[o] = (int32_t)(s < cnt ? bj[s] : -1);
            if (out_d2) out_d2[o] = s < cnt ? bd[s] : INFINITY;
            if (out_dist) out_dist[o] = s < cnt ? (float)sqrt(bd[s]) : INFINITY;
        }
        free(bd);
        free(bj);
    }
    return fail ? -1 : 0;
}

/* Exact squared distances of given (i, j) pairs of one matrix, float64. */
int oracle_pair_d2(const float *X, int64_t n, int d, const int64_t *ii, const int64_t *jj, int64_t m,
                   double *out) {
    for (int64_t p = 0; p < m; ++p) {
        if (ii[p] < 0 || ii[p] >= n || jj[p] < 0 || jj[p] >= n) return -1;
        out[p] = sq_dist(X + ii[p] * (int64_t)d, X + jj[p] * (int64_t)d, d);
    }
    return 0;
}

/* Sum over the k-1 neighbour slots of exp(-max(0, d - rho) / sigma). */
static double membership_sum(const double *dd, int m, double rho, double sigma) {
    double s = 0.0;
    for (int j = 0; j < m; ++j) {
        double g = dd[j] - rho;
        if (g < 0.0) g = 0.0;
        s = s + exp(-g / sigma);
    }
    return s;
}

/*
 * Smooth-kNN calibration of one row (UMAP's local fuzzy set).
 *
 * dd: the k-1 non-self neighbour distances (float64 copies of the float32
 * kNN output).  Writes rho, sigma and the directed weights a[0..k-2]; returns
 * 1 for a degenerate row (no positive sigma reaches log2 k), else 0.
 */
static int smooth_row(const double *dd, int m, int k, double *rho_out, double *sigma_out, double *a) {
    const double target = log2((double)k);
    double rho = 0.0;
    for (int j = 0; j < m; ++j)
        if (dd[j] > 0.0 && (rho == 0.0 || dd[j] < rho)) rho = dd[j];
    int at_rho = 0; /* slots whose weight is 1 for every sigma */
    for (int j = 0; j < m; ++j)
        if (dd[j] <= rho) ++at_rho;
    *rho_out = rho;
    if ((double)at_rho >= target) {
        *sigma_out = 0.0;
        for (int j = 0; j < m; ++j) a[j] = dd[j] <= rho ? 1.0 : 0.0;
        return 1;
    }
    double sigma = 1.0, lo = 0.0, hi = INFINITY;
    for (int it = 0; it < 200; ++it) {
        double f = membership_sum(dd, m, rho, sigma);
        if (fabs(f - target) <= 1e-12 * target) break;
        if (f > target)
            hi = sigma;
        else
            lo = sigma;
        if (isinf(hi))
            sigma = sigma * 2.0;
        else
            sigma = (lo + hi) / 2.0;
        if (!isinf(hi) && hi - lo <= ldexp(hi, -52)) break;
    }
    *sigma_out = sigma;
    for (int j = 0; j < m; ++j) {
        double g = dd[j] - rho;
        if (g < 0.0) g = 0.0;
        a[j] = exp(-g / sigma);
    }
    return 0;
}

/*
 * rho, sigma and directed weights for every row of a kNN result.
 * idx/dist: n x k (self in slot 0).  a: n x (k-1) float64 (slot s+1 -> a[s]).
 * rho/sigma may be NULL.  Returns the number of degenerate rows, or -1.
 */
int64_t oracle_smooth_knn(const int32_t *idx, const float *dist, int64_t n, int k, double *rho, double *sigma,
                          double *a) {
    (void)idx;
    if (n < 0 || k < 1) return -1;
    int m = k - 1;
    int64_t degenerate = 0;
#pragma omp parallel for reduction(+ : degenerate) schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double dd[1024];
        double r = 0.0, s = 0.0;
        double *ai = a + i * (int64_t)m;
        if (m > 1024) continue;
        for (int j = 0; j < m; ++j) dd[j] = (double)dist[i * (int64_t)k + 1 + j];
        degenerate += smooth_row(dd, m, k, &r, &s, ai);
        if (rho) rho[i] = r;
        if (sigma) sigma[i] = s;
    }
    return (m > 1024) ? -1 : degenerate;
}

typedef struct {
    int64_t row, col;
    double w;
    int dir; /* 0: edge row -> col; 1: edge col -> row */
} coo_t;

static int coo_cmp(const void *pa, const void *pb) {
    const coo_t *a = (const coo_t *)pa, *b = (const coo_t *)pb;
    if (a->row != b->row) return a->row < b->row ? -1 : 1;
    if (a->col != b->col) return a->col < b->col ? -1 : 1;
    return 0;
}

/*
 * Fuzzy union of the directed graph (i -> idx[i][s], a[i][s-1]), s = 1..k-1:
 * the matrix A + A^T - A o A^T, as CSR.  Every directed edge contributes its
 * weight to (i, j) and to (j, i); an entry reached twice is a pair joined
 * both ways and takes a + b - a*b.  Values are rounded to float32; zeros are
 * dropped.  cap: capacity of indices/data.  Returns nnz, -1 on bad input,
 * -2 if cap is too small.
 */
int64_t oracle_fuzzy_union(const int32_t *idx, const double *a, int64_t n, int k, int64_t *indptr,
                           int32_t *indices, float *data, int64_t cap) {
    if (n < 0 || k < 1) return -1;
    int m = k - 1;
    int64_t ne = n * (int64_t)m;
    coo_t *e = (coo_t *)malloc(sizeof(coo_t) * (size_t)(2 * ne + 1));
    if (!e) return -1;
    int64_t c = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int s = 0; s < m; ++s) {
            int64_t j = idx[i * (int64_t)k + 1 + s];
            if (j < 0 || j >= n || j == i) {
                free(e);
                return -1;
            }
            double w = a[i * (int64_t)m + s];
            e[c].row = i;
            e[c].col = j;
            e[c].w = w;
            e[c].dir = 0;
            ++c;
            e[c].row = j;
            e[c].col = i;
            e[c].w = w;
            e[c].dir = 1;
            ++c;
        }
    }
    qsort(e, (size_t)c, sizeof(coo_t), coo_cmp);
    int64_t nnz = 0, p = 0;
    for (int64_t r = 0; r <= n; ++r) {
        if (r < n) indptr[r] = nnz;
        if (r == n) break;
        while (p < c && e[p].row == r) {
            double w = e[p].w;
            int64_t col = e[p].col;
            if (p + 1 < c && e[p + 1].row == r && e[p + 1].col == col) {
                double b = e[p + 1].w;
                if (e[p + 1].dir == e[p].dir || (p + 2 < c && e[p + 2].row == r && e[p + 2].col == col)) {
                    free(e); /* a neighbour listed twice in one row */
                    return -1;
                }
                w = (w + b) - w * b;
                p += 2;
            } else {
                p += 1;
            }
            float wf = (float)w;
            if (wf != 0.0f) {
                if (nnz >= cap) {
                    free(e);
                    return -2;
                }
                indices[nnz] = (int32_t)col;
                data[nnz] = wf;
                ++nnz;
            }
        }
    }
    indptr[n] = nnz;
    free(e);
    return nnz;
}

/*
 * Exact kNN restricted to given candidate sets (the routed form's result
 * for a query is the exact nearest neighbours among the references of the
 * partitions it probes).
 *
 * Query i is row qrows[i] of X (row i when qrows is NULL; nq queries); its
 * candidates are cand_ids[cand_off[i] .. cand_off[i+1]) (row ids of X, each
 * at most once; the query's own row may be among them and is ignored).
 * Slot 0 is the query's row with distance 0; slots 1..k-1 hold the nearest
 * candidates by (d2, index); slots left empty get index -1 and an infinite
 * distance.  Returns 0, or -1 on bad arguments.
 */
int oracle_knn_subset(const float *X, int64_t n, int d, int k, const int64_t *qrows, int64_t nq,
                      const int64_t *cand_off, const int64_t *cand_ids, int32_t *out_idx, double *out_d2,
                      float *out_dist) {
    if (n < 0 || nq < 0 || d < 1 || k < 1) return -1;
    int fail = 0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nq; ++i) {
        const int64_t q = qrows ? qrows[i] : i;
        if (q < 0 || q >= n) {
            fail = 1;
            continue;
        }
        const float *x = X + q * (int64_t)d;
        double *bd = (double *)malloc(sizeof(double) * (size_t)k);
        int64_t *bj = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
        if (!bd || !bj) {
            fail = 1;
            free(bd);
            free(bj);
            continue;
        }
        bd[0] = 0.0;
        bj[0] = q;
        int cnt = 1; /* slots [1, cnt) sorted ascending */
        for (int64_t c = cand_off[i]; c < cand_off[i + 1]; ++c) {
            int64_t j = cand_ids[c];
            if (j < 0 || j >= n) {
                fail = 1;
                break;
            }
            if (j == q) continue;
            double v = sq_dist(x, X + j * (int64_t)d, d);
            int p;
            if (cnt < k) {
                p = cnt++;
            } else if (k > 1 && before(v, j, bd[k - 1], bj[k - 1])) {
                p = k - 1;
            } else {
                continue;
            }
            while (p > 1 && before(v, j, bd[p - 1], bj[p - 1])) {
                bd[p] = bd[p - 1];
                bj[p] = bj[p - 1];
                --p;
            }
            bd[p] = v;
            bj[p] = j;
        }
        for (int s = 0; s < k; ++s) {
            int64_t o = i * (int64_t)k + s;
            out_idx[o] = (int32_t)(s < cnt ? bj[s] : -1);
            if (out_d2) out_d2[o] = s < cnt ? bd[s] : INFINITY;
            if (out_dist) out_dist[o] = s < cnt ? (float)sqrt(bd[s]) : INFINITY;
        }
        free(bd);
        free(bj);
    }
    return fail ? -1 : 0;
}

/*
 * Cosine distance of two float32 rows in float64: 1 - x.y / (||x|| ||y||),
 * the dot product and both squared norms summed in dimension order, each
 * product and sum rounded on its own.  A row of zero norm has no direction:
 * its distance to every row is 1 (cosine 0).
 */
static double cos_dist(const float *x, const float *y, int d) {
    double xy = 0.0, xx = 0.0, yy = 0.0;
    for (int t = 0; t < d; ++t) {
        double a = (double)x[t], b = (double)y[t];
        xy = xy + a * b;
        xx = xx + a * a;
        yy = yy + b * b;
    }
    if (xx == 0.0 || yy == 0.0) return 1.0;
    return 1.0 - xy / (sqrt(xx) * sqrt(yy));
}

/*
 * Exact kNN under the cosine distance, otherwise as oracle_knn (self in slot
 * 0 when self_ids is given, (distance, index) order, ties to the lower
 * index).  out_d2 receives the cosine distances in float64, out_dist the
 * same rounded to float32.
 */
int oracle_knn_cosine(const float *Q, int64_t nq, const int64_t *self_ids, const float *R, int64_t nr, int d,
                      int k, int32_t *out_idx, double *out_d, float *out_dist) {
    if (nq < 0 || nr < 1 || d < 1 || k < 1 || k > nr) return -1;
    int fail = 0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < nq; ++q) {
        const float *x = Q + q * (int64_t)d;
        int64_t self = self_ids ? self_ids[q] : -1;
        double *bd = (double *)malloc(sizeof(double) * (size_t)k);
        int64_t *bj = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
        if (!bd || !bj) {
            fail = 1;
            free(bd);
            free(bj);
            continue;
        }
        int start = 0;
        if (self >= 0) {
            bd[0] = 0.0;
            bj[0] = self;
            start = 1;
        }
        int cnt = start;
        for (int64_t j = 0; j < nr; ++j) {
            if (j == self) continue;
            double v = cos_dist(x, R + j * (int64_t)d, d);
            int p;
            if (cnt < k) {
                p = cnt++;
            } else if (k > start && before(v, j, bd[k - 1], bj[k - 1])) {
                p = k - 1;
            } else {
                continue;
            }
            while (p > start && before(v, j, bd[p - 1], bj[p - 1])) {
                bd[p] = bd[p - 1];
                bj[p] = bj[p - 1];
                --p;
            }
            bd[p] = v;
            bj[p] = j;
        }
        for (int s = 0; s < k; ++s) {
            int64_t o = q * (int64_t)k + s;
            out_idx[o] = (int32_t)(s < cnt ? bj[s] : -1);
            if (out_d) out_d[o] = s < cnt ? bd[s] : INFINITY;
            if (out_dist) out_dist[o] = s < cnt ? (float)bd[s] : INFINITY;
        }
        free(bd);
        free(bj);
    }
    return fail ? -1 : 0;
}

/*
 * Group-pair distance sums for the energy distance (Methods, "Perturbation
 * distance computation").  Cells are grouped through category offsets and a
 * sorted cell-index array: group g holds the rows cells[offsets[g] ..
 * offsets[g+1]).  For every listed pair (a, b):
 *
 *   a != b   out = sum over i in a, j in b of ||x_i - x_j||
 *   a == b   out = sum over i < j (positions within the group) of
 *            ||x_i - x_j||, the upper triangle only; 0 for a group with
 *            fewer than two cells
 *
 * Each distance is the square root of the float64 sum of squared direct
 * differences; the sums run sequentially in float64, rows of a outer.
 * Returns 0, or -1 for invalid arguments (a group id out of range, offsets
 * not ascending, a cell index out of range).
 */
int oracle_edistance_sums(const float *X, int64_t n, int d, const int64_t *offsets, int64_t G,
                          const int32_t *cells, const int32_t *pairs, int64_t npairs, double *out) {
    if (n < 0 || d < 1 || G < 1 || npairs < 0) return -1;
    if (offsets[0] != 0) return -1;
    for (int64_t g = 0; g < G; ++g)
        if (offsets[g + 1] < offsets[g]) return -1;
    for (int64_t c = 0; c < offsets[G]; ++c)
        if (cells[c] < 0 || cells[c] >= n) return -1;
    for (int64_t p = 0; p < npairs; ++p)
        if (pairs[2 * p] < 0 || pairs[2 * p] >= G || pairs[2 * p + 1] < 0 || pairs[2 * p + 1] >= G) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < npairs; ++p) {
        const int64_t a = pairs[2 * p], b = pairs[2 * p + 1];
        double s = 0.0;
        for (int64_t u = offsets[a]; u < offsets[a + 1]; ++u) {
            const float *x = X + (int64_t)cells[u] * d;
            const int64_t v0 = a == b ? u + 1 : offsets[b];
            for (int64_t v = v0; v < offsets[b + 1]; ++v) s = s + sqrt(sq_dist(x, X + (int64_t)cells[v] * d, d));
        }
        out[p] = s;
    }
    return 0;
}

/*
 * UMAP layout by stochastic gradient descent over the edges of the fuzzy
 * graph (the layout step of UMAP, reference [15] of the paper's Technical
 * architecture section; the paper runs it on the graph this library builds).
 * One reading of the method, written out plainly:
 *
 *   q(d2)      = 1 / (1 + a d2^b), d2 the squared embedding distance
 *   eps_e      = w_max / w_e epochs between samples of edge e (never
 *                sampled if w_e < w_max / n_epochs); first due at eps_e
 *   epoch t    (0 .. n_epochs-1), alpha_t = alpha0 (1 - t / n_epochs):
 *              every move is computed from the embedding at the start of
 *              the epoch (Y); vertex i sums the moves of its own edges in
 *              CSR order, then Y_i += the sum.  For each edge e = (i, j)
 *              of row i that is due (next_e <= t; then next_e += eps_e):
 *                attraction: d2 = |Y_i - Y_j|^2, g = -2 a b d2^(b-1) /
 *                  (a d2^b + 1) if d2 > 0 else 0 (UMAP's published
 *                  gradient of -log q, both powers as written);
 *                  move_i += clip(g (Y_i - Y_j)) alpha_t per coordinate;
 *                `neg` repulsions from vertices k = splitmix64(seed, t, e,
 *                  p) mod n, p = 0 .. neg-1 (k == i skipped): d2 = |Y_i -
 *                  Y_k|^2, if d2 > 0: g = 2 gamma b / ((0.001 + d2)(a d2^b
 *                  + 1)), move_i += clip(g (Y_i - Y_k)) alpha_t, else
 *                  move_i += 4 alpha_t per coordinate;
 *   clip(x)    = max(-4, min(4, x));
 *   d2^b, d2^(b-1)  each power rounded to the nearest double (evaluated
 *              in quadruple precision, then rounded), so that the result is
 *              one defined function of the inputs, whatever library computes
 *              it; b - 1 is the float64 difference.
 *
 * splitmix64: state s = seed + (t * 2^40 + e * 2^6 + p + 1) * 0x9E3779B97F4A7C15
 * (mod 2^64), then the SplitMix64 finaliser (xor-shift 30, multiply by
 * 0xBF58476D1CE4E5B9, xor-shift 27, multiply by 0x94D049BB133111EB,
 * xor-shift 31); k = (out >> 11) mod n.  The edge term's stride 2^6 is the
 * largest `neg` (64), so no two (edge, draw) pairs of an epoch share a
 * counter (e < 2^32 keeps e * 2^6 below the epoch term).
 *
 * Y is n x dim float64, updated in place.  Returns 0, or -1 for invalid
 * arguments.
 */
static uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t oracle_splitmix64_next(uint64_t state) { return sm64_mix(state + 0x9E3779B97F4A7C15ull); }

/* The vertex that negative sample p of edge e draws in epoch t. */
int64_t oracle_umap_negative(uint64_t seed, int t, int64_t e, int p, int64_t n) {
    uint64_t st = seed + ((uint64_t)t * (1ull << 40) + (uint64_t)e * 64ull + (uint64_t)p + 1ull) *
                             0x9E3779B97F4A7C15ull;
    return (int64_t)((sm64_mix(st) >> 11) % (uint64_t)n);
}

static double clip4(double x) { return x > 4.0 ? 4.0 : (x < -4.0 ? -4.0 : x); }

/* x^y rounded to nearest: the quadruple-precision power (about 113 bits) rounded to double */
static double pow_rn(double x, double y) { return (double)powq((__float128)x, (__float128)y); }

int oracle_umap_layout(const int64_t *indptr, const int32_t *indices, const float *weights, int64_t n, int dim,
                       double *Y, int n_epochs, double a, double b, double gamma, double alpha0, int neg,
                       uint64_t seed) {
    if (n < 1 || dim < 1 || n_epochs < 0 || neg < 0 || neg > 64) return -1;
    int64_t nnz = indptr[n];
    double wmax = 0.0;
    for (int64_t e = 0; e < nnz; ++e)
        if ((double)weights[e] > wmax) wmax = (double)weights[e];
    double *eps = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    double *next = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    double *Y0 = (double *)malloc(sizeof(double) * (size_t)n * dim);
    if (!eps || !next || !Y0) {
        free(eps); free(next); free(Y0);
        return -1;
    }
    for (int64_t e = 0; e < nnz; ++e) {
        double w = (double)weights[e];
        eps[e] = (w > 0.0 && w >= wmax / (double)n_epochs) ? wmax / w : -1.0;
        next[e] = eps[e];
    }
    for (int t = 0; t < n_epochs; ++t) {
        double alpha = alpha0 * (1.0 - (double)t / (double)n_epochs);
        memcpy(Y0, Y, sizeof(double) * (size_t)n * dim);
        /* vertex i reads only Y0 and writes only Y_i and its own row's next[] */
#pragma omp parallel for schedule(dynamic, 512)
        for (int64_t i = 0; i < n; ++i) {
            const double *yi = Y0 + i * dim;
            double mv[dim];
            for (int c = 0; c < dim; ++c) mv[c] = 0.0;
            for (int64_t e = indptr[i]; e < indptr[i + 1]; ++e) {
                if (eps[e] < 0.0 || next[e] > (double)t) continue;
                next[e] = next[e] + eps[e];
                const double *yj = Y0 + (int64_t)indices[e] * dim;
                double d2 = 0.0;
                for (int c = 0; c < dim; ++c) d2 = d2 + (yi[c] - yj[c]) * (yi[c] - yj[c]);
                double g = 0.0;
                if (d2 > 0.0) g = (-2.0 * a * b * pow_rn(d2, b - 1.0)) / (a * pow_rn(d2, b) + 1.0);
                for (int c = 0; c < dim; ++c) mv[c] = mv[c] + clip4(g * (yi[c] - yj[c])) * alpha;
                for (int p = 0; p < neg; ++p) {
                    int64_t k = oracle_umap_negative(seed, t, e, p, n);
                    if (k == i) continue;
                    const double *yk = Y0 + k * dim;
                    double dk = 0.0;
                    for (int c = 0; c < dim; ++c) dk = dk + (yi[c] - yk[c]) * (yi[c] - yk[c]);
                    if (dk > 0.0) {
                        double gr = (2.0 * gamma * b) / ((0.001 + dk) * (a * pow_rn(dk, b) + 1.0));
                        for (int c = 0; c < dim; ++c) mv[c] = mv[c] + clip4(gr * (yi[c] - yk[c])) * alpha;
                    } else {
                        for (int c = 0; c < dim; ++c) mv[c] = mv[c] + 4.0 * alpha;
                    }
                }
            }
            for (int c = 0; c < dim; ++c) Y[i * dim + c] = yi[c] + mv[c];
        }
    }
    free(eps); free(next); free(Y0);
    return 0;
}
