/*
 * CPU oracle of Leiden community detection on the connectivities graph
 * (test infrastructure only: the test suite, the package smoke check and the
 * benchmark's CPU baseline leg call it; nothing here is shared with the HIP
 * library).
 *
 * The paper clusters cells by Leiden on the neighbourhood graph (Technical
 * architecture; Methods, "Dimensionality reduction and graph analysis") and
 * validates the GPU clustering against the CPU one by agreement of the
 * partitions (Methods, "Numerical validation"), not by identical labels,
 * because the published algorithm visits vertices in random order and draws
 * its refinement merges at random.  This is one deterministic reading of
 * the algorithm of Traag, Waltman and van Eck ("From Louvain to Leiden"),
 * written so that a parallel implementation can reach the same labels:
 *
 * Quality: modularity with resolution gamma,
 *     Q = 1/(2m) sum_c [ In(c) - gamma Tot(c)^2 / (2m) ],
 * In(c) the weight of the ordered pairs inside c (diagonal entries of an
 * aggregated graph included), Tot(c) the sum of the degrees k_v of its
 * vertices, 2m the sum of all degrees.
 *
 * Weights: every weight w is turned into the integer W = rint(w 2^S) with
 * S = 62 - ceil(log2 nnz) - ceil(log2 w_max), so that every sum of weights
 * (degrees, community totals, aggregated edges) is an exact int64 and does
 * not depend on the order of summation.  A gain is evaluated in float64
 * from these integers, each operation rounded as written:
 *     h(v, c) = K(v, c) - ((gamma k_v) T(c)) / 2m
 * with K(v, c) the weight from v to the other vertices of c and T(c) the
 * total of c without v.
 *
 * Level (graph G, initial labels L; level 0: singletons L[v] = v):
 *   1. local moving, in sweeps: in each sweep every vertex looks at the
 *      labels as they stood at the start of the sweep and takes the
 *      neighbouring community with the largest gain, if that gain is
 *      strictly above the gain of staying (ties: the lowest label); odd
 *      sweeps allow only moves to higher labels, even sweeps only to lower
 *      ones, so that two vertices cannot swap back and forth.  The phase
 *      ends after an upward and a downward sweep in a row without moves (or
 *      after 64 sweeps).
 *   2. refinement, in rounds, inside every community C of step 1: the
 *      refined partition starts from singletons; in a round, every vertex
 *      that is still a singleton and is well connected to C (K(v, C) >=
 *      gamma k_v (Tot(C) - k_v) / 2m) may join the refined community R of
 *      a neighbour in C with a smaller label, if R is well connected to C
 *      (E(R, C - R) >= gamma Tot(R) (Tot(C) - Tot(R)) / 2m) and the gain
 *      h(v, R) is >= 0; it takes the largest gain (ties: the lowest label).
 *      A join into a singleton that itself moves in the same round is
 *      cancelled.  A refined community's label stays its smallest vertex.
 *      The phase ends after a round without joins (or after 64 rounds).
 *   3. aggregation: the refined communities become the vertices of the next
 *      level (numbered in the order of their smallest vertex), the weight
 *      between two of them the sum of the weights between their vertices
 *      (a community's own weight on the diagonal); each starts in the
 *      community of step 1 that holds it, labelled by the smallest new
 *      vertex id of that community.
 * The levels end when step 1 moves no vertex (or after 32 levels).  The
 * labels of the last level are carried down to the input vertices and
 * renumbered in order of first appearance (vertex 0's community is 0).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t n;
    int64_t *ptr; /* n + 1 */
    int64_t *col; /* columns ascending per row */
    int64_t *w;   /* int64 weights */
} lgraph;

static void lg_free(lgraph *g) {
    free(g->ptr);
    free(g->col);
    free(g->w);
    g->ptr = NULL;
    g->col = NULL;
    g->w = NULL;
}

static int cmp_i64(const void *a, const void *b) {
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* h = K - ((gamma k) T) / 2m, every operation rounded as written */
static double gain(int64_t K, double gamma, int64_t k, int64_t T, int64_t two_m) {
    double t = gamma * (double)k;
    double u = t * (double)T;
    double q = u / (double)two_m;
    return (double)K - q;
}

/* The fixed-point exponent S for weights up to wmax over nnz entries. */
int oracle_leiden_scale(int64_t nnz, double wmax) {
    int c = 0, e = 0;
    while (((int64_t)1 << c) < nnz) ++c;
    if (wmax > 0.0) {
        frexp(wmax, &e); /* wmax = f 2^e, f in [0.5, 1): wmax <= 2^e */
    }
    return 62 - c - e;
}

/* Step 1: local moving of G's vertices from labels L (in place).  Returns
 * the number of vertex moves made. */
static int64_t local_moving(const lgraph *g, const int64_t *k, int64_t two_m, double gamma, int64_t *L) {
    int64_t n = g->n;
    int64_t *tot = calloc((size_t)n, sizeof(int64_t));
    int64_t *K = calloc((size_t)n, sizeof(int64_t));
    int64_t *touched = malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t *next = malloc(sizeof(int64_t) * (size_t)n);
    int64_t moves = 0;
    int quiet = 0;
    for (int sweep = 1; sweep <= 64 && quiet < 2; ++sweep) {
        int up = sweep % 2 == 1;
        memset(tot, 0, sizeof(int64_t) * (size_t)n);
        for (int64_t v = 0; v < n; ++v) tot[L[v]] += k[v];
        int64_t moved = 0;
        for (int64_t v = 0; v < n; ++v) {
            int64_t a = L[v], nt = 0;
            for (int64_t e = g->ptr[v]; e < g->ptr[v + 1]; ++e) {
                int64_t u = g->col[e];
                if (u == v) continue;
                int64_t c = L[u];
                if (K[c] == 0) touched[nt++] = c;
                K[c] += g->w[e];
            }
            /* a community reached only through zero-weight edges is still a
               candidate, with K = 0 (it may enter the list more than once;
               repeats change nothing) */
            double best_h = gain(K[a], gamma, k[v], tot[a] - k[v], two_m);
            int64_t best = a;
            qsort(touched, (size_t)nt, sizeof(int64_t), cmp_i64);
            for (int64_t t = 0; t < nt; ++t) {
                int64_t c = touched[t];
                if (c == a || (up ? c < a : c > a)) continue;
                double h = gain(K[c], gamma, k[v], tot[c], two_m);
                if (h > best_h) {
                    best_h = h;
                    best = c;
                }
            }
            for (int64_t t = 0; t < nt; ++t) K[touched[t]] = 0;
            next[v] = best;
            moved += best != a;
        }
        memcpy(L, next, sizeof(int64_t) * (size_t)n);
        moves += moved;
        quiet = moved ? 0 : quiet + 1;
    }
    free(tot);
    free(K);
    free(touched);
    free(next);
    return moves;
}

/* Step 2: refined labels R (R[v] = smallest vertex of v's refined
 * community) inside the communities L. */
static void refine(const lgraph *g, const int64_t *k, int64_t two_m, double gamma, const int64_t *L, int64_t *R) {
    int64_t n = g->n;
    int64_t *totC = calloc((size_t)n, sizeof(int64_t));  /* by community label */
    int64_t *totR = calloc((size_t)n, sizeof(int64_t));  /* by refined label */
    int64_t *extR = calloc((size_t)n, sizeof(int64_t));  /* E(R, C - R) by refined label */
    int64_t *size = calloc((size_t)n, sizeof(int64_t));  /* members by refined label */
    int64_t *kin = calloc((size_t)n, sizeof(int64_t));   /* K(v, C - v) */
    int64_t *K = calloc((size_t)n, sizeof(int64_t));
    int64_t *touched = malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t *prop = malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t v = 0; v < n; ++v) {
        R[v] = v;
        totC[L[v]] += k[v];
        for (int64_t e = g->ptr[v]; e < g->ptr[v + 1]; ++e)
            if (g->col[e] != v && L[g->col[e]] == L[v]) kin[v] += g->w[e];
    }
    for (int round = 1; round <= 64; ++round) {
        memset(totR, 0, sizeof(int64_t) * (size_t)n);
        memset(extR, 0, sizeof(int64_t) * (size_t)n);
        memset(size, 0, sizeof(int64_t) * (size_t)n);
        for (int64_t v = 0; v < n; ++v) {
            totR[R[v]] += k[v];
            size[R[v]] += 1;
            for (int64_t e = g->ptr[v]; e < g->ptr[v + 1]; ++e) {
                int64_t u = g->col[e];
                if (L[u] == L[v] && R[u] != R[v]) extR[R[v]] += g->w[e];
            }
        }
        for (int64_t v = 0; v < n; ++v) {
            prop[v] = -1;
            if (R[v] != v || size[v] != 1) continue; /* not a singleton */
            int64_t C = L[v];
            double need_v = (gamma * (double)k[v]) * (double)(totC[C] - k[v]) / (double)two_m;
            if (!((double)kin[v] >= need_v)) continue; /* not well connected to C */
            int64_t nt = 0;
            for (int64_t e = g->ptr[v]; e < g->ptr[v + 1]; ++e) {
                int64_t u = g->col[e];
                if (u == v || L[u] != C) continue;
                int64_t r = R[u];
                if (r >= v) continue; /* only refined communities with a smaller label */
                if (K[r] == 0) touched[nt++] = r;
                K[r] += g->w[e];
            }
            qsort(touched, (size_t)nt, sizeof(int64_t), cmp_i64);
            double best_h = 0.0;
            int64_t best = -1;
            for (int64_t t = 0; t < nt; ++t) {
                int64_t r = touched[t];
                double need_r = (gamma * (double)totR[r]) * (double)(totC[C] - totR[r]) / (double)two_m;
                if (!((double)extR[r] >= need_r)) continue; /* R not well connected to C */
                double h = gain(K[r], gamma, k[v], totR[r], two_m);
                if (h >= 0.0 && (best < 0 || h > best_h)) {
                    best_h = h;
                    best = r;
                }
            }
            for (int64_t t = 0; t < nt; ++t) K[touched[t]] = 0;
            prop[v] = best;
        }
        int64_t joins = 0;
        for (int64_t v = 0; v < n; ++v) {
            int64_t t = prop[v];
            if (t < 0) continue;
            if (size[t] == 1 && prop[t] >= 0) continue; /* the target singleton moves away */
            R[v] = t;
            ++joins;
        }
        if (!joins) break;
    }
    free(totC);
    free(totR);
    free(extR);
    free(size);
    free(kin);
    free(K);
    free(touched);
    free(prop);
}

/* Step 2 alone, for the tests: the refined labels of the input graph's
 * vertices inside the given communities (labels: int32 n, each a vertex id
 * in [0, n)).  Returns 0, or -1 for invalid input. */
int oracle_leiden_refine(const int64_t *indptr, const int32_t *indices, const float *weights, int64_t n,
                         double gamma, const int32_t *labels, int32_t *refined) {
    if (n < 1 || !(gamma > 0.0) || indptr[0] != 0) return -1;
    int64_t nnz = indptr[n];
    double wmax = 0.0;
    for (int64_t e = 0; e < nnz; ++e) {
        if (!(weights[e] >= 0.0f) || isinf(weights[e]) || indices[e] < 0 || indices[e] >= n) return -1;
        if ((double)weights[e] > wmax) wmax = (double)weights[e];
    }
    for (int64_t v = 0; v < n; ++v)
        if (labels[v] < 0 || labels[v] >= n) return -1;
    int S = oracle_leiden_scale(nnz > 0 ? nnz : 1, wmax);
    lgraph g;
    g.n = n;
    g.ptr = malloc(sizeof(int64_t) * (size_t)(n + 1));
    g.col = malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
    g.w = malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
    int64_t *k = calloc((size_t)n, sizeof(int64_t));
    int64_t *L = malloc(sizeof(int64_t) * (size_t)n);
    int64_t *R = malloc(sizeof(int64_t) * (size_t)n);
    int64_t two_m = 0;
    for (int64_t i = 0; i <= n; ++i) g.ptr[i] = indptr[i];
    for (int64_t v = 0; v < n; ++v) {
        L[v] = labels[v];
        for (int64_t e = indptr[v]; e < indptr[v + 1]; ++e) {
            g.col[e] = indices[e];
            g.w[e] = (int64_t)rint(ldexp((double)weights[e], S));
            k[v] += g.w[e];
        }
        two_m += k[v];
    }
    if (two_m > 0) {
        refine(&g, k, two_m, gamma, L, R);
    } else {
        for (int64_t v = 0; v < n; ++v) R[v] = v;
    }
    for (int64_t v = 0; v < n; ++v) refined[v] = (int32_t)R[v];
    free(k);
    free(L);
    free(R);
    lg_free(&g);
    return 0;
}

typedef struct {
    int64_t a, b, w;
} triple;

static int cmp_triple(const void *pa, const void *pb) {
    const triple *x = pa, *y = pb;
    if (x->a != y->a) return (x->a > y->a) - (x->a < y->a);
    return (x->b > y->b) - (x->b < y->b);
}

/*
 * Leiden labels of a symmetric CSR graph (weights >= 0; a diagonal entry is
 * allowed and counts once in its vertex's degree).  labels: int32 n
 * (output, numbered from 0 in order of first appearance).  quality: the
 * modularity of the result (float64, may be NULL).  levels (may be NULL):
 * levels run.  Returns 0, or -1 for invalid input.
 */
int oracle_leiden(const int64_t *indptr, const int32_t *indices, const float *weights, int64_t n, double gamma,
                  int32_t *labels, double *quality, int32_t *levels) {
    if (n < 1 || !(gamma > 0.0) || indptr[0] != 0) return -1;
    int64_t nnz = indptr[n];
    double wmax = 0.0;
    for (int64_t e = 0; e < nnz; ++e) {
        if (!(weights[e] >= 0.0f) || isinf(weights[e]) || indices[e] < 0 || indices[e] >= n) return -1;
        if ((double)weights[e] > wmax) wmax = (double)weights[e];
    }
    int S = oracle_leiden_scale(nnz > 0 ? nnz : 1, wmax);
    lgraph g;
    g.n = n;
    g.ptr = malloc(sizeof(int64_t) * (size_t)(n + 1));
    g.col = malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
    g.w = malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
    for (int64_t i = 0; i <= n; ++i) g.ptr[i] = indptr[i];
    for (int64_t e = 0; e < nnz; ++e) {
        g.col[e] = indices[e];
        g.w[e] = (int64_t)rint(ldexp((double)weights[e], S));
    }
    /* top[v]: the vertex of the current level that input vertex v belongs to */
    int64_t *top = malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t v = 0; v < n; ++v) top[v] = v;
    int64_t *L = malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t v = 0; v < n; ++v) L[v] = v;
    int lv = 0;
    int64_t two_m = 0;
    for (;;) {
        int64_t N = g.n;
        int64_t *k = calloc((size_t)N, sizeof(int64_t));
        two_m = 0;
        for (int64_t v = 0; v < N; ++v) {
            for (int64_t e = g.ptr[v]; e < g.ptr[v + 1]; ++e) k[v] += g.w[e];
            two_m += k[v];
        }
        if (two_m == 0) {
            free(k);
            break;
        }
        int64_t moves = local_moving(&g, k, two_m, gamma, L);
        ++lv;
        if (moves == 0 || lv >= 32) {
            free(k);
            break;
        }
        int64_t *R = malloc(sizeof(int64_t) * (size_t)N);
        refine(&g, k, two_m, gamma, L, R);
        free(k);
        /* new ids of the refined communities, in order of their smallest vertex */
        int64_t *id = malloc(sizeof(int64_t) * (size_t)N);
        int64_t K2 = 0;
        for (int64_t v = 0; v < N; ++v) id[v] = R[v] == v ? K2++ : -1;
        /* aggregated graph */
        int64_t m2 = g.ptr[N];
        triple *t = malloc(sizeof(triple) * (size_t)(m2 > 0 ? m2 : 1));
        for (int64_t v = 0; v < N; ++v)
            for (int64_t e = g.ptr[v]; e < g.ptr[v + 1]; ++e) {
                t[e].a = id[R[v]];
                t[e].b = id[R[g.col[e]]];
                t[e].w = g.w[e];
            }
        qsort(t, (size_t)m2, sizeof(triple), cmp_triple);
        lgraph h;
        h.n = K2;
        h.ptr = calloc((size_t)(K2 + 1), sizeof(int64_t));
        h.col = malloc(sizeof(int64_t) * (size_t)(m2 > 0 ? m2 : 1));
        h.w = malloc(sizeof(int64_t) * (size_t)(m2 > 0 ? m2 : 1));
        int64_t q = 0;
        for (int64_t e = 0; e < m2; ++e) {
            if (q > 0 && h.col[q - 1] == t[e].b && e > 0 && t[e - 1].a == t[e].a) {
                h.w[q - 1] += t[e].w;
                continue;
            }
            h.col[q] = t[e].b;
            h.w[q] = t[e].w;
            h.ptr[t[e].a + 1] += 1;
            ++q;
        }
        for (int64_t p = 0; p < K2; ++p) h.ptr[p + 1] += h.ptr[p];
        free(t);
        /* initial labels: the smallest new id among the refined communities of each community */
        int64_t *minid = malloc(sizeof(int64_t) * (size_t)N);
        for (int64_t v = 0; v < N; ++v) minid[v] = INT64_MAX;
        for (int64_t v = 0; v < N; ++v)
            if (id[R[v]] < minid[L[v]]) minid[L[v]] = id[R[v]];
        int64_t *L2 = malloc(sizeof(int64_t) * (size_t)(K2 > 0 ? K2 : 1));
        for (int64_t v = 0; v < N; ++v) L2[id[R[v]]] = minid[L[v]];
        for (int64_t v = 0; v < n; ++v) top[v] = id[R[top[v]]];
        free(minid);
        free(id);
        free(R);
        free(L);
        L = L2;
        lg_free(&g);
        g = h;
    }
    /* carry the last labels down and number them by first appearance */
    int64_t *num = malloc(sizeof(int64_t) * (size_t)g.n);
    for (int64_t v = 0; v < g.n; ++v) num[v] = -1;
    int64_t next_label = 0;
    for (int64_t v = 0; v < n; ++v) {
        int64_t c = L[top[v]];
        if (num[c] < 0) num[c] = next_label++;
        labels[v] = (int32_t)num[c];
    }
    free(num);
    if (quality) {
        /* modularity of the labels on the input graph, from the exact integer sums */
        int64_t *in = calloc((size_t)n, sizeof(int64_t)), *tot = calloc((size_t)n, sizeof(int64_t));
        int64_t tm = 0;
        for (int64_t v = 0; v < n; ++v)
            for (int64_t e = indptr[v]; e < indptr[v + 1]; ++e) {
                int64_t w = (int64_t)rint(ldexp((double)weights[e], S));
                tot[labels[v]] += w;
                tm += w;
                if (labels[indices[e]] == labels[v]) in[labels[v]] += w;
            }
        double Q = 0.0;
        if (tm > 0)
            for (int64_t c = 0; c < n; ++c)
                if (tot[c]) Q += (double)in[c] / (double)tm - gamma * ((double)tot[c] / (double)tm) * ((double)tot[c] / (double)tm);
        *quality = Q;
        free(in);
        free(tot);
    }
    if (levels) *levels = lv;
    free(L);
    free(top);
    lg_free(&g);
    return 0;
}
