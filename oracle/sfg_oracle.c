/*
 * Plain CPU FP64 reference of the SF-GRASS local-spectral-embedding path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; it shares no code with the GPU path.  Only the tests,
 * the smoke check and the benchmark's CPU-baseline leg use it.
 *
 * Every routine is the definition written out, one element at a time, in a
 * fixed and documented order.  Build with -O3 -ffp-contract=off (no FMA
 * contraction, no fast-math) so each operation rounds once, as written.
 *
 * Paper references are to Zhang, Zhao, Feng, "SF-GRASS: Solver-Free Graph
 * Spectral Sparsification", ICCAD 2020.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Rows (and edges) are independent within a sweep (or a scoring pass), and  */
/* each one is computed by one thread in the fixed order written below, so   */
/* the results are bit-identical for any number of threads.                  */
void orc_set_threads(int32_t t)
{
#ifdef _OPENMP
    omp_set_num_threads(t > 0 ? t : 1);
#else
    (void)t;
#endif
}

int32_t orc_max_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Graph Laplacian (Sec. 2.1, Eq. 1 and the definition L = D - A that        */
/* follows it).  Input: canonical edge list (u<v, sorted by (u,v), unique).  */
/* Output: symmetric CSR of A with ascending columns per row, the edge id of  */
/* every entry, and the weighted degree D(p,p) = sum of the weights of the    */
/* edges at p, added in ascending edge id.                                    */
/* ------------------------------------------------------------------------ */

typedef struct { int32_t row, col, eid; double w; } orc_entry;

static int cmp_entry(const void *a, const void *b)
{
    const orc_entry *x = (const orc_entry *)a, *y = (const orc_entry *)b;
    if (x->row != y->row) return x->row < y->row ? -1 : 1;
    if (x->col != y->col) return x->col < y->col ? -1 : 1;
    return 0;
}

int orc_laplacian_csr(int64_t n, int64_t m, const int32_t *u, const int32_t *v,
                      const double *w, int64_t *rowptr, int32_t *col, double *val,
                      int32_t *eid, double *deg)
{
    orc_entry *ent = (orc_entry *)malloc(sizeof(orc_entry) * (size_t)(2 * m + 1));
    if (!ent) return -1;
    for (int64_t e = 0; e < m; ++e) {
        ent[2 * e].row = u[e]; ent[2 * e].col = v[e]; ent[2 * e].eid = (int32_t)e; ent[2 * e].w = w[e];
        ent[2 * e + 1].row = v[e]; ent[2 * e + 1].col = u[e]; ent[2 * e + 1].eid = (int32_t)e; ent[2 * e + 1].w = w[e];
    }
    qsort(ent, (size_t)(2 * m), sizeof(orc_entry), cmp_entry);
    for (int64_t p = 0; p <= n; ++p) rowptr[p] = 0;
    for (int64_t j = 0; j < 2 * m; ++j) rowptr[ent[j].row + 1] += 1;
    for (int64_t p = 0; p < n; ++p) rowptr[p + 1] += rowptr[p];
    for (int64_t j = 0; j < 2 * m; ++j) { col[j] = ent[j].col; val[j] = ent[j].w; eid[j] = ent[j].eid; }
    free(ent);
    for (int64_t p = 0; p < n; ++p) deg[p] = 0.0;
    for (int64_t e = 0; e < m; ++e) { deg[u[e]] = deg[u[e]] + w[e]; deg[v[e]] = deg[v[e]] + w[e]; }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Local spectral embedding by low-pass smoothing (Sec. 3.2).  The paper     */
/* relaxes L x = 0 from random starts; read here as damped Jacobi:            */
/*   y_p = (1-omega) x_p + omega * (s_p / D_pp),                              */
/*   s_p = sum over the row's entries, ascending column, of (A_pq * x_q),     */
/* each product rounded, then added left to right starting from 0.            */
/* X, Y are n-by-k row-major.  After `sweeps` sweeps the result is in X.      */
/* ------------------------------------------------------------------------ */
void orc_smooth(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                const double *deg, int32_t k, int32_t sweeps, double omega,
                double *X, double *Y)
{
    const double keep = 1.0 - omega;
    for (int32_t t = 0; t < sweeps; ++t) {
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < n; ++p) {
            for (int32_t c = 0; c < k; ++c) {
                double s = 0.0;
                for (int64_t j = rowptr[p]; j < rowptr[p + 1]; ++j) {
                    double prod = val[j] * X[(int64_t)col[j] * k + c];
                    s = s + prod;
                }
                double a = keep * X[p * k + c];
                double b = s / deg[p];
                double bo = omega * b;
                Y[p * k + c] = a + bo;
            }
        }
        memcpy(X, Y, sizeof(double) * (size_t)(n * k));
    }
}

/* ------------------------------------------------------------------------ */
/* Multicolouring for a Gauss-Seidel reading of the smoother (Sec. 3.2 names */
/* Gauss-Seidel relaxations).  Jones-Plassmann rounds with a fixed priority: */
/* a node's priority is the pair (h(p), p) with h the multiply-xorshift      */
/* integer mixer below; in round r every uncoloured node whose priority      */
/* exceeds that of all its uncoloured neighbours takes the smallest colour   */
/* not used by a neighbour coloured in an earlier round.  Returns the number */
/* of colours; color[p] >= 0.                                                */
/* ------------------------------------------------------------------------ */
static uint32_t orc_mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

static int orc_prio_greater(int64_t p, int64_t q)
{
    const uint32_t hp = orc_mix32((uint32_t)p), hq = orc_mix32((uint32_t)q);
    return hp > hq || (hp == hq && p > q);
}

int32_t orc_color(int64_t n, const int64_t *rowptr, const int32_t *col, int32_t *color)
{
    int32_t *round = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t p = 0; p < n; ++p) { color[p] = -1; round[p] = -1; }
    int64_t left = n;
    int32_t ncolors = 0;
    for (int32_t r = 0; left > 0; ++r) {
        /* decide the whole round from the state before it */
        for (int64_t p = 0; p < n; ++p) {
            if (round[p] >= 0) continue;
            int is_max = 1;
            for (int64_t j = rowptr[p]; j < rowptr[p + 1] && is_max; ++j) {
                const int64_t q = col[j];
                /* uncoloured before this round (chosen earlier in this scan counts too) */
                if ((round[q] < 0 || round[q] == r) && orc_prio_greater(q, p)) is_max = 0;
            }
            if (is_max) round[p] = r;   /* chosen in this round (not yet coloured) */
        }
        for (int64_t p = 0; p < n; ++p) {
            if (round[p] != r) continue;
            int32_t c = 0;
            for (;;) {   /* smallest colour unused by neighbours coloured earlier */
                int used = 0;
                for (int64_t j = rowptr[p]; j < rowptr[p + 1]; ++j) {
                    const int64_t q = col[j];
                    if (round[q] >= 0 && round[q] < r && color[q] == c) { used = 1; break; }
                }
                if (!used) break;
                ++c;
            }
            color[p] = c;
            if (c + 1 > ncolors) ncolors = c + 1;
            --left;
        }
    }
    free(round);
    return ncolors;
}

/* Gauss-Seidel reading of the smoother: one sweep updates the colours in    */
/* order 0, 1, ..., in place; a row of colour c takes                        */
/*   x_p = (1-omega) x_p + omega * (s_p / D_pp)                               */
/* with s_p summed as in orc_smooth over the current values (its neighbours  */
/* have other colours, so the order inside a colour does not matter).        */
void orc_smooth_gs(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                   const double *deg, int32_t k, int32_t sweeps, double omega, const int32_t *color,
                   int32_t ncolors, double *X)
{
    const double keep = 1.0 - omega;
    for (int32_t t = 0; t < sweeps; ++t) {
        for (int32_t cc = 0; cc < ncolors; ++cc) {
            for (int64_t p = 0; p < n; ++p) {
                if (color[p] != cc) continue;
                for (int32_t c = 0; c < k; ++c) {
                    double s = 0.0;
                    for (int64_t j = rowptr[p]; j < rowptr[p + 1]; ++j) {
                        double prod = val[j] * X[(int64_t)col[j] * k + c];
                        s = s + prod;
                    }
                    double a = keep * X[p * k + c];
                    double b = s / deg[p];
                    double bo = omega * b;
                    X[p * k + c] = a + bo;
                }
            }
        }
    }
}

/* Same smoothing restricted to rows with dist[p] <= sweeps - t at sweep t   */
/* (t = 1..sweeps).  Rows outside the window keep stale values; the rows a   */
/* score at distance 0 depends on are exact.  Used to pin the GPU's           */
/* dependency-cone recomputation against the plain definition.                */
void orc_smooth_masked(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                       const double *deg, int32_t k, int32_t sweeps, double omega,
                       const int32_t *dist, double *X, double *Y)
{
    const double keep = 1.0 - omega;
    memcpy(Y, X, sizeof(double) * (size_t)(n * k));
    for (int32_t t = 1; t <= sweeps; ++t) {
        for (int64_t p = 0; p < n; ++p) {
            if (dist[p] > sweeps - t) continue;
            for (int32_t c = 0; c < k; ++c) {
                double s = 0.0;
                for (int64_t j = rowptr[p]; j < rowptr[p + 1]; ++j) {
                    double prod = val[j] * X[(int64_t)col[j] * k + c];
                    s = s + prod;
                }
                double a = keep * X[p * k + c];
                double b = s / deg[p];
                double bo = omega * b;
                Y[p * k + c] = a + bo;
            }
        }
        memcpy(X, Y, sizeof(double) * (size_t)(n * k));
    }
}

/* ------------------------------------------------------------------------ */
/* Edge score (Eq. 18 with the embedding of Sec. 3.2; Alg. 1 edge           */
/* distortion): s_e = w_e * sum_c (X_pc - X_qc)^2, c ascending, squares       */
/* rounded then added left to right from 0, then one multiply by w_e.         */
/* ------------------------------------------------------------------------ */
void orc_edge_scores(int32_t k, const double *X, int64_t ne, const int32_t *u, const int32_t *v,
                     const double *w, double *score)
{
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < ne; ++e) {
        double acc = 0.0;
        for (int32_t c = 0; c < k; ++c) {
            double d = X[(int64_t)u[e] * k + c] - X[(int64_t)v[e] * k + c];
            double d2 = d * d;
            acc = acc + d2;
        }
        score[e] = w[e] * acc;
    }
}

/* ------------------------------------------------------------------------ */
/* Node affinity of the algebraic-distance type (Sec. 3.2, the commented     */
/* affinity formula): a_pq = (Xb_p . Xb_q)^2 / (|Xb_p|^2 |Xb_q|^2), where Xb  */
/* is the caller's column-centred block.  Dot products and squared norms add  */
/* products left to right over ascending column; a := 0 when a norm is 0.    */
/* ------------------------------------------------------------------------ */
void orc_affinity(int32_t k, const double *Xb, int64_t ne, const int32_t *u, const int32_t *v,
                  double *aff)
{
    for (int64_t e = 0; e < ne; ++e) {
        double dot = 0.0, np_ = 0.0, nq = 0.0;
        for (int32_t c = 0; c < k; ++c) {
            double xp = Xb[(int64_t)u[e] * k + c], xq = Xb[(int64_t)v[e] * k + c];
            double a = xp * xq, b = xp * xp, d = xq * xq;
            dot = dot + a; np_ = np_ + b; nq = nq + d;
        }
        if (np_ == 0.0 || nq == 0.0) { aff[e] = 0.0; continue; }
        double num = dot * dot;
        double den = np_ * nq;
        aff[e] = num / den;
    }
}

/* ------------------------------------------------------------------------ */
/* Top-k selection ("include top few edges with large distortion", Alg. 1). */
/* Candidates are ordered by score descending, then edge id ascending; the    */
/* first k are chosen.  Writes their candidate positions in that order and    */
/* the k-th score as the threshold.                                           */
/* ------------------------------------------------------------------------ */
static const double *g_sel_score;
static const int32_t *g_sel_eid;

static int cmp_sel(const void *a, const void *b)
{
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    double si = g_sel_score[i], sj = g_sel_score[j];
    if (si != sj) return si > sj ? -1 : 1;
    int32_t ei = g_sel_eid[i], ej = g_sel_eid[j];
    return (ei < ej) ? -1 : (ei > ej);
}

int orc_select_topk(int64_t ne, const double *score, const int32_t *eid, int64_t k,
                    int64_t *chosen, double *tau)
{
    if (k < 0 || k > ne) return -1;
    int64_t *ord = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ne + 1));
    if (!ord) return -1;
    for (int64_t i = 0; i < ne; ++i) ord[i] = i;
    g_sel_score = score; g_sel_eid = eid;
    qsort(ord, (size_t)ne, sizeof(int64_t), cmp_sel);
    for (int64_t i = 0; i < k; ++i) chosen[i] = ord[i];
    *tau = (k > 0) ? score[ord[k - 1]] : INFINITY;
    free(ord);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Maximum-weight spanning tree (the MST stand-in for a low-stretch tree,    */
/* Sec. 3.4): Kruskal over edges ordered by weight descending, then edge id   */
/* ascending; union-find with path halving.  Marks in_tree[e] = 1.  Returns   */
/* the number of components of the resulting forest.                          */
/* Optional `allowed` restricts the candidate edges (NULL = all).             */
/* ------------------------------------------------------------------------ */
static const double *g_mst_w;

static int cmp_mst(const void *a, const void *b)
{
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    double wi = g_mst_w[i], wj = g_mst_w[j];
    if (wi != wj) return wi > wj ? -1 : 1;
    return (i < j) ? -1 : (i > j);
}

static int64_t uf_find(int64_t *par, int64_t x)
{
    while (par[x] != x) { par[x] = par[par[x]]; x = par[x]; }
    return x;
}

int64_t orc_max_spanning_forest(int64_t n, int64_t m, const int32_t *u, const int32_t *v,
                                const double *w, const uint8_t *allowed, uint8_t *in_tree)
{
    int64_t *ord = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
    int64_t *par = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!ord || !par) { free(ord); free(par); return -1; }
    int64_t cnt = 0;
    for (int64_t e = 0; e < m; ++e) { in_tree[e] = 0; if (!allowed || allowed[e]) ord[cnt++] = e; }
    g_mst_w = w;
    qsort(ord, (size_t)cnt, sizeof(int64_t), cmp_mst);
    for (int64_t p = 0; p < n; ++p) par[p] = p;
    int64_t comps = n;
    for (int64_t i = 0; i < cnt; ++i) {
        int64_t e = ord[i];
        int64_t a = uf_find(par, u[e]), b = uf_find(par, v[e]);
        if (a == b) continue;
        if (a < b) par[b] = a; else par[a] = b;
        in_tree[e] = 1;
        --comps;
    }
    free(ord); free(par);
    return comps;
}

/* Number of connected components of (n, edge list restricted to mask). */
int64_t orc_components(int64_t n, int64_t m, const int32_t *u, const int32_t *v,
                       const uint8_t *mask, int32_t *label)
{
    int64_t *par = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!par) return -1;
    for (int64_t p = 0; p < n; ++p) par[p] = p;
    for (int64_t e = 0; e < m; ++e) {
        if (mask && !mask[e]) continue;
        int64_t a = uf_find(par, u[e]), b = uf_find(par, v[e]);
        if (a == b) continue;
        if (a < b) par[b] = a; else par[a] = b;
    }
    int64_t c = 0;
    for (int64_t p = 0; p < n; ++p) {
        int64_t r = uf_find(par, p);
        if (r == p) label[p] = (int32_t)(c++);
        else label[p] = label[r];           /* r < p: already labelled */
    }
    free(par);
    return c;
}

/* ------------------------------------------------------------------------ */
/* Aggregation sets for coarsening (Sec. 3.2: cluster nodes that are close   */
/* in the embedding).  The paper does not fix the rule; here every node       */
/* points to the neighbour with the largest (affinity, weight, -id) key, and  */
/* the aggregates are the connected components of the undirected pointer      */
/* graph, numbered by ascending smallest member.  aff_entry is per CSR entry. */
/* Returns the number of aggregates.                                          */
/* ------------------------------------------------------------------------ */
int64_t orc_aggregate(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                      const double *aff_entry, int32_t *ptr, int32_t *agg)
{
    int64_t *par = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!par) return -1;
    for (int64_t p = 0; p < n; ++p) {
        int64_t best = -1;
        for (int64_t j = rowptr[p]; j < rowptr[p + 1]; ++j) {
            if (best < 0) { best = j; continue; }
            double a = aff_entry[j], ab = aff_entry[best];
            if (a > ab || (a == ab && (val[j] > val[best] ||
                          (val[j] == val[best] && col[j] < col[best]))))
                best = j;
        }
        ptr[p] = best < 0 ? (int32_t)p : col[best];
    }
    for (int64_t p = 0; p < n; ++p) par[p] = p;
    for (int64_t p = 0; p < n; ++p) {
        int64_t a = uf_find(par, p), b = uf_find(par, ptr[p]);
        if (a == b) continue;
        if (a < b) par[b] = a; else par[a] = b;
    }
    int64_t c = 0;
    for (int64_t p = 0; p < n; ++p) {
        int64_t r = uf_find(par, p);
        if (r == p) agg[p] = (int32_t)(c++);
        else agg[p] = agg[r];
    }
    free(par);
    return c;
}

/* ------------------------------------------------------------------------ */
/* Galerkin coarse graph (Eq. 3 with H and H+ of Eqs. 4-5): the coarse edge  */
/* (I,J), I<J, carries the sum of the weights of the fine edges between       */
/* aggregates I and J, added in ascending fine edge id.  Edges inside an      */
/* aggregate vanish.  Also returns, per coarse edge, the fine edge of largest */
/* weight between the two aggregates (ties: smallest id), which the backward  */
/* mapping of Sec. 3.4 keeps.  Output is in canonical (I,J) order; returns    */
/* the number of coarse edges.  Capacity of the outputs: m.                   */
/* ------------------------------------------------------------------------ */
typedef struct { int64_t key; int64_t e; } orc_kv;

static int cmp_kv(const void *a, const void *b)
{
    const orc_kv *x = (const orc_kv *)a, *y = (const orc_kv *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->e < y->e) ? -1 : (x->e > y->e);
}

int64_t orc_galerkin(int64_t m, const int32_t *u, const int32_t *v, const double *w,
                     const int32_t *agg, int64_t nc, int32_t *cu, int32_t *cv, double *cw,
                     int32_t *crep)
{
    orc_kv *kv = (orc_kv *)malloc(sizeof(orc_kv) * (size_t)(m + 1));
    if (!kv) return -1;
    int64_t cnt = 0;
    for (int64_t e = 0; e < m; ++e) {
        int64_t I = agg[u[e]], J = agg[v[e]];
        if (I == J) continue;
        int64_t lo = I < J ? I : J, hi = I < J ? J : I;
        kv[cnt].key = lo * nc + hi; kv[cnt].e = e; ++cnt;
    }
    qsort(kv, (size_t)cnt, sizeof(orc_kv), cmp_kv);
    int64_t out = -1;
    for (int64_t i = 0; i < cnt; ++i) {
        int64_t e = kv[i].e;
        if (i == 0 || kv[i].key != kv[i - 1].key) {
            ++out;
            cu[out] = (int32_t)(kv[i].key / nc); cv[out] = (int32_t)(kv[i].key % nc);
            cw[out] = w[e]; crep[out] = (int32_t)e;
        } else {
            cw[out] = cw[out] + w[e];
            if (w[e] > w[crep[out]]) crep[out] = (int32_t)e;   /* ascending e: ties keep the first */
        }
    }
    free(kv);
    return out + 1;
}

/* Exactly rounded sum (Shewchuk's adaptive partials, as in Python fsum). */
double orc_exact_sum(int64_t n, const double *x, int64_t stride)
{
    int cap = 64, np_ = 0;
    double *part = (double *)malloc(sizeof(double) * (size_t)cap);
    double special = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double xv = x[i * stride];
        if (!isfinite(xv)) { special += xv; continue; }
        int j = 0;
        for (int r = 0; r < np_; ++r) {
            double y = part[r];
            if (fabs(xv) < fabs(y)) { double t = xv; xv = y; y = t; }
            double hi = xv + y;
            double lo = y - (hi - xv);
            if (lo != 0.0) part[j++] = lo;
            xv = hi;
        }
        if (j >= cap) { cap *= 2; part = (double *)realloc(part, sizeof(double) * (size_t)cap); }
        if (xv != 0.0) part[j++] = xv;
        np_ = j;
    }
    if (special != 0.0 || isnan(special)) { free(part); return special; }
    /* round the partials exactly, from the top (same final step as fsum) */
    double hi = 0.0;
    if (np_ > 0) {
        int i = np_ - 1;
        hi = part[i];
        double lo = 0.0;
        while (i > 0) {
            double xv = hi;
            double y = part[--i];
            hi = xv + y;
            double yr = hi - xv;
            lo = y - yr;
            if (lo != 0.0) break;
        }
        if (i > 0 && ((lo < 0.0 && part[i - 1] < 0.0) || (lo > 0.0 && part[i - 1] > 0.0))) {
            double y = lo * 2.0;
            double xv = hi + y;
            double yr = xv - hi;
            if (y == yr) hi = xv;
        }
    }
    free(part);
    return hi;
}

/* Column centring (Sec. 3.2: random vectors orthogonal to the all-one       */
/* vector): mean_c = (exactly rounded column sum) / n, then X_pc -= mean_c.  */
void orc_center(int64_t n, int32_t k, double *X, double *mean)
{
    for (int32_t c = 0; c < k; ++c) {
        double s = orc_exact_sum(n, X + c, k);
        mean[c] = s / (double)n;
    }
    for (int64_t p = 0; p < n; ++p)
        for (int32_t c = 0; c < k; ++c) X[p * k + c] = X[p * k + c] - mean[c];
}

/* ------------------------------------------------------------------------ */
/* Random test vectors (Sec. 3.2 starts from random vectors).  Counter-based */
/* generator Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds   */
/* of two 32x32->64-bit multiplies (constants 0xD2511F53, 0xCD9E8D57) mixing */
/* the counter words with the key, the key bumped by (0x9E3779B9,            */
/* 0xBB67AE85) between rounds.  Standard normals by Box-Muller: element pair */
/* j of block b (row-major n-by-k, elements 2j and 2j+1) uses counter        */
/* (lo32 j, hi32 j, b, 0) and key (lo32 seed, hi32 seed); with words r0..r3, */
/* u1 = ((r0:r1) >> 11) 2^-53, u2 = ((r2:r3) >> 11) 2^-53,                   */
/* rho = sqrt(-2 log(1 - u1)), z0 = rho cos(2 pi u2), z1 = rho sin(2 pi u2).  */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9U; k1 += 0xBB67AE85U; }
        const uint64_t p0 = (uint64_t)0xD2511F53U * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57U * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void orc_random_block(int64_t n, int32_t k, uint64_t seed, uint32_t block, double *X)
{
    const int64_t total = n * (int64_t)k;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    const double two_pi = 6.283185307179586476925286766559;
    for (int64_t j = 0; 2 * j < total; ++j) {
        const uint32_t ctr[4] = {(uint32_t)j, (uint32_t)((uint64_t)j >> 32), block, 0};
        uint32_t r[4];
        orc_philox4x32_10(ctr, key, r);
        const double u1 = (double)(((((uint64_t)r[0]) << 32) | r[1]) >> 11) * 0x1.0p-53;
        const double u2 = (double)(((((uint64_t)r[2]) << 32) | r[3]) >> 11) * 0x1.0p-53;
        const double rho = sqrt(-2.0 * log(1.0 - u1));
        const double th = two_pi * u2;
        X[2 * j] = rho * cos(th);
        if (2 * j + 1 < total) X[2 * j + 1] = rho * sin(th);
    }
}
