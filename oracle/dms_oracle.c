/*
 * dms_oracle.c -- plain CPU oracle for the discrete-gradient step of
 * Discrete Morse Sandwich (global vertex order, Robins' ProcessLowerStars on
 * the Freudenthal triangulation of a 3D grid, critical-simplex extraction,
 * and the D0 extremum-saddle pairing used by the differentiable form).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or generator with the GPU library: the star tables below are
 * generated at run time from the Kuhn chain rule, independently of the GPU
 * side, and a test compares the two.
 *
 * Everything here is written to be checked by eye against the paper, not to
 * be fast: cell keys are explicit lists of vertex orders compared
 * lexicographically, priority queues are unsorted arrays scanned for their
 * minimum, and there is no blocking or fusion.
 *
 * Parity status of each function (what pins it) is stated above it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Kuhn (Freudenthal) star tables.                                          */
/*                                                                          */
/* Input data (Section 2.1): a regular grid is implicitly triangulated with */
/* the Freudenthal triangulation; the paper does not fix the diagonal.      */
/* Reading used here: the Kuhn triangulation along +(1,1,1).  A vertex set  */
/* is a simplex iff every pair of its offsets differs by a non-zero vector  */
/* in {0,1}^3 or in {0,-1}^3 (the triangulation is a flag complex).         */
/* The 14 neighbours of a vertex are therefore the offsets in              */
/* {0,1}^3 u {0,-1}^3 minus the origin, numbered in (dz, dy, dx)            */
/* lexicographic order, which is the order of their linear memory offsets.  */
/* Pinned by: star counts 14/36/24, link Euler characteristic 2, whole-grid */
/* simplex counts in closed form (tests/test_oracle_tables.py).            */
/* ------------------------------------------------------------------------ */

static int NB[14][3];          /* (dx, dy, dz) of neighbour e              */
static int TRI[36][2];         /* star triangle {x, a, b}, a < b            */
static int TET[24][3];         /* star tet {x, a, b, c}, a < b < c          */
static int TRI_ID[14][14];     /* triangle index of {a, b}, or -1           */
static int EDGE_TRIS[14][6];   /* star triangles containing edge e, ascending */
static int EDGE_NTRI[14];
static int TRI_TETS[36][2];    /* the two star tets containing triangle t   */
static int TRI_NTET[36];
static int TET_TRIS[24][3];    /* facets of tet q that contain x            */
static int tables_built = 0;

static int offsets_compatible(const int *a, const int *b)
{
    /* a - b must be a non-zero vector with all components in {0,1} or all
     * components in {0,-1}. */
    int pos = 0, neg = 0, nz = 0;
    for (int c = 0; c < 3; ++c) {
        int d = a[c] - b[c];
        if (d > 1 || d < -1) return 0;
        if (d == 1) pos = 1;
        if (d == -1) neg = 1;
        if (d != 0) nz = 1;
    }
    return nz && !(pos && neg);
}

static void build_tables(void)
{
    if (tables_built) return;
    static const int origin[3] = {0, 0, 0};
    int n = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int o[3] = {dx, dy, dz};
                if (offsets_compatible(o, origin)) {
                    NB[n][0] = dx; NB[n][1] = dy; NB[n][2] = dz;
                    ++n;
                }
            }
    for (int a = 0; a < 14; ++a)
        for (int b = 0; b < 14; ++b) TRI_ID[a][b] = -1;
    int nt = 0;
    for (int a = 0; a < 14; ++a)
        for (int b = a + 1; b < 14; ++b)
            if (offsets_compatible(NB[a], NB[b])) {
                TRI[nt][0] = a; TRI[nt][1] = b;
                TRI_ID[a][b] = TRI_ID[b][a] = nt;
                ++nt;
            }
    int nq = 0;
    for (int a = 0; a < 14; ++a)
        for (int b = a + 1; b < 14; ++b)
            for (int c = b + 1; c < 14; ++c)
                if (offsets_compatible(NB[a], NB[b]) && offsets_compatible(NB[a], NB[c]) &&
                    offsets_compatible(NB[b], NB[c])) {
                    TET[nq][0] = a; TET[nq][1] = b; TET[nq][2] = c;
                    ++nq;
                }
    for (int e = 0; e < 14; ++e) EDGE_NTRI[e] = 0;
    for (int t = 0; t < nt; ++t)
        for (int s = 0; s < 2; ++s) {
            int e = TRI[t][s];
            EDGE_TRIS[e][EDGE_NTRI[e]++] = t;
        }
    for (int t = 0; t < nt; ++t) TRI_NTET[t] = 0;
    for (int q = 0; q < nq; ++q) {
        int a = TET[q][0], b = TET[q][1], c = TET[q][2];
        TET_TRIS[q][0] = TRI_ID[a][b];
        TET_TRIS[q][1] = TRI_ID[a][c];
        TET_TRIS[q][2] = TRI_ID[b][c];
        for (int s = 0; s < 3; ++s) {
            int t = TET_TRIS[q][s];
            TRI_TETS[t][TRI_NTET[t]++] = q;
        }
    }
    /* The counts are checked by the tests through oracle_star_tables(). */
    tables_built = (n == 14 && nt == 36 && nq == 24) ? 1 : -1;
}

/* Copies the tables out so that tests can pin them and compare them with the
 * GPU library's own tables.  Returns 0, or -1 if generation went wrong. */
int oracle_star_tables(int32_t *nb /*14*3*/, int32_t *tri /*36*2*/, int32_t *tet /*24*3*/,
                       int32_t *edge_tris /*14*6, -1 padded*/, int32_t *tri_tets /*36*2*/)
{
    build_tables();
    if (tables_built != 1) return -1;
    for (int e = 0; e < 14; ++e) {
        for (int c = 0; c < 3; ++c) nb[3 * e + c] = NB[e][c];
        for (int s = 0; s < 6; ++s) edge_tris[6 * e + s] = s < EDGE_NTRI[e] ? EDGE_TRIS[e][s] : -1;
    }
    for (int t = 0; t < 36; ++t) {
        tri[2 * t] = TRI[t][0]; tri[2 * t + 1] = TRI[t][1];
        tri_tets[2 * t] = TRI_TETS[t][0]; tri_tets[2 * t + 1] = TRI_TETS[t][1];
    }
    for (int q = 0; q < 24; ++q)
        for (int c = 0; c < 3; ++c) tet[3 * q + c] = TET[q][c];
    return 0;
}

/* ------------------------------------------------------------------------ */
/* O-1  Global vertex order (Section 2.1; Array Preconditioning, Section 3).*/
/*                                                                          */
/* Vertices are sorted by increasing value, ties broken by the vertex       */
/* offset in memory; order[v] is v's position in that sort.  -0.0 compares */
/* equal to +0.0 (it is the same real number); NaN has no place in a total  */
/* order and is rejected.  Pinned by: order is a permutation, a constant    */
/* field gives order == id, agreement with numpy's stable argsort, and the */
/* tie-heavy U[0,1) float32 field.                                         */
/* ------------------------------------------------------------------------ */

typedef struct { double v; int64_t id; } vid_t;

static int cmp_vid(const void *pa, const void *pb)
{
    const vid_t *a = (const vid_t *)pa, *b = (const vid_t *)pb;
    if (a->v < b->v) return -1;
    if (a->v > b->v) return 1;
    return (a->id < b->id) ? -1 : (a->id > b->id);
}

/* Number of threads a call uses: nthreads if positive, else every thread
 * OpenMP offers. */
static int threads_for(int nthreads)
{
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* Merges the sorted runs a[0, na) and b[0, nb) into out (a first on ties,
 * so the merge is stable). */
static void merge_runs(const vid_t *a, int64_t na, const vid_t *b, int64_t nb, vid_t *out)
{
    int64_t i = 0, j = 0, k = 0;
    while (i < na && j < nb) out[k++] = cmp_vid(&b[j], &a[i]) < 0 ? b[j++] : a[i++];
    while (i < na) out[k++] = a[i++];
    while (j < nb) out[k++] = b[j++];
}

/* Sorts the pairs by (value, id): with several threads, one qsort per run
 * of n / threads pairs, then rounds of pairwise merges of adjacent runs.
 * Returns 0, or 2 if the merge buffer cannot be allocated. */
static int sort_pairs(vid_t *p, int64_t n, int nthreads)
{
    int t = threads_for(nthreads);
    if (t <= 1 || n < 4096) {
        qsort(p, (size_t)n, sizeof(vid_t), cmp_vid);
        return 0;
    }
    int64_t *b = (int64_t *)malloc(sizeof(int64_t) * (size_t)(t + 1));
    vid_t *tmp = (vid_t *)malloc(sizeof(vid_t) * (size_t)n);
    if (!b || !tmp) { free(b); free(tmp); return 2; }
    for (int i = 0; i <= t; ++i) b[i] = n * i / t;
#pragma omp parallel for num_threads(t) schedule(static, 1)
    for (int i = 0; i < t; ++i) qsort(p + b[i], (size_t)(b[i + 1] - b[i]), sizeof(vid_t), cmp_vid);
    vid_t *src = p, *dst = tmp;
    for (int w = 1; w < t; w *= 2) {
#pragma omp parallel for num_threads(t) schedule(dynamic, 1)
        for (int i = 0; i < t; i += 2 * w) {
            int m = i + w < t ? i + w : t, e = i + 2 * w < t ? i + 2 * w : t;
            merge_runs(src + b[i], b[m] - b[i], src + b[m], b[e] - b[m], dst + b[i]);
        }
        vid_t *x = src; src = dst; dst = x;
    }
    if (src != p) memcpy(p, src, sizeof(vid_t) * (size_t)n);
    free(b);
    free(tmp);
    return 0;
}

static int order_from_pairs(vid_t *p, int64_t n, int32_t *order, int nthreads)
{
    if (sort_pairs(p, n, nthreads)) return 2;
    for (int64_t r = 0; r < n; ++r) order[p[r].id] = (int32_t)r;
    return 0;
}

/* nthreads: threads of the sort (0 = all).  Returns 0 on success, 1 if a
 * NaN was found, 2 on bad size / allocation. */
int oracle_order_f32(const float *values, int64_t n, int32_t *order, int nthreads)
{
    if (n < 0 || n > 2147483647LL) return 2;
    vid_t *p = (vid_t *)malloc(sizeof(vid_t) * (size_t)(n > 0 ? n : 1));
    if (!p) return 2;
    for (int64_t i = 0; i < n; ++i) {
        double v = (double)values[i]; /* exact widening */
        if (isnan(v)) { free(p); return 1; }
        p[i].v = (v == 0.0) ? 0.0 : v; /* -0.0 -> +0.0 */
        p[i].id = i;
    }
    int rc = order_from_pairs(p, n, order, nthreads);
    free(p);
    return rc;
}

int oracle_order_f64(const double *values, int64_t n, int32_t *order, int nthreads)
{
    if (n < 0 || n > 2147483647LL) return 2;
    vid_t *p = (vid_t *)malloc(sizeof(vid_t) * (size_t)(n > 0 ? n : 1));
    if (!p) return 2;
    for (int64_t i = 0; i < n; ++i) {
        double v = values[i];
        if (isnan(v)) { free(p); return 1; }
        p[i].v = (v == 0.0) ? 0.0 : v;
        p[i].id = i;
    }
    int rc = order_from_pairs(p, n, order, nthreads);
    free(p);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* O-3  ProcessLowerStars (Robins, Wood and Sheppard 2011, the gradient     */
/* algorithm the paper adopts in Section 2.3 and Section 3).                */
/*                                                                          */
/* For a vertex x, the lower star L(x) holds x and every simplex of the     */
/* star of x whose other vertices all precede x in the vertex order.  Cells */
/* are compared as in Section 2.1: list the vertex orders of a simplex in   */
/* decreasing order and compare the lists lexicographically (a proper       */
/* prefix is smaller).  The steps, in Robins' order:                       */
/*   - if L(x) = {x}, x is critical;                                        */
/*   - otherwise pair x with delta, the smallest edge of L(x); every other  */
/*     edge goes to PQzero; the cofacets of delta in L(x) with exactly one  */
/*     unpaired facet in L(x) go to PQone;                                  */
/*   - while either queue is non-empty: drain PQone (pop the smallest       */
/*     alpha; if it has no unpaired facet it moves to PQzero, otherwise it  */
/*     is paired with its only unpaired facet, which leaves PQzero, and the */
/*     cofacets of both with exactly one unpaired facet enter PQone); then  */
/*     pop the smallest still-unpaired cell of PQzero, declare it critical  */
/*     and push its cofacets with exactly one unpaired facet to PQone.      */
/*                                                                          */
/* Readings (where Robins' text leaves a choice):                           */
/*   - "unpaired" means neither paired nor critical;                        */
/*   - only unpaired cells are pushed to PQone; with literal != 0 the push  */
/*     ignores the cell's own state instead, and every case where the two   */
/*     readings could act differently is counted in *anomalies;             */
/*   - PQzero deletions are lazy (a popped cell that is no longer unpaired  */
/*     is skipped).                                                         */
/* Pinned by: matching property, acyclicity by brute force on small grids,  */
/* Euler characteristic, the ramp and separated-Gaussian counts, lower-link */
/* Betti numbers, textbook union-find D0 and boundary-matrix reduction      */
/* (tests/test_oracle_*.py).  The identity of the chosen pairs beyond those */
/* pins is parity unpinned.                                                 */
/* ------------------------------------------------------------------------ */

enum { ST_OUT = 0, ST_FREE = 1, ST_TAIL = 2, ST_HEAD = 3, ST_CRIT = 4 };

/* Cell numbering inside one lower star: 0 = x, 1..14 = edges,
 * 15..50 = triangles, 51..74 = tets. */
#define C_EDGE(e) (1 + (e))
#define C_TRI(t) (15 + (t))
#define C_TET(q) (51 + (q))
#define NCELL 75

typedef struct {
    int dim;          /* 0..3 */
    int inL;          /* member of L(x) */
    int nkey;         /* number of vertices */
    int64_t key[4];   /* vertex orders, decreasing */
    int state;
    int partner;      /* paired cell (cell number), -1 if none */
} cell_t;

static int key_less(const cell_t *a, const cell_t *b)
{
    int n = a->nkey < b->nkey ? a->nkey : b->nkey;
    for (int i = 0; i < n; ++i) {
        if (a->key[i] < b->key[i]) return 1;
        if (a->key[i] > b->key[i]) return 0;
    }
    return a->nkey < b->nkey; /* a proper prefix is smaller */
}

static void sort_desc(int64_t *k, int n)
{
    for (int i = 1; i < n; ++i) {
        int64_t v = k[i];
        int j = i - 1;
        while (j >= 0 && k[j] < v) { k[j + 1] = k[j]; --j; }
        k[j + 1] = v;
    }
}

/* facets of a cell that contain x, as cell numbers; returns their count */
static int facets_in_star(int c, int *out)
{
    if (c >= C_TET(0)) {
        int q = c - C_TET(0);
        for (int s = 0; s < 3; ++s) out[s] = C_TRI(TET_TRIS[q][s]);
        return 3;
    }
    if (c >= C_TRI(0)) {
        int t = c - C_TRI(0);
        out[0] = C_EDGE(TRI[t][0]);
        out[1] = C_EDGE(TRI[t][1]);
        return 2;
    }
    if (c >= C_EDGE(0)) { out[0] = 0; return 1; }
    return 0;
}

/* cofacets of a cell inside the star of x, as cell numbers */
static int cofacets_in_star(int c, int *out)
{
    if (c >= C_TET(0)) return 0;
    if (c >= C_TRI(0)) {
        int t = c - C_TRI(0);
        for (int s = 0; s < TRI_NTET[t]; ++s) out[s] = C_TET(TRI_TETS[t][s]);
        return TRI_NTET[t];
    }
    if (c >= C_EDGE(0)) {
        int e = c - C_EDGE(0);
        for (int s = 0; s < EDGE_NTRI[e]; ++s) out[s] = C_TRI(EDGE_TRIS[e][s]);
        return EDGE_NTRI[e];
    }
    return 0; /* x: its cofacets are the edges; never pushed to PQone */
}

static int count_free_facets(const cell_t *cells, int c, int *the_free)
{
    int f[4], nf = facets_in_star(c, f), k = 0;
    for (int s = 0; s < nf; ++s)
        if (cells[f[s]].inL && cells[f[s]].state == ST_FREE) { ++k; *the_free = f[s]; }
    return k;
}

typedef struct { int item[512]; int n; } queue_t;

static void q_push(queue_t *q, int c, int64_t *anomalies)
{
    if (q->n >= 512) { ++*anomalies; return; }
    q->item[q->n++] = c;
}

/* remove and return the entry with the smallest key; -1 if empty */
static int q_pop_min(queue_t *q, const cell_t *cells)
{
    if (q->n == 0) return -1;
    int best = 0;
    for (int i = 1; i < q->n; ++i)
        if (key_less(&cells[q->item[i]], &cells[q->item[best]])) best = i;
    int c = q->item[best];
    q->item[best] = q->item[--q->n];
    return c;
}

static void push_cofacets(queue_t *pq_one, cell_t *cells, int c, int literal, int64_t *anomalies)
{
    int co[8], nco = cofacets_in_star(c, co), dummy;
    for (int s = 0; s < nco; ++s) {
        cell_t *g = &cells[co[s]];
        if (!g->inL) continue;
        if (count_free_facets(cells, co[s], &dummy) != 1) continue;
        if (g->state != ST_FREE) {
            if (!literal) continue;
        }
        q_push(pq_one, co[s], anomalies);
    }
}

static void make_pair(cell_t *cells, int tail, int head)
{
    cells[tail].state = ST_TAIL; cells[tail].partner = head;
    cells[head].state = ST_HEAD; cells[head].partner = tail;
}

/*
 * Processes one lower star.  okey[0] is the order of x, okey[1 + e] the order
 * of neighbour e, or -1 if that neighbour lies outside the grid.  Orders only
 * need to be comparable (any strictly increasing relabelling gives the same
 * result).  Writes the cell states (ST_*) to states[75] if non-null and the
 * 128-bit record to rec[4] if non-null.
 *
 * Record layout (one 16-byte word per vertex, little-endian bit numbering):
 *   bits [4e, 4e+4), e = 0..13: edge e -- 0 not in L(x), 1 paired with x,
 *     2 critical, 3+j paired with the j-th star triangle containing e;
 *   bits [56+2t, 58+2t), t = 0..35: triangle t -- 0 not paired with a tet,
 *     1+j paired with the j-th star tet containing t.
 * Every other state follows from these fields.
 */
static void pls_one(const int64_t *okey, int literal, int64_t *anomalies, int8_t *states,
                    uint32_t *rec)
{
    cell_t cells[NCELL];
    int64_t ox = okey[0];
    memset(cells, 0, sizeof(cells));
    for (int c = 0; c < NCELL; ++c) cells[c].partner = -1;

    /* x itself */
    cells[0].dim = 0; cells[0].inL = 1; cells[0].nkey = 1; cells[0].key[0] = ox;
    int lower[14];
    for (int e = 0; e < 14; ++e) lower[e] = okey[1 + e] >= 0 && okey[1 + e] < ox;
    for (int e = 0; e < 14; ++e) {
        cell_t *c = &cells[C_EDGE(e)];
        c->dim = 1; c->inL = lower[e]; c->nkey = 2;
        c->key[0] = ox; c->key[1] = okey[1 + e];
    }
    for (int t = 0; t < 36; ++t) {
        cell_t *c = &cells[C_TRI(t)];
        int a = TRI[t][0], b = TRI[t][1];
        c->dim = 2; c->inL = lower[a] && lower[b]; c->nkey = 3;
        c->key[0] = ox; c->key[1] = okey[1 + a]; c->key[2] = okey[1 + b];
        sort_desc(c->key + 1, 2);
    }
    for (int q = 0; q < 24; ++q) {
        cell_t *c = &cells[C_TET(q)];
        int a = TET[q][0], b = TET[q][1], d = TET[q][2];
        c->dim = 3; c->inL = lower[a] && lower[b] && lower[d]; c->nkey = 4;
        c->key[0] = ox; c->key[1] = okey[1 + a]; c->key[2] = okey[1 + b]; c->key[3] = okey[1 + d];
        sort_desc(c->key + 1, 3);
    }
    for (int c = 0; c < NCELL; ++c) cells[c].state = cells[c].inL ? ST_FREE : ST_OUT;

    int delta = -1;
    for (int e = 0; e < 14; ++e)
        if (lower[e] && (delta < 0 || key_less(&cells[C_EDGE(e)], &cells[delta]))) delta = C_EDGE(e);

    if (delta < 0) {
        cells[0].state = ST_CRIT; /* L(x) = {x}: a minimum */
    } else {
        queue_t pq_zero, pq_one;
        pq_zero.n = 0; pq_one.n = 0;
        make_pair(cells, 0, delta);
        for (int e = 0; e < 14; ++e)
            if (lower[e] && C_EDGE(e) != delta) q_push(&pq_zero, C_EDGE(e), anomalies);
        push_cofacets(&pq_one, cells, delta, literal, anomalies);

        while (pq_one.n > 0 || pq_zero.n > 0) {
            while (pq_one.n > 0) {
                int a = q_pop_min(&pq_one, cells);
                int b = -1;
                int nf = count_free_facets(cells, a, &b);
                if (cells[a].state != ST_FREE) {
                    /* Only reachable when pushes ignore the state.  With no
                     * unpaired facet it would merely be skipped later; with one
                     * the literal steps would pair it a second time. */
                    if (nf != 0 || !literal) ++*anomalies;
                    if (nf == 0) q_push(&pq_zero, a, anomalies);
                    continue;
                }
                if (nf == 0) {
                    q_push(&pq_zero, a, anomalies);
                } else {
                    if (nf != 1) ++*anomalies; /* cannot happen: pushed with one */
                    make_pair(cells, b, a);    /* b leaves PQzero lazily */
                    push_cofacets(&pq_one, cells, a, literal, anomalies);
                    push_cofacets(&pq_one, cells, b, literal, anomalies);
                }
            }
            int g = -1;
            while (pq_zero.n > 0) {
                int c = q_pop_min(&pq_zero, cells);
                if (cells[c].state == ST_FREE) { g = c; break; }
            }
            if (g >= 0) {
                cells[g].state = ST_CRIT;
                push_cofacets(&pq_one, cells, g, literal, anomalies);
            }
        }
        for (int c = 0; c < NCELL; ++c)
            if (cells[c].state == ST_FREE) ++*anomalies; /* every cell must end decided */
    }

    if (states)
        for (int c = 0; c < NCELL; ++c) states[c] = (int8_t)cells[c].state;

    if (rec) {
        uint32_t w[4] = {0, 0, 0, 0};
        for (int e = 0; e < 14; ++e) {
            const cell_t *c = &cells[C_EDGE(e)];
            uint32_t v = 0;
            if (c->inL) {
                if (c->state == ST_HEAD) v = 1;        /* paired with x */
                else if (c->state == ST_CRIT) v = 2;
                else if (c->state == ST_TAIL) {
                    int t = c->partner - C_TRI(0);
                    int j = 0;
                    while (EDGE_TRIS[e][j] != t) ++j;
                    v = 3 + (uint32_t)j;
                }
            }
            int bit = 4 * e;
            w[bit / 32] |= v << (bit % 32);
        }
        for (int t = 0; t < 36; ++t) {
            const cell_t *c = &cells[C_TRI(t)];
            uint32_t v = 0;
            if (c->inL && c->state == ST_TAIL) {
                int q = c->partner - C_TET(0);
                v = (TRI_TETS[t][0] == q) ? 1 : 2;
            }
            int bit = 56 + 2 * t;
            w[bit / 32] |= v << (bit % 32);
        }
        for (int i = 0; i < 4; ++i) rec[i] = w[i];
    }
}

/* One lower star from explicit keys (tests use this for hand-built cases). */
int oracle_pls_local(const int64_t *okey /*15*/, int literal, int8_t *states /*75*/,
                     uint32_t *rec /*4*/, int64_t *anomalies)
{
    build_tables();
    if (tables_built != 1) return -1;
    int64_t an = 0;
    pls_one(okey, literal, &an, states, rec);
    if (anomalies) *anomalies += an;
    return 0;
}

/*
 * Many lower stars from explicit keys: keys holds m rows of 15 small keys
 * (x, then neighbours 0..13; 255 = the neighbour is absent), rec receives 4
 * words per row.  Each row is one pls_one call, as oracle_pls_local makes
 * it; nthreads threads (0 = all) share the rows.  Returns 0, or -1.
 */
int oracle_pls_batch(const uint8_t *keys, int64_t m, uint32_t *rec, int nthreads,
                     int64_t *anomalies)
{
    build_tables();
    if (tables_built != 1 || m < 0) return -1;
    int64_t an = 0;
    int nt = threads_for(nthreads);
#pragma omp parallel for num_threads(nt) schedule(dynamic, 1024) reduction(+ : an)
    for (int64_t r = 0; r < m; ++r) {
        int64_t okey[15];
        for (int u = 0; u < 15; ++u) okey[u] = keys[15 * r + u] == 255 ? -1 : (int64_t)keys[15 * r + u];
        pls_one(okey, 0, &an, NULL, rec + 4 * r);
    }
    if (anomalies) *anomalies += an;
    return 0;
}

static int box_ok(const int64_t *dims, const int64_t *lo, const int64_t *hi)
{
    for (int c = 0; c < 3; ++c) {
        if (dims[c] < 1) return 0;
        if (lo[c] < 0 || hi[c] > dims[c] || lo[c] > hi[c]) return 0;
    }
    return 1;
}

/* Gathers the keys of x = (i, j, k) and its 14 neighbours from order[]. */
static void gather_keys(const int32_t *order, const int64_t *dims, int64_t i, int64_t j, int64_t k,
                        int64_t *okey)
{
    int64_t nx = dims[0], ny = dims[1], nz = dims[2];
    okey[0] = order[i + nx * (j + ny * k)];
    for (int e = 0; e < 14; ++e) {
        int64_t a = i + NB[e][0], b = j + NB[e][1], c = k + NB[e][2];
        if (a < 0 || b < 0 || c < 0 || a >= nx || b >= ny || c >= nz) okey[1 + e] = -1;
        else okey[1 + e] = order[a + nx * (b + ny * c)];
    }
}

/*
 * ProcessLowerStars over every vertex of the half-open box [lo, hi) of a grid
 * of dims (nx, ny, nz) (vertex id = i + nx*(j + ny*k)).  Neighbours outside
 * the box but inside the grid (a ghost layer) are read, not processed.
 * rec receives 4 words per box vertex, x fastest over the box.  counts[4]
 * receives the number of critical cells of each dimension.  Returns 0, or
 * -1 for bad arguments.
 */
int oracle_lower_stars(const int32_t *order, const int64_t *dims, const int64_t *lo,
                       const int64_t *hi, uint32_t *rec, int64_t *counts, int literal,
                       int nthreads, int64_t *anomalies)
{
    build_tables();
    if (tables_built != 1 || !box_ok(dims, lo, hi)) return -1;
    int64_t w0 = hi[0] - lo[0], w1 = hi[1] - lo[1], w2 = hi[2] - lo[2];
    int64_t c0 = 0, c1 = 0, c2 = 0, c3 = 0, an = 0;
    int nt = threads_for(nthreads);
    int64_t rows = w1 * w2;
#pragma omp parallel for num_threads(nt) schedule(dynamic, 4) reduction(+ : c0, c1, c2, c3, an)
    for (int64_t r = 0; r < rows; ++r) {
        int64_t j = lo[1] + r % w1, k = lo[2] + r / w1;
        for (int64_t i = lo[0]; i < hi[0]; ++i) {
            int64_t okey[15];
            int8_t st[NCELL];
            gather_keys(order, dims, i, j, k, okey);
            int64_t idx = (i - lo[0]) + w0 * r;
            pls_one(okey, literal, &an, st, rec ? rec + 4 * idx : NULL);
            for (int c = 0; c < NCELL; ++c)
                if (st[c] == ST_CRIT) {
                    if (c == 0) ++c0;
                    else if (c < C_TRI(0)) ++c1;
                    else if (c < C_TET(0)) ++c2;
                    else ++c3;
                }
        }
    }
    if (counts) { counts[0] = c0; counts[1] = c1; counts[2] = c2; counts[3] = c3; }
    if (anomalies) *anomalies += an;
    return 0;
}

/*
 * ProcessLowerStars at sampled vertices, straight from the values: the
 * orders of x and its neighbours are replaced by their ranks among those 15
 * vertices under the (value, id) comparison of Section 2.1, which is the
 * same relative order the global order gives.  dtype 0 = float32,
 * 1 = float64.  rec receives 4 words per sample.  Returns 0, -1 on bad
 * arguments, 1 if a NaN is met.
 */
int oracle_lower_stars_sampled(const void *values, int dtype, const int64_t *dims,
                               const int64_t *vids, int64_t m, uint32_t *rec, int nthreads,
                               int64_t *anomalies)
{
    build_tables();
    if (tables_built != 1 || dims[0] < 1 || dims[1] < 1 || dims[2] < 1) return -1;
    int64_t nx = dims[0], ny = dims[1], nz = dims[2], n = nx * ny * nz;
    int64_t an = 0;
    int nan_seen = 0, bad = 0;
    int nt = threads_for(nthreads);
#pragma omp parallel for num_threads(nt) schedule(dynamic, 64) reduction(+ : an) reduction(| : nan_seen, bad)
    for (int64_t s = 0; s < m; ++s) {
        int64_t v = vids[s];
        if (v < 0 || v >= n) { bad = 1; continue; }
        int64_t i = v % nx, j = (v / nx) % ny, k = v / (nx * ny);
        int64_t id[15];
        double val[15];
        int present[15];
        id[0] = v;
        for (int e = 0; e < 14; ++e) {
            int64_t a = i + NB[e][0], b = j + NB[e][1], c = k + NB[e][2];
            present[1 + e] = !(a < 0 || b < 0 || c < 0 || a >= nx || b >= ny || c >= nz);
            id[1 + e] = present[1 + e] ? a + nx * (b + ny * c) : -1;
        }
        present[0] = 1;
        for (int u = 0; u < 15; ++u) {
            if (!present[u]) { val[u] = 0.0; continue; }
            double x = dtype == 0 ? (double)((const float *)values)[id[u]]
                                  : ((const double *)values)[id[u]];
            if (isnan(x)) nan_seen = 1;
            val[u] = (x == 0.0) ? 0.0 : x;
        }
        int64_t okey[15];
        for (int u = 0; u < 15; ++u) {
            if (!present[u]) { okey[u] = -1; continue; }
            int64_t r = 0;
            for (int w = 0; w < 15; ++w) {
                if (!present[w] || w == u) continue;
                if (val[w] < val[u] || (val[w] == val[u] && id[w] < id[u])) ++r;
            }
            okey[u] = r;
        }
        pls_one(okey, 0, &an, NULL, rec + 4 * s);
    }
    if (anomalies) *anomalies += an;
    if (bad) return -1;
    return nan_seen ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* O-4  Critical-simplex extraction, the zero-persistence skip (Section     */
/* 2.6): a cell of L(x) that is neither tail nor head of a discrete vector  */
/* is critical.  Decodes the records only (no order is re-read).  Codes are */
/* (max vertex id << 8) | index in that vertex's star table of the cell's   */
/* dimension, listed in (max vertex id, index) order.  Pinned by: c0 equals */
/* the number of vertices with no lower neighbour, Euler characteristic 1,  */
/* and agreement with the states ProcessLowerStars itself reports.          */
/* ------------------------------------------------------------------------ */

static void decode_record(const uint32_t *w, int8_t *st)
{
    int ef[14], tf[36];
    for (int e = 0; e < 14; ++e) { int b = 4 * e; ef[e] = (int)((w[b / 32] >> (b % 32)) & 15u); }
    for (int t = 0; t < 36; ++t) { int b = 56 + 2 * t; tf[t] = (int)((w[b / 32] >> (b % 32)) & 3u); }
    int any = 0;
    for (int e = 0; e < 14; ++e) if (ef[e]) any = 1;
    st[0] = any ? ST_TAIL : ST_CRIT;
    int tri_head[36] = {0}, tet_head[24] = {0};
    for (int e = 0; e < 14; ++e)
        if (ef[e] >= 3) tri_head[EDGE_TRIS[e][ef[e] - 3]] = 1;
    for (int t = 0; t < 36; ++t)
        if (tf[t]) tet_head[TRI_TETS[t][tf[t] - 1]] = 1;
    for (int e = 0; e < 14; ++e)
        st[C_EDGE(e)] = ef[e] == 0 ? ST_OUT : ef[e] == 1 ? ST_HEAD : ef[e] == 2 ? ST_CRIT : ST_TAIL;
    for (int t = 0; t < 36; ++t) {
        int in = ef[TRI[t][0]] && ef[TRI[t][1]];
        st[C_TRI(t)] = !in ? ST_OUT : tf[t] ? ST_TAIL : tri_head[t] ? ST_HEAD : ST_CRIT;
    }
    for (int q = 0; q < 24; ++q) {
        int in = ef[TET[q][0]] && ef[TET[q][1]] && ef[TET[q][2]];
        st[C_TET(q)] = !in ? ST_OUT : tet_head[q] ? ST_HEAD : ST_CRIT;
    }
}

/* Decodes one record into 75 cell states (tests). */
int oracle_decode_record(const uint32_t *rec, int8_t *states)
{
    build_tables();
    if (tables_built != 1) return -1;
    decode_record(rec, states);
    return 0;
}

/* Visits the records of one row (j, k) of box [lo, hi): cnt[d] counts its
 * critical cells of dimension d, and when crit is non-null each is written
 * to crit[d][base[d] + its number in the row] if below cap[d]. */
static void critical_row(const uint32_t *rec, const int64_t *dims, const int64_t *lo, const int64_t *hi,
                         int64_t j, int64_t k, int64_t *const *crit, const int64_t *cap,
                         const int64_t *base, int64_t *cnt)
{
    int64_t nx = dims[0], ny = dims[1];
    int64_t w0 = hi[0] - lo[0], w1 = hi[1] - lo[1];
    for (int d = 0; d < 4; ++d) cnt[d] = 0;
    for (int64_t i = lo[0]; i < hi[0]; ++i) {
        int64_t idx = (i - lo[0]) + w0 * ((j - lo[1]) + w1 * (k - lo[2]));
        int64_t v = i + nx * (j + ny * k);
        int8_t st[NCELL];
        decode_record(rec + 4 * idx, st);
        for (int c = 0; c < NCELL; ++c) {
            if (st[c] != ST_CRIT) continue;
            int d = c == 0 ? 0 : c < C_TRI(0) ? 1 : c < C_TET(0) ? 2 : 3;
            int local = c == 0 ? 0 : c < C_TRI(0) ? c - C_EDGE(0)
                                   : c < C_TET(0) ? c - C_TRI(0) : c - C_TET(0);
            if (crit && crit[d] && base[d] + cnt[d] < cap[d]) crit[d][base[d] + cnt[d]] = (v << 8) | local;
            ++cnt[d];
        }
    }
}

/*
 * Lists the critical cells of the records of box [lo, hi), in vertex-id
 * order.  crit[d] (host arrays, may be NULL) receive at most cap[d] codes;
 * counts[d] always receives the full count.  With several threads (nthreads,
 * 0 = all) the rows of the box are counted first, their counts summed in row
 * order into each row's first slot, and then every row writes its own
 * slots.  Returns 0, -1 for bad arguments, -2 if memory runs out.
 */
int oracle_critical_simplices(const uint32_t *rec, const int64_t *dims, const int64_t *lo,
                              const int64_t *hi, int64_t *crit0, int64_t *crit1, int64_t *crit2,
                              int64_t *crit3, const int64_t *cap, int64_t *counts, int nthreads)
{
    build_tables();
    if (tables_built != 1 || !box_ok(dims, lo, hi)) return -1;
    int64_t *crit[4] = {crit0, crit1, crit2, crit3};
    int64_t w1 = hi[1] - lo[1], w2 = hi[2] - lo[2], rows = w1 * w2;
    int64_t *rc = (int64_t *)malloc(sizeof(int64_t) * 4 * (size_t)(rows + 1));
    if (!rc) return -2;
    int nt = threads_for(nthreads);
#pragma omp parallel for num_threads(nt) schedule(dynamic, 16)
    for (int64_t r = 0; r < rows; ++r)
        critical_row(rec, dims, lo, hi, lo[1] + r % w1, lo[2] + r / w1, NULL, cap, NULL, rc + 4 * (r + 1));
    for (int d = 0; d < 4; ++d) rc[d] = 0;
    for (int64_t r = 1; r <= rows; ++r)
        for (int d = 0; d < 4; ++d) rc[4 * r + d] += rc[4 * (r - 1) + d]; /* rc[4 r] = first slots of row r */
    for (int d = 0; d < 4; ++d) counts[d] = rc[4 * rows + d];
#pragma omp parallel for num_threads(nt) schedule(dynamic, 16)
    for (int64_t r = 0; r < rows; ++r) {
        int64_t cnt[4];
        critical_row(rec, dims, lo, hi, lo[1] + r % w1, lo[2] + r / w1, crit, cap, rc + 4 * r, cnt);
    }
    free(rc);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* O-6  D0 pairing from the gradient (Section 2.6 and Algorithm 1           */
/* PairExtremaSaddles), on a whole grid (records of every vertex).          */
/*   - For each critical edge sigma, follow the gradient down from each of  */
/*     its two vertices until a critical vertex: t0 from the edge's higher  */
/*     vertex, t1 from the other.  Keep (sigma, t0, t1) if t0 != t1.        */
/*   - Visit the kept triplets in increasing order of sigma (Section 2.1    */
/*     comparison).  r0, r1 = representatives of t0, t1; if they differ,    */
/*     make r0 the one with the higher order, pair (sigma, r0), and set the */
/*     representative of r0 and of t0 to r1.                                */
/* The one minimum that stays unpaired is the infinite class (Section 3).   */
/* Pinned by: #pairs = c0 - 1 on a connected grid, and equality with the    */
/* textbook union-find D0 of all edges restricted to non-zero persistence  */
/* (tests/test_oracle_d0.py).                                               */
/* ------------------------------------------------------------------------ */

static int64_t descend(const uint32_t *rec, const int64_t *dims, int64_t v)
{
    int64_t nx = dims[0], ny = dims[1];
    for (;;) {
        const uint32_t *w = rec + 4 * v;
        int delta = -1;
        for (int e = 0; e < 14; ++e) {
            int b = 4 * e;
            if (((w[b / 32] >> (b % 32)) & 15u) == 1u) delta = e;
        }
        if (delta < 0) return v; /* critical vertex */
        v += NB[delta][0] + nx * (NB[delta][1] + ny * NB[delta][2]);
    }
}

typedef struct { int64_t k0, k1; int64_t sigma, t0, t1; } trip_t;

static int cmp_trip(const void *pa, const void *pb)
{
    const trip_t *a = (const trip_t *)pa, *b = (const trip_t *)pb;
    if (a->k0 != b->k0) return a->k0 < b->k0 ? -1 : 1;
    if (a->k1 != b->k1) return a->k1 < b->k1 ? -1 : 1;
    return 0;
}

int oracle_d0_pairs(const int32_t *order, const uint32_t *rec, const int64_t *dims,
                    const int64_t *crit1, int64_t n1, int64_t *pair_edge, int64_t *pair_min,
                    int64_t *npairs)
{
    build_tables();
    if (tables_built != 1) return -1;
    int64_t nx = dims[0], ny = dims[1], n = dims[0] * dims[1] * dims[2];
    trip_t *tr = (trip_t *)malloc(sizeof(trip_t) * (size_t)(n1 > 0 ? n1 : 1));
    int64_t *rep = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!tr || !rep) { free(tr); free(rep); return -2; }
    int64_t nt = 0;
    for (int64_t s = 0; s < n1; ++s) {
        int64_t a = crit1[s] >> 8;
        int e = (int)(crit1[s] & 255);
        int64_t b = a + NB[e][0] + nx * (NB[e][1] + ny * NB[e][2]);
        int64_t t0 = descend(rec, dims, a), t1 = descend(rec, dims, b);
        if (t0 == t1) continue;
        tr[nt].k0 = order[a]; tr[nt].k1 = order[b];
        tr[nt].sigma = crit1[s]; tr[nt].t0 = t0; tr[nt].t1 = t1;
        ++nt;
    }
    qsort(tr, (size_t)nt, sizeof(trip_t), cmp_trip);
    for (int64_t v = 0; v < n; ++v) rep[v] = v;
    int64_t np = 0;
    for (int64_t s = 0; s < nt; ++s) {
        int64_t r0 = tr[s].t0, r1 = tr[s].t1;
        while (rep[r0] != r0) r0 = rep[r0];
        while (rep[r1] != r1) r1 = rep[r1];
        if (r0 == r1) continue;
        if (order[r0] < order[r1]) { int64_t t = r0; r0 = r1; r1 = t; }
        pair_edge[np] = tr[s].sigma;
        pair_min[np] = r0;
        ++np;
        rep[r0] = r1;
        rep[tr[s].t0] = r1;
    }
    *npairs = np;
    free(tr);
    free(rep);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* O-7  Critical cells in filtration order (Section 2.1).  Two cells of one */
/* dimension compare by the lists of their vertex orders, each sorted       */
/* decreasingly, lexicographically; distinct cells have distinct lists, so  */
/* the sorted result is unique.  Input codes are (maxv << 8) | local index  */
/* as O-5 writes them: local index 0 for a vertex, neighbour e of maxv for  */
/* an edge, star triangle t for a triangle, star tet q for a tet.           */
/* Returns -3 for a code that names no cell of the grid.                    */
/* Pinned by: for vertices it is the sort by order (numpy argsort); a       */
/* hand-worked 2x2x2 example (tests/golden/filtration_cube2.*) with ties    */
/* broken at the second, third and fourth entries; the output is a         */
/* permutation of the input with non-decreasing highest-vertex order        */
/* (tests/test_oracle_filtration.py).                                       */
/* ------------------------------------------------------------------------ */

typedef struct { int64_t key[4]; int64_t code; } fcell_t;

static int cmp_fcell(const void *pa, const void *pb)
{
    const fcell_t *a = (const fcell_t *)pa, *b = (const fcell_t *)pb;
    for (int i = 0; i < 4; ++i)
        if (a->key[i] != b->key[i]) return a->key[i] < b->key[i] ? -1 : 1;
    return 0;
}

/* vertex id of neighbour e of v, or -1 outside the grid */
static int64_t neighbour_of(const int64_t *dims, int64_t v, int e)
{
    int64_t nx = dims[0], ny = dims[1], nz = dims[2];
    int64_t x = v % nx, y = (v / nx) % ny, z = v / (nx * ny);
    int64_t a = x + NB[e][0], b = y + NB[e][1], c = z + NB[e][2];
    if (a < 0 || b < 0 || c < 0 || a >= nx || b >= ny || c >= nz) return -1;
    return a + nx * (b + ny * c);
}

int oracle_filtration_sort(const int32_t *order, const int64_t *dims, const int64_t *codes, int64_t n,
                           int dim, int64_t *out)
{
    build_tables();
    if (tables_built != 1) return -1;
    if (dim < 0 || dim > 3) return -3;
    int64_t nv = dims[0] * dims[1] * dims[2];
    fcell_t *c = (fcell_t *)malloc(sizeof(fcell_t) * (size_t)(n > 0 ? n : 1));
    if (!c) return -2;
    for (int64_t i = 0; i < n; ++i) {
        int64_t v = codes[i] >> 8;
        int loc = (int)(codes[i] & 255);
        int64_t vert[4] = {v, -1, -1, -1};
        int others[3] = {-1, -1, -1};
        if (v < 0 || v >= nv) { free(c); return -3; }
        if (dim == 0 && loc != 0) { free(c); return -3; }
        if (dim == 1) { if (loc >= 14) { free(c); return -3; } others[0] = loc; }
        if (dim == 2) { if (loc >= 36) { free(c); return -3; } others[0] = TRI[loc][0]; others[1] = TRI[loc][1]; }
        if (dim == 3) {
            if (loc >= 24) { free(c); return -3; }
            others[0] = TET[loc][0]; others[1] = TET[loc][1]; others[2] = TET[loc][2];
        }
        for (int k = 0; k < dim; ++k) {
            vert[k + 1] = neighbour_of(dims, v, others[k]);
            if (vert[k + 1] < 0) { free(c); return -3; }
        }
        for (int k = 0; k < 4; ++k) c[i].key[k] = k <= dim ? (int64_t)order[vert[k]] : -1;
        sort_desc(c[i].key, dim + 1);
        c[i].code = codes[i];
    }
    qsort(c, (size_t)n, sizeof(fcell_t), cmp_fcell);
    for (int64_t i = 0; i < n; ++i) out[i] = c[i].code;
    free(c);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* O-8  D2 pairing from the gradient (Section 2.6: D2 is computed like D0,   */
/* on the dual complex, where every discrete vector is reversed).  Reading: */
/* the dual graph has one node per tet plus one node for the outside of the */
/* grid; two tets sharing a triangle are adjacent, and a triangle on the    */
/* grid boundary joins its one tet to the outside node.                     */
/*   - A tet that is the head of a gradient pair (triangle s, tet) is left  */
/*     through s to the other tet containing s (the outside node if s is on */
/*     the boundary); a critical tet ends the walk (a maximum).             */
/*   - For each critical triangle sigma, walk from each of its cofacet tets */
/*     (the outside node for a missing one): t0, t1.  Keep (sigma, t0, t1)  */
/*     if t0 != t1.                                                         */
/*   - Visit the kept triplets in decreasing order of sigma (Section 2.1    */
/*     comparison).  r0, r1 = representatives of t0, t1; if they differ,    */
/*     make r0 the lower one (tets compared as in Section 2.1, the outside  */
/*     node above every tet), pair (sigma, r0), and set the representative  */
/*     of r0 and of t0 to r1.                                               */
/* Codes are (max vertex << 8) | local index, as O-5 writes them.           */
/* Pinned by: equality with the (triangle, tet) pairs of non-zero            */
/* persistence of a mod-2 boundary-matrix reduction of the lexicographic    */
/* filtration (tests/brute.py) on small grids; #pairs = c3 (every maximum   */
/* dies: the grid is a ball); empty on flat grids (tests/test_oracle_d2.py).*/
/* ------------------------------------------------------------------------ */

#define D2_OUTSIDE (-1)

/* neighbour index e with to = from + NB[e], or -1 */
static int nb_index(const int64_t *dims, int64_t from, int64_t to)
{
    for (int e = 0; e < 14; ++e)
        if (neighbour_of(dims, from, e) == to) return e;
    return -1;
}

static int64_t cell_code_of(const int32_t *order, const int64_t *dims, const int64_t *vs, int k)
{
    int m = 0;
    for (int i = 1; i < k; ++i)
        if (order[vs[i]] > order[vs[m]]) m = i;
    int es[3], ne = 0;
    for (int i = 0; i < k; ++i)
        if (i != m) es[ne++] = nb_index(dims, vs[m], vs[i]);
    for (int i = 0; i < ne; ++i)
        for (int j = i + 1; j < ne; ++j)
            if (es[j] < es[i]) { int t = es[i]; es[i] = es[j]; es[j] = t; }
    int loc = -1;
    if (k == 3) loc = TRI_ID[es[0]][es[1]];
    if (k == 4)
        for (int q = 0; q < 24; ++q)
            if (TET[q][0] == es[0] && TET[q][1] == es[1] && TET[q][2] == es[2]) loc = q;
    return (vs[m] << 8) | loc;
}

static void cell_vertices(const int64_t *dims, int64_t code, int k, int64_t *vs)
{
    int64_t v = code >> 8;
    int loc = (int)(code & 255);
    vs[0] = v;
    if (k == 3) { vs[1] = neighbour_of(dims, v, TRI[loc][0]); vs[2] = neighbour_of(dims, v, TRI[loc][1]); }
    if (k == 4)
        for (int i = 0; i < 3; ++i) vs[i + 1] = neighbour_of(dims, v, TET[loc][i]);
}

/* fourth vertices d of the tets containing triangle {a, b, c}, other than
 * `skip`; returns how many (at most 2) */
static int tri_cofacets(const int64_t *dims, const int64_t *abc, int64_t skip, int64_t *d)
{
    int n = 0;
    for (int e = 0; e < 14; ++e) {
        int64_t x = neighbour_of(dims, abc[0], e);
        if (x < 0 || x == abc[1] || x == abc[2] || x == skip) continue;
        if (nb_index(dims, abc[1], x) < 0 || nb_index(dims, abc[2], x) < 0) continue;
        if (n < 2) d[n] = x;
        ++n;
    }
    return n;
}

static int tri_state(const uint32_t *rec, int64_t v, int t)
{
    int b = 56 + 2 * t;
    return (int)((rec[4 * v + b / 32] >> (b % 32)) & 3u);
}

/* the maximum reached from tet `code`, or D2_OUTSIDE */
static int64_t ascend(const int32_t *order, const uint32_t *rec, const int64_t *dims, int64_t code)
{
    for (;;) {
        int64_t m = code >> 8;
        int q = (int)(code & 255);
        int tail = -1;
        for (int s = 0; s < 3; ++s) {
            int t = TET_TRIS[q][s];
            int g = tri_state(rec, m, t);
            if (g && TRI_TETS[t][g - 1] == q) tail = t;
        }
        if (tail < 0) return code; /* critical tet */
        int64_t tv[4], abc[3], d[2];
        cell_vertices(dims, code, 4, tv);
        abc[0] = m;
        abc[1] = neighbour_of(dims, m, TRI[tail][0]);
        abc[2] = neighbour_of(dims, m, TRI[tail][1]);
        int64_t fourth = -1;
        for (int i = 1; i < 4; ++i)
            if (tv[i] != abc[1] && tv[i] != abc[2]) fourth = tv[i];
        if (tri_cofacets(dims, abc, fourth, d) == 0) return D2_OUTSIDE;
        int64_t nv[4] = {abc[0], abc[1], abc[2], d[0]};
        code = cell_code_of(order, dims, nv, 4);
    }
}

typedef struct { int64_t key[3]; int64_t sigma, t0, t1; } trip2_t;

static int cmp_trip2_desc(const void *pa, const void *pb)
{
    const trip2_t *a = (const trip2_t *)pa, *b = (const trip2_t *)pb;
    for (int i = 0; i < 3; ++i)
        if (a->key[i] != b->key[i]) return a->key[i] > b->key[i] ? -1 : 1;
    return 0;
}

static int cmp_i64(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    return a < b ? -1 : a > b;
}

/* index of a maximum in the sorted list of critical tets; n3 for outside */
static int64_t max_index(const int64_t *sorted3, int64_t n3, int64_t code)
{
    if (code == D2_OUTSIDE) return n3;
    const int64_t *p = (const int64_t *)bsearch(&code, sorted3, (size_t)n3, sizeof(int64_t), cmp_i64);
    return p ? (int64_t)(p - sorted3) : -1;
}

/* Section 2.1 comparison of two maxima by index (n3 = the outside node) */
static int max_lower(const int32_t *order, const int64_t *dims, const int64_t *sorted3, int64_t n3,
                     int64_t a, int64_t b)
{
    if (a == n3) return 0;
    if (b == n3) return 1;
    int64_t va[4], vb[4], ka[4], kb[4];
    cell_vertices(dims, sorted3[a], 4, va);
    cell_vertices(dims, sorted3[b], 4, vb);
    for (int i = 0; i < 4; ++i) { ka[i] = order[va[i]]; kb[i] = order[vb[i]]; }
    sort_desc(ka, 4);
    sort_desc(kb, 4);
    for (int i = 0; i < 4; ++i)
        if (ka[i] != kb[i]) return ka[i] < kb[i];
    return 0;
}

int oracle_d2_pairs(const int32_t *order, const uint32_t *rec, const int64_t *dims, const int64_t *crit2,
                    int64_t n2, const int64_t *crit3, int64_t n3, int64_t *pair_tri, int64_t *pair_tet,
                    int64_t *npairs)
{
    build_tables();
    if (tables_built != 1) return -1;
    trip2_t *tr = (trip2_t *)malloc(sizeof(trip2_t) * (size_t)(n2 > 0 ? n2 : 1));
    int64_t *s3 = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n3 > 0 ? n3 : 1));
    int64_t *rep = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n3 + 1));
    if (!tr || !s3 || !rep) { free(tr); free(s3); free(rep); return -2; }
    for (int64_t i = 0; i < n3; ++i) s3[i] = crit3[i];
    qsort(s3, (size_t)n3, sizeof(int64_t), cmp_i64);
    int64_t nt = 0;
    for (int64_t s = 0; s < n2; ++s) {
        int64_t abc[3], d[2], t[2] = {D2_OUTSIDE, D2_OUTSIDE};
        cell_vertices(dims, crit2[s], 3, abc);
        int nc = tri_cofacets(dims, abc, -1, d);
        for (int c = 0; c < nc && c < 2; ++c) {
            int64_t tv[4] = {abc[0], abc[1], abc[2], d[c]};
            t[c] = ascend(order, rec, dims, cell_code_of(order, dims, tv, 4));
        }
        int64_t i0 = max_index(s3, n3, t[0]), i1 = max_index(s3, n3, t[1]);
        if (i0 < 0 || i1 < 0) { free(tr); free(s3); free(rep); return -3; }
        if (i0 == i1) continue;
        int64_t k[3] = {order[abc[0]], order[abc[1]], order[abc[2]]};
        sort_desc(k, 3);
        for (int i = 0; i < 3; ++i) tr[nt].key[i] = k[i];
        tr[nt].sigma = crit2[s];
        tr[nt].t0 = i0;
        tr[nt].t1 = i1;
        ++nt;
    }
    qsort(tr, (size_t)nt, sizeof(trip2_t), cmp_trip2_desc);
    for (int64_t i = 0; i <= n3; ++i) rep[i] = i;
    int64_t np = 0;
    for (int64_t s = 0; s < nt; ++s) {
        int64_t r0 = tr[s].t0, r1 = tr[s].t1;
        while (rep[r0] != r0) r0 = rep[r0];
        while (rep[r1] != r1) r1 = rep[r1];
        if (r0 == r1) continue;
        if (max_lower(order, dims, s3, n3, r1, r0)) { int64_t x = r0; r0 = r1; r1 = x; }
        pair_tri[np] = tr[s].sigma;
        pair_tet[np] = s3[r0];
        ++np;
        rep[r0] = r1;
        rep[tr[s].t0] = r1;
    }
    *npairs = np;
    free(tr);
    free(s3);
    free(rep);
    return 0;
}
