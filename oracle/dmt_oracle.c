/* Plain CPU oracle for the MSC-preserving correction stage (DMTz, arXiv 2409.17346).
 *
 * TEST INFRASTRUCTURE ONLY: used by tests, the smoke check and the benchmark's CPU
 * baseline leg, never by the product path.  Shares no code with the GPU library.
 *
 * Deliberately slow and literal: every step walks an explicit simplicial complex
 * (vertex lists + cofacet lists) in the order the paper describes.  Readings of
 * places where the paper is silent are marked "Reading:" in the comments.
 */
#include "dmt_oracle.h"

#include <assert.h>
#include <fenv.h>
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------------------------ */
/* Complex                                                                                     */

struct ocx {
    int top;
    int64_t nv;
    int64_t *key;           /* SoS key of each vertex */
    int64_t ncell[4];
    uint8_t *exists[4];
    int32_t *verts[4];      /* (d+1) ascending vertex indices per cell id */
    int64_t *cof_off[4];    /* cofacet CSR, for d < top */
    int64_t *cof[4];
    /* grid description (is_grid) */
    int is_grid;
    int64_t nx, ny, nz;
    int ntypes[4];
    int chain[4][16][3];    /* direction bits of the offsets a+c1, ..., a+cd of type t */
};

static void *xcalloc(size_t n, size_t s) {
    void *p = calloc(n ? n : 1, s);
    if (!p) abort();
    return p;
}

int ocx_top(const ocx *cx) { return cx->top; }
int64_t ocx_ncell(const ocx *cx, int d) { return (d < 0 || d > cx->top) ? 0 : cx->ncell[d]; }
int ocx_exists(const ocx *cx, int d, int64_t id) {
    if (d < 0 || d > cx->top || id < 0 || id >= cx->ncell[d]) return 0;
    return cx->exists[d][id];
}
int ocx_cell_vertices(const ocx *cx, int d, int64_t id, int32_t *out) {
    if (!ocx_exists(cx, d, id)) return -1;
    memcpy(out, cx->verts[d] + id * (d + 1), sizeof(int32_t) * (size_t)(d + 1));
    return 0;
}

/* Cell lookup from an ascending vertex list; -1 if no such cell. */
static int64_t lookup(const ocx *cx, int d, const int32_t *vs) {
    if (d == 0) return vs[0];
    if (cx->is_grid) {
        /* Freudenthal grid: the anchor is the componentwise minimum vertex, which is the
         * smallest vertex index; the other vertices are anchor + c_k with c_1 < ... < c_d a
         * strictly increasing chain of direction bit sets. */
        int64_t a = vs[0];
        int64_t ax = a % cx->nx, ay = (a / cx->nx) % cx->ny, az = a / (cx->nx * cx->ny);
        int c[3];
        for (int k = 1; k <= d; k++) {
            int64_t v = vs[k];
            int64_t dx = v % cx->nx - ax, dy = (v / cx->nx) % cx->ny - ay, dz = v / (cx->nx * cx->ny) - az;
            if (dx < 0 || dx > 1 || dy < 0 || dy > 1 || dz < 0 || dz > 1) return -1;
            c[k - 1] = (int)(dx + 2 * dy + 4 * dz);
        }
        for (int t = 0; t < cx->ntypes[d]; t++) {
            int ok = 1;
            for (int k = 0; k < d; k++) ok &= (cx->chain[d][t][k] == c[k]);
            if (ok) {
                int64_t id = a * cx->ntypes[d] + t;
                return cx->exists[d][id] ? id : -1;
            }
        }
        return -1;
    }
    for (int64_t id = 0; id < cx->ncell[d]; id++) {
        if (!cx->exists[d][id]) continue;
        if (memcmp(cx->verts[d] + id * (d + 1), vs, sizeof(int32_t) * (size_t)(d + 1)) == 0) return id;
    }
    return -1;
}

/* Cofacet lists, ascending by cofacet id: for every (d+1)-cell, register it with each facet. */
static void build_cofacets(ocx *cx) {
    for (int d = 0; d < cx->top; d++) {
        int64_t n = cx->ncell[d];
        int64_t *cnt = xcalloc((size_t)n + 1, sizeof(int64_t));
        int32_t fv[4];
        for (int pass = 0; pass < 2; pass++) {
            int64_t *fill = NULL;
            if (pass == 1) {
                cx->cof_off[d] = xcalloc((size_t)n + 1, sizeof(int64_t));
                for (int64_t i = 0; i < n; i++) cx->cof_off[d][i + 1] = cx->cof_off[d][i] + cnt[i];
                cx->cof[d] = xcalloc((size_t)cx->cof_off[d][n], sizeof(int64_t));
                fill = xcalloc((size_t)n, sizeof(int64_t));
            }
            for (int64_t t = 0; t < cx->ncell[d + 1]; t++) {
                if (!cx->exists[d + 1][t]) continue;
                const int32_t *tv = cx->verts[d + 1] + t * (d + 2);
                for (int skip = 0; skip <= d + 1; skip++) {
                    int m = 0;
                    for (int k = 0; k <= d + 1; k++)
                        if (k != skip) fv[m++] = tv[k];
                    int64_t fid = lookup(cx, d, fv);
                    assert(fid >= 0);
                    if (pass == 0) cnt[fid]++;
                    else cx->cof[d][cx->cof_off[d][fid] + fill[fid]++] = t;
                }
            }
            if (pass == 1) free(fill);
        }
        free(cnt);
    }
}

static void enumerate_types(ocx *cx) {
    int full = cx->top == 2 ? 3 : 7;
    for (int d = 1; d <= cx->top; d++) {
        int nt = 0;
        /* all chains 0 < c1 < c2 < ... (strict bitwise inclusion), lexicographic by value */
        for (int c1 = 1; c1 <= full; c1++) {
            if (d == 1) { cx->chain[1][nt][0] = c1; nt++; continue; }
            for (int c2 = c1 + 1; c2 <= full; c2++) {
                if ((c1 & ~c2) != 0) continue;
                if (d == 2) { cx->chain[2][nt][0] = c1; cx->chain[2][nt][1] = c2; nt++; continue; }
                for (int c3 = c2 + 1; c3 <= full; c3++) {
                    if ((c2 & ~c3) != 0) continue;
                    cx->chain[3][nt][0] = c1; cx->chain[3][nt][1] = c2; cx->chain[3][nt][2] = c3;
                    nt++;
                }
            }
        }
        cx->ntypes[d] = nt;
    }
    cx->ntypes[0] = 1;
}

ocx *ocx_grid(int64_t nx, int64_t ny, int64_t nz, const int64_t *key) {
    if (nx < 2 || ny < 2 || nz < 1 || nz == 0) return NULL;
    ocx *cx = xcalloc(1, sizeof(ocx));
    cx->is_grid = 1;
    cx->nx = nx; cx->ny = ny; cx->nz = nz;
    cx->top = nz == 1 ? 2 : 3;
    if (cx->top == 3 && nz < 2) { free(cx); return NULL; }
    cx->nv = nx * ny * nz;
    cx->key = xcalloc((size_t)cx->nv, sizeof(int64_t));
    for (int64_t v = 0; v < cx->nv; v++) cx->key[v] = key ? key[v] : v;
    enumerate_types(cx);
    for (int d = 0; d <= cx->top; d++) {
        int nt = cx->ntypes[d];
        cx->ncell[d] = cx->nv * nt;
        cx->exists[d] = xcalloc((size_t)cx->ncell[d], 1);
        cx->verts[d] = xcalloc((size_t)cx->ncell[d] * (size_t)(d + 1), sizeof(int32_t));
        for (int64_t a = 0; a < cx->nv; a++) {
            int64_t ax = a % nx, ay = (a / nx) % ny, az = a / (nx * ny);
            for (int t = 0; t < nt; t++) {
                int64_t id = a * nt + t;
                int32_t *vs = cx->verts[d] + id * (d + 1);
                vs[0] = (int32_t)a;
                int ok = 1;
                for (int k = 0; k < d; k++) {
                    int c = cx->chain[d][t][k];
                    int64_t x = ax + (c & 1), y = ay + ((c >> 1) & 1), z = az + ((c >> 2) & 1);
                    if (x >= nx || y >= ny || z >= nz) ok = 0;
                    vs[k + 1] = ok ? (int32_t)(x + nx * (y + ny * z)) : -1;
                }
                cx->exists[d][id] = (uint8_t)ok;
            }
        }
    }
    build_cofacets(cx);
    return cx;
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

ocx *ocx_explicit(int top, int64_t nv, const int64_t n[4], const int32_t *edges,
                  const int32_t *tris, const int32_t *tets) {
    if (top < 1 || top > 3 || nv < 1) return NULL;
    ocx *cx = xcalloc(1, sizeof(ocx));
    cx->top = top;
    cx->nv = nv;
    cx->key = xcalloc((size_t)nv, sizeof(int64_t));
    for (int64_t v = 0; v < nv; v++) cx->key[v] = v;
    const int32_t *src[4] = {NULL, edges, tris, tets};
    for (int d = 0; d <= top; d++) {
        int64_t m = d == 0 ? nv : n[d];
        cx->ncell[d] = m;
        cx->exists[d] = xcalloc((size_t)m, 1);
        cx->verts[d] = xcalloc((size_t)m * (size_t)(d + 1), sizeof(int32_t));
        for (int64_t i = 0; i < m; i++) {
            int32_t *vs = cx->verts[d] + i * (d + 1);
            if (d == 0) vs[0] = (int32_t)i;
            else {
                memcpy(vs, src[d] + i * (d + 1), sizeof(int32_t) * (size_t)(d + 1));
                qsort(vs, (size_t)(d + 1), sizeof(int32_t), cmp_i32);
            }
            cx->exists[d][i] = 1;
        }
    }
    build_cofacets(cx);
    return cx;
}

void ocx_free(ocx *cx) {
    if (!cx) return;
    for (int d = 0; d < 4; d++) {
        free(cx->exists[d]); free(cx->verts[d]); free(cx->cof_off[d]); free(cx->cof[d]);
    }
    free(cx->key);
    free(cx);
}

/* ------------------------------------------------------------------------------------------ */
/* Vertex order with simulation of simplicity (Section 4.1): larger key wins ties.             */

static int prec(const ocx *cx, const float *h, int64_t a, int64_t b) {
    return h[a] < h[b] || (h[a] == h[b] && cx->key[a] < cx->key[b]);
}

/* The vertex of the (d+1)-cell hi that is not a vertex of the d-cell lo. */
static int32_t apex_vertex(const ocx *cx, int d, int64_t lo, int64_t hi) {
    const int32_t *lv = cx->verts[d] + lo * (d + 1);
    const int32_t *hv = cx->verts[d + 1] + hi * (d + 2);
    for (int k = 0; k <= d + 1; k++) {
        int found = 0;
        for (int j = 0; j <= d; j++) found |= (hv[k] == lv[j]);
        if (!found) return hv[k];
    }
    abort();
}

/* ------------------------------------------------------------------------------------------ */
/* Discrete gradient (Section 3.1 "Gradient pairing", pairing rules of Section 4.2).           */
/* By increasing dimension: a cell already claimed by a facet is paired; otherwise it pairs   */
/* with the cofacet sigma+{x} whose added vertex x precedes every vertex of sigma, choosing   */
/* the smallest such x; with no such cofacet it is critical.  (Equation 1's extension makes   */
/* sigma the highest facet of sigma+{x} exactly when x is below all of sigma, and orders those */
/* cofacets by x.)                                                                             */

void oracle_gradient(const ocx *cx, const float *h, int64_t *up[4], int64_t *down[4]) {
    for (int d = 0; d <= cx->top; d++) {
        for (int64_t i = 0; i < cx->ncell[d]; i++) { up[d][i] = -1; down[d][i] = -1; }
    }
    for (int d = 0; d < cx->top; d++) {
        for (int64_t s = 0; s < cx->ncell[d]; s++) {
            if (!cx->exists[d][s]) continue;
            if (down[d][s] >= 0) continue;             /* claimed by a facet */
            const int32_t *sv = cx->verts[d] + s * (d + 1);
            int64_t best = -1;
            int32_t bestx = -1;
            for (int64_t k = cx->cof_off[d][s]; k < cx->cof_off[d][s + 1]; k++) {
                int64_t t = cx->cof[d][k];
                int32_t x = apex_vertex(cx, d, s, t);
                int below_all = 1;
                for (int j = 0; j <= d; j++) below_all &= prec(cx, h, x, sv[j]);
                if (!below_all) continue;
                if (best < 0 || prec(cx, h, x, bestx)) { best = t; bestx = x; }
            }
            if (best >= 0) {
                assert(down[d + 1][best] < 0);          /* a cofacet has one highest facet */
                up[d][s] = best;
                down[d + 1][best] = s;
            }
        }
    }
}

typedef struct {
    int64_t *up[4], *down[4];
} grad_t;

static void grad_alloc(const ocx *cx, grad_t *g) {
    memset(g, 0, sizeof(*g));
    for (int d = 0; d <= cx->top; d++) {
        g->up[d] = xcalloc((size_t)cx->ncell[d], sizeof(int64_t));
        g->down[d] = xcalloc((size_t)cx->ncell[d], sizeof(int64_t));
    }
}
static void grad_free(grad_t *g) {
    for (int d = 0; d < 4; d++) { free(g->up[d]); free(g->down[d]); }
}
static int is_crit(const ocx *cx, const grad_t *g, int d, int64_t i) {
    return cx->exists[d][i] && g->up[d][i] < 0 && g->down[d][i] < 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Morse-Smale complex (Section 3.1: critical cells and V-paths between them).                */

typedef struct { int64_t *p; int64_t n, cap; } vec;
static void vpush(vec *v, int64_t x) {
    if (v->n == v->cap) {
        v->cap = v->cap ? v->cap * 2 : 64;
        v->p = realloc(v->p, (size_t)v->cap * sizeof(int64_t));
        if (!v->p) abort();
    }
    v->p[v->n++] = x;
}

struct omsc {
    vec crit[4];
    vec dsad, doff, dcell, dterm;   /* descending branches (saddle -> minimum) */
    vec asad, aoff, acell, aterm;   /* ascending branches ((n-1)-saddle -> maximum) */
    int64_t *min_label, n_min_label;
    int64_t *max_label, n_max_label;
};

/* Descending V-path from vertex v: v, then the other end of v's paired edge, ... until a
 * critical vertex (a minimum). */
static int64_t walk_desc(const ocx *cx, const grad_t *g, int64_t v, vec *out) {
    for (;;) {
        if (out) vpush(out, v);
        int64_t e = g->up[0][v];
        if (e < 0) return v;
        const int32_t *ev = cx->verts[1] + e * 2;
        v = ev[0] == v ? ev[1] : ev[0];
    }
}

/* Ascending V-path from top cell T: a critical T ends it; otherwise go through T's paired
 * facet to that facet's other top cofacet.  Reading: a facet on the domain boundary has no
 * other cofacet, and the path ends at BOUNDARY (-1). */
static int64_t walk_asc(const ocx *cx, const grad_t *g, int64_t T, vec *out) {
    int n = cx->top;
    for (;;) {
        if (out) vpush(out, T);
        int64_t f = g->down[n][T];
        if (f < 0) return T;
        int64_t other = -1;
        for (int64_t k = cx->cof_off[n - 1][f]; k < cx->cof_off[n - 1][f + 1]; k++)
            if (cx->cof[n - 1][k] != T) other = cx->cof[n - 1][k];
        if (other < 0) return -1;
        T = other;
    }
}

static omsc *msc_from_grad(const ocx *cx, const grad_t *g) {
    omsc *m = xcalloc(1, sizeof(omsc));
    int n = cx->top;
    for (int d = 0; d <= n; d++)
        for (int64_t i = 0; i < cx->ncell[d]; i++)
            if (is_crit(cx, g, d, i)) vpush(&m->crit[d], i);
    /* descending: each 1-saddle, each endpoint in vertex order */
    vpush(&m->doff, 0);
    for (int64_t k = 0; k < m->crit[1].n; k++) {
        int64_t e = m->crit[1].p[k];
        for (int j = 0; j < 2; j++) {
            int64_t t = walk_desc(cx, g, cx->verts[1][e * 2 + j], &m->dcell);
            vpush(&m->dsad, e);
            vpush(&m->dterm, t);
            vpush(&m->doff, m->dcell.n);
        }
    }
    /* ascending: each (n-1)-saddle, each top cofacet in id order */
    vpush(&m->aoff, 0);
    for (int64_t k = 0; k < m->crit[n - 1].n; k++) {
        int64_t s = m->crit[n - 1].p[k];
        for (int64_t c = cx->cof_off[n - 1][s]; c < cx->cof_off[n - 1][s + 1]; c++) {
            int64_t t = walk_asc(cx, g, cx->cof[n - 1][c], &m->acell);
            vpush(&m->asad, s);
            vpush(&m->aterm, t);
            vpush(&m->aoff, m->acell.n);
        }
    }
    /* labels: terminal of every vertex's descending path / every top cell's ascending path.
     * Paths are followed until they meet a cell whose label is already known. */
    m->n_min_label = cx->nv;
    m->min_label = xcalloc((size_t)cx->nv, sizeof(int64_t));
    for (int64_t v = 0; v < cx->nv; v++) m->min_label[v] = -3;
    vec path = {0};
    for (int64_t v0 = 0; v0 < cx->nv; v0++) {
        path.n = 0;
        int64_t v = v0, lab;
        for (;;) {
            if (m->min_label[v] != -3) { lab = m->min_label[v]; break; }
            vpush(&path, v);
            int64_t e = g->up[0][v];
            if (e < 0) { lab = v; break; }
            const int32_t *ev = cx->verts[1] + e * 2;
            v = ev[0] == v ? ev[1] : ev[0];
        }
        for (int64_t i = 0; i < path.n; i++) m->min_label[path.p[i]] = lab;
    }
    m->n_max_label = cx->ncell[n];
    m->max_label = xcalloc((size_t)cx->ncell[n], sizeof(int64_t));
    for (int64_t T = 0; T < cx->ncell[n]; T++) m->max_label[T] = cx->exists[n][T] ? -3 : -2;
    for (int64_t T0 = 0; T0 < cx->ncell[n]; T0++) {
        if (!cx->exists[n][T0]) continue;
        path.n = 0;
        int64_t T = T0, lab;
        for (;;) {
            if (m->max_label[T] != -3) { lab = m->max_label[T]; break; }
            vpush(&path, T);
            int64_t f = g->down[n][T];
            if (f < 0) { lab = T; break; }
            int64_t other = -1;
            for (int64_t k = cx->cof_off[n - 1][f]; k < cx->cof_off[n - 1][f + 1]; k++)
                if (cx->cof[n - 1][k] != T) other = cx->cof[n - 1][k];
            if (other < 0) { lab = -1; break; }
            T = other;
        }
        for (int64_t i = 0; i < path.n; i++) m->max_label[path.p[i]] = lab;
    }
    free(path.p);
    return m;
}

omsc *oracle_msc(const ocx *cx, const float *h) {
    grad_t g;
    grad_alloc(cx, &g);
    oracle_gradient(cx, h, g.up, g.down);
    omsc *m = msc_from_grad(cx, &g);
    grad_free(&g);
    return m;
}

static const vec *omsc_vec(const omsc *m, int what) {
    switch (what) {
    case OMSC_CRIT0: case OMSC_CRIT1: case OMSC_CRIT2: case OMSC_CRIT3: return &m->crit[what];
    case OMSC_DESC_SADDLE: return &m->dsad;
    case OMSC_DESC_OFFSETS: return &m->doff;
    case OMSC_DESC_CELLS: return &m->dcell;
    case OMSC_DESC_TERMINAL: return &m->dterm;
    case OMSC_ASC_SADDLE: return &m->asad;
    case OMSC_ASC_OFFSETS: return &m->aoff;
    case OMSC_ASC_CELLS: return &m->acell;
    case OMSC_ASC_TERMINAL: return &m->aterm;
    default: return NULL;
    }
}
int64_t omsc_count(const omsc *m, int what) {
    if (what == OMSC_MIN_LABEL) return m->n_min_label;
    if (what == OMSC_MAX_LABEL) return m->n_max_label;
    const vec *v = omsc_vec(m, what);
    return v ? v->n : -1;
}
void omsc_copy(const omsc *m, int what, int64_t *dst) {
    if (what == OMSC_MIN_LABEL) { memcpy(dst, m->min_label, sizeof(int64_t) * (size_t)m->n_min_label); return; }
    if (what == OMSC_MAX_LABEL) { memcpy(dst, m->max_label, sizeof(int64_t) * (size_t)m->n_max_label); return; }
    const vec *v = omsc_vec(m, what);
    if (v && v->n) memcpy(dst, v->p, sizeof(int64_t) * (size_t)v->n);
}
void omsc_free(omsc *m) {
    if (!m) return;
    for (int d = 0; d < 4; d++) free(m->crit[d].p);
    free(m->dsad.p); free(m->doff.p); free(m->dcell.p); free(m->dterm.p);
    free(m->asad.p); free(m->aoff.p); free(m->acell.p); free(m->aterm.p);
    free(m->min_label); free(m->max_label);
    free(m);
}

/* ------------------------------------------------------------------------------------------ */
/* Bounds (problem statement, Section 4.1: |f - g| <= xi must hold exactly).                  */
/* Computed with the FPU's directed rounding modes: one correctly rounded subtraction toward  */
/* +inf gives the smallest fp32 at or above f - xi; one addition toward -inf gives the largest */
/* fp32 at or below f + xi.                                                                    */

void oracle_bounds(const float *f, int64_t n, float xi, float *lo, float *hi) {
    int old = fegetround();
    volatile float b = xi;
    fesetround(FE_UPWARD);
    for (int64_t i = 0; i < n; i++) { volatile float a = f[i]; volatile float r = a - b; lo[i] = r; }
    fesetround(FE_DOWNWARD);
    for (int64_t i = 0; i < n; i++) { volatile float a = f[i]; volatile float r = a + b; hi[i] = r; }
    fesetround(old);
}

void oracle_decode(const float *g_hat, const uint8_t *q, int64_t n, const int64_t *idx,
                   const float *val, int64_t n_lossless, float xi, int q_max, float *g_out) {
    float delta = ldexpf(xi, -q_max);
    for (int64_t i = 0; i < n; i++)
        g_out[i] = q[i] == 0xFF ? g_hat[i] : fmaf(-(float)q[i], delta, g_hat[i]);
    for (int64_t k = 0; k < n_lossless; k++) g_out[idx[k]] = val[k];
}

/* ------------------------------------------------------------------------------------------ */
/* Correction loop (Sections 4.2-4.6).                                                         */

typedef struct {
    const ocx *cx;
    const float *f, *ghat;
    float *g;          /* current edited field g^(k) */
    float *lo;         /* floor: smallest fp32 >= f - xi */
    uint8_t *q;        /* quantized edit count */
    uint8_t *floored;  /* edited to the floor (stored losslessly) */
    uint8_t *req;      /* vertices requested this iteration */
    float delta;
    int q_max;
} state_t;

/* Apex of the pair (sigma, tau) that cell (d, c) belongs to in gradient G, and that pair's
 * lower cell.  Returns -1 if the cell is critical. */
static int32_t pair_apex(const ocx *cx, const grad_t *G, int d, int64_t c, int *lo_d, int64_t *lo_id) {
    if (G->up[d][c] >= 0) { *lo_d = d; *lo_id = c; return apex_vertex(cx, d, c, G->up[d][c]); }
    if (d > 0 && G->down[d][c] >= 0) {
        *lo_d = d - 1; *lo_id = G->down[d][c];
        return apex_vertex(cx, d - 1, G->down[d][c], c);
    }
    return -1;
}

/* C-loop detection (Section 4.3).  For every cell whose criticality differs between f and g
 * (dimensions restricted to {0, n} at tier 1), pick the vertex to decrease:
 *  - false positive (paired in f, critical in g): the apex of the f-pair, i.e. the vertex
 *    whose value must drop below the cell's (FPmin: j; FPmax: j in 2D, l in 3D; the saddle
 *    cases pick a vertex of the cell paired with it in f).
 *  - false negative (critical in f, paired in g as (sigma, sigma+{x})): a vertex w of sigma
 *    that precedes x in f, so lowering it restores an order f has and g violates (FNmin: i;
 *    FN saddles/maxima: "i or j", "i, j or k"); Reading: with several candidates the one
 *    lowest in g is taken.  If no vertex of sigma precedes x in f, then x is below all of
 *    sigma in f too, sigma is paired in f, and the apex of sigma's f-pair is lowered so that
 *    sigma returns to its f-partner.
 * Marks targets in st->req; adds counts to cnt[2d] (FP) and cnt[2d+1] (FN); returns total. */
static int64_t c_detect(state_t *st, const grad_t *F, const grad_t *G, int tier, int64_t *cnt, vec *where) {
    const ocx *cx = st->cx;
    int n = cx->top;
    int64_t total = 0;
    for (int d = 0; d <= n; d++) {
        if (tier == 1 && d != 0 && d != n) continue;
        for (int64_t c = 0; c < cx->ncell[d]; c++) {
            if (!cx->exists[d][c]) continue;
            int fc = is_crit(cx, F, d, c), gc = is_crit(cx, G, d, c);
            if (fc == gc) continue;
            int lo_d; int64_t lo_id;
            int32_t target;
            if (!fc) {
                target = pair_apex(cx, F, d, c, &lo_d, &lo_id);
                cnt[2 * d]++;
            } else {
                int32_t x = pair_apex(cx, G, d, c, &lo_d, &lo_id);
                const int32_t *sv = cx->verts[lo_d] + lo_id * (lo_d + 1);
                target = -1;
                for (int j = 0; j <= lo_d; j++) {
                    if (!prec(cx, st->f, sv[j], x)) continue;
                    if (target < 0 || prec(cx, st->g, sv[j], target)) target = sv[j];
                }
                if (target < 0) {
                    int d2; int64_t i2;
                    target = pair_apex(cx, F, lo_d, lo_id, &d2, &i2);
                    assert(target >= 0);
                }
                cnt[2 * d + 1]++;
            }
            st->req[target] = 1;
            if (where) { vpush(where, d); vpush(where, c); }
            total++;
        }
    }
    return total;
}

/* S-loop detection (Section 4.4).  For each separatrix branch of f, follow its cells and find
 * the first one whose pairing in g differs from f (the troublemaker); lower the apex of its
 * f-pair (0-dim troublemaker i paired with ij in f: lower j; a top cell paired with facet tau
 * in f: lower the vertex it adds to tau).  Tier 4 fixes every branch with a troublemaker;
 * tier 3 (Reading) only those whose g-path ends at a different extremum than the f-path.
 * Reading: the first divergence along f's branch is where tracing the same separatrix in g
 * leaves it, so g's separatrices need not be extracted separately. */
static int64_t s_detect(state_t *st, const grad_t *F, const grad_t *G, const omsc *mf, int tier,
                        int64_t *tm_desc, int64_t *tm_asc, vec *where) {
    const ocx *cx = st->cx;
    int n = cx->top;
    int64_t total = 0;
    for (int64_t b = 0; b + 1 < mf->doff.n; b++) {
        for (int64_t k = mf->doff.p[b]; k < mf->doff.p[b + 1]; k++) {
            int64_t v = mf->dcell.p[k];
            if (G->up[0][v] == F->up[0][v]) continue;
            int ok = 1;
            if (tier == 3) ok = walk_desc(cx, G, mf->dcell.p[mf->doff.p[b]], NULL) != mf->dterm.p[b];
            if (ok) {
                int lo_d; int64_t lo_id;
                st->req[pair_apex(cx, F, 0, v, &lo_d, &lo_id)] = 1;
                if (where) { vpush(where, 0); vpush(where, v); }
                (*tm_desc)++;
                total++;
            }
            break;
        }
    }
    for (int64_t b = 0; b + 1 < mf->aoff.n; b++) {
        for (int64_t k = mf->aoff.p[b]; k < mf->aoff.p[b + 1]; k++) {
            int64_t T = mf->acell.p[k];
            if (G->down[n][T] == F->down[n][T]) continue;
            int ok = 1;
            if (tier == 3) ok = walk_asc(cx, G, mf->acell.p[mf->aoff.p[b]], NULL) != mf->aterm.p[b];
            if (ok) {
                int lo_d; int64_t lo_id;
                st->req[pair_apex(cx, F, n, T, &lo_d, &lo_id)] = 1;
                if (where) { vpush(where, n); vpush(where, T); }
                (*tm_asc)++;
                total++;
            }
            break;
        }
    }
    return total;
}

/* Saddle-saddle connectors (Section 3.1; Section 4.4, 1-dimensional troublemakers), in 3D.
 * The V-paths of the 1-2 level of f descend from every critical triangle (2-saddle): from a
 * triangle to each of its edges other than the one it is paired with, and from an edge paired
 * with a triangle in f on to that triangle; a path ends at a critical edge (a 1-saddle, which
 * makes it a saddle-saddle connector) or at an edge paired with a vertex.  These paths form a
 * DAG from each 2-saddle.  Reading: tracing g's paths from the same 2-saddle follows f's as long
 * as the edges met are paired alike; an edge whose pairing differs in g is where g's paths leave
 * f's, the 1-dimensional troublemaker.  Its target is the apex of its f-pair (edge ij paired
 * with triangle ijk in f but with ijl in g: lower k).  Edges beyond a troublemaker are not
 * examined.  The troublemakers are the edges with a differing pairing that are reachable from a
 * 2-saddle through edges paired alike, whatever order the DAG is walked in. */
static void push_triangle_edges(const ocx *cx, int64_t t, int64_t skip, vec *stack) {
    const int32_t *v = cx->verts[2] + t * 3;
    const int32_t pairs[3][2] = {{v[0], v[1]}, {v[0], v[2]}, {v[1], v[2]}};
    for (int k = 0; k < 3; k++) {
        int64_t e = lookup(cx, 1, pairs[k]);
        if (e >= 0 && e != skip) vpush(stack, e);
    }
}

static int64_t ss_detect(state_t *st, const grad_t *F, const grad_t *G, int64_t *tm_ss, vec *where) {
    const ocx *cx = st->cx;
    if (cx->top != 3) return 0;
    uint8_t *seen = xcalloc((size_t)cx->ncell[1], 1);
    vec stack = {0};
    for (int64_t t = 0; t < cx->ncell[2]; t++)
        if (is_crit(cx, F, 2, t)) push_triangle_edges(cx, t, -1, &stack);
    int64_t total = 0;
    while (stack.n > 0) {
        int64_t e = stack.p[--stack.n];
        if (seen[e]) continue;
        seen[e] = 1;
        if (G->up[1][e] != F->up[1][e] || G->down[1][e] != F->down[1][e]) {
            int lo_d; int64_t lo_id;
            int32_t target = pair_apex(cx, F, 1, e, &lo_d, &lo_id);
            if (target >= 0) {
                st->req[target] = 1;
                if (where) { vpush(where, 1); vpush(where, e); }
                (*tm_ss)++;
                total++;
            }
            continue;
        }
        if (F->up[1][e] >= 0) push_triangle_edges(cx, F->up[1][e], e, &stack);
    }
    free(stack.p);
    free(seen);
    return total;
}

/* Equation 2, once for every requested vertex (Jacobi: all requests of an iteration are
 * collected on g^(k) first, then each requested vertex takes exactly one step).
 * Reading: g = g_hat - q*Delta is formed from g_hat in one rounding (not by repeated
 * subtraction), so the decoder reproduces it exactly; the step is taken while q < q_max and
 * the result stays at or above the floor, otherwise g drops to the floor and is final. */
static int64_t apply_requests(state_t *st, int64_t *n_req) {
    int64_t changed = 0, nr = 0;
    for (int64_t v = 0; v < st->cx->nv; v++) {
        if (!st->req[v]) continue;
        st->req[v] = 0;
        nr++;
        if (st->floored[v]) continue;
        int q = st->q[v];
        float t = fmaf(-(float)(q + 1), st->delta, st->ghat[v]);
        if (q < st->q_max && t >= st->lo[v]) {
            st->q[v] = (uint8_t)(q + 1);
            st->g[v] = t;
        } else {
            st->g[v] = st->lo[v];
            st->floored[v] = 1;
        }
        changed++;
    }
    *n_req = nr;
    return changed;
}

static uint32_t fbits(float x) { uint32_t u; memcpy(&u, &x, 4); return u; }

int oracle_correct(const ocx *cx, const float *f, const float *g_hat, float xi, int tier, int ss,
                   int q_max, int64_t max_iters, float *g_out, uint8_t *q_out, int64_t *stats,
                   int64_t *log, int64_t log_cap) {
    memset(stats, 0, sizeof(int64_t) * 10);
    int64_t nv = cx->nv;
    if (tier < 1 || tier > 4 || q_max < 0 || q_max > 7 || max_iters < 0) { stats[9] = -1; return -1; }
    if (!(xi > 0.0f) || !isfinite(xi)) { stats[9] = -1; return -1; }
    float delta = ldexpf(xi, -q_max);
    if (!(delta >= FLT_MIN)) { stats[9] = -1; return -1; }
    for (int64_t i = 0; i < nv; i++)
        if (!isfinite(f[i]) || !isfinite(g_hat[i])) { stats[9] = -3; return -3; }
    state_t st = {0};
    st.cx = cx; st.f = f; st.ghat = g_hat; st.delta = delta; st.q_max = q_max;
    st.g = xcalloc((size_t)nv, sizeof(float));
    st.lo = xcalloc((size_t)nv, sizeof(float));
    float *hi = xcalloc((size_t)nv, sizeof(float));
    oracle_bounds(f, nv, xi, st.lo, hi);
    for (int64_t i = 0; i < nv; i++) {
        if (!(st.lo[i] <= g_hat[i] && g_hat[i] <= hi[i])) {
            free(st.g); free(st.lo); free(hi);
            stats[9] = -2;
            return -2;
        }
    }
    free(hi);
    st.q = xcalloc((size_t)nv, 1);
    st.floored = xcalloc((size_t)nv, 1);
    st.req = xcalloc((size_t)nv, 1);
    memcpy(st.g, g_hat, sizeof(float) * (size_t)nv);

    grad_t F, G;
    grad_alloc(cx, &F);
    grad_alloc(cx, &G);
    oracle_gradient(cx, f, F.up, F.down);
    omsc *mf = tier >= 3 ? msc_from_grad(cx, &F) : NULL;

    int64_t it = 0, c_it = 0, s_it = 0, residual = 0;
    int converged = 0, stalled = 0;
    for (;;) {
        oracle_gradient(cx, st.g, G.up, G.down);
        int64_t rec[16] = {0};
        int64_t viol = c_detect(&st, &F, &G, tier, rec + 1, NULL);
        int kind = 1;
        if (viol == 0 && tier >= 3) {
            viol = s_detect(&st, &F, &G, mf, tier, rec + 9, rec + 10, NULL);
            if (tier == 4 && ss) viol += ss_detect(&st, &F, &G, rec + 13, NULL);
            kind = 2;
        }
        if (viol == 0) { converged = 1; break; }
        if (it == max_iters) {
            residual = viol;
            memset(st.req, 0, (size_t)nv);
            break;
        }
        int64_t nreq;
        int64_t changed = apply_requests(&st, &nreq);
        if (changed == 0) { stalled = 1; residual = viol; break; }
        rec[0] = kind; rec[11] = nreq; rec[12] = changed;
        if (log && it < log_cap) memcpy(log + it * 16, rec, sizeof(rec));
        it++;
        if (kind == 1) c_it++; else s_it++;
    }

    int64_t n_edit = 0, n_quant = 0, n_lossless = 0;
    for (int64_t v = 0; v < nv; v++) {
        g_out[v] = st.g[v];
        uint8_t qo = st.q[v];
        if (st.floored[v]) qo = fbits(st.g[v]) != fbits(g_hat[v]) ? 0xFF : 0;
        q_out[v] = qo;
        if (qo) n_edit++;
        if (qo == 0xFF) n_lossless++;
        else if (qo) n_quant++;
    }
    stats[0] = it; stats[1] = c_it; stats[2] = s_it; stats[3] = n_edit; stats[4] = n_quant;
    stats[5] = n_lossless; stats[6] = residual; stats[7] = converged; stats[8] = stalled;
    stats[9] = converged ? 0 : 1;
    omsc_free(mf);
    grad_free(&F);
    grad_free(&G);
    free(st.g); free(st.lo); free(st.q); free(st.floored); free(st.req);
    return (int)stats[9];
}

/* The violations of g against f that the correction loop would see at this state: the cells
 * whose criticality differs (Section 4.3), or, when there are none and tier >= 3, the first
 * differing cell of every separatrix branch that the tier checks (Section 4.4), one entry per
 * branch.  Writes up to cap (dimension, cell id) pairs; returns the total count. */
int64_t oracle_residual(const ocx *cx, const float *f, const float *g, int tier, int ss, int64_t *dims,
                        int64_t *ids, int64_t cap) {
    int64_t nv = cx->nv;
    state_t st = {0};
    st.cx = cx; st.f = f; st.ghat = g; st.g = (float *)g;
    st.req = xcalloc((size_t)nv, 1);
    grad_t F, G;
    grad_alloc(cx, &F);
    grad_alloc(cx, &G);
    oracle_gradient(cx, f, F.up, F.down);
    oracle_gradient(cx, g, G.up, G.down);
    vec where = {0};
    int64_t cnt[16] = {0};
    int64_t viol = c_detect(&st, &F, &G, tier, cnt + 1, &where);
    if (viol == 0 && tier >= 3) {
        omsc *mf = msc_from_grad(cx, &F);
        viol = s_detect(&st, &F, &G, mf, tier, cnt + 9, cnt + 10, &where);
        if (tier == 4 && ss) viol += ss_detect(&st, &F, &G, cnt + 13, &where);
        omsc_free(mf);
    }
    for (int64_t k = 0; k < viol && k < cap; k++) { dims[k] = where.p[2 * k]; ids[k] = where.p[2 * k + 1]; }
    free(where.p);
    free(st.req);
    grad_free(&F);
    grad_free(&G);
    return viol;
}
