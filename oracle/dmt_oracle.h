/* Plain CPU oracle for the MSC-preserving correction stage (DMTz, arXiv 2409.17346).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests, the smoke check
 * and the CPU baseline leg of the benchmark can compare the GPU path against a
 * slow, obviously correct implementation written from the paper.  The product
 * path never links, loads or calls it, and it shares no code with the GPU path.
 *
 * Everything works on an explicit simplicial complex: per dimension d, a cell
 * id space [0, ncell[d]), an "exists" flag, the cell's vertices (ascending
 * vertex index) and its cofacets.  A regular grid becomes such a complex
 * through the Freudenthal (Kuhn) triangulation; its cell ids follow the
 * anchor/type scheme (id = anchor * T_d + type) documented with the library
 * interface, so results can be compared with the GPU id for id.
 *
 * Vertex order (simulation of simplicity, Section 4.1 "Degeneracy handling"):
 * a precedes b  iff  h[a] < h[b], or h[a] == h[b] and key[a] < key[b], where key
 * is the vertex's global linear id.
 */
#ifndef DMT_ORACLE_H
#define DMT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ocx ocx;      /* explicit complex */
typedef struct omsc omsc;    /* extracted Morse-Smale complex */

/* Grid complex of nx*ny*nz vertices (nz == 1 -> 2D).  key may be NULL (key = local id)
 * or point at nx*ny*nz global ids (used for windows cut out of a larger grid). */
ocx *ocx_grid(int64_t nx, int64_t ny, int64_t nz, const int64_t *key);
/* Explicit complex of dimension top (1..3): n[d] cells of dimension d given by their
 * vertex lists (d+1 vertex indices each, any order).  Vertices are 0..nv-1, key = index. */
ocx *ocx_explicit(int top, int64_t nv, const int64_t n[4], const int32_t *edges,
                  const int32_t *tris, const int32_t *tets);
void ocx_free(ocx *cx);
int ocx_top(const ocx *cx);
int64_t ocx_ncell(const ocx *cx, int d);
int ocx_exists(const ocx *cx, int d, int64_t id);
/* Writes the d+1 vertex indices of cell (d, id); returns 0, or -1 if it does not exist. */
int ocx_cell_vertices(const ocx *cx, int d, int64_t id, int32_t *out);

/* Discrete gradient of field h (Section 3.1 pairing rules): up[d][id] = paired cofacet id
 * or -1, down[d][id] = paired facet id or -1.  Arrays are ncell[d] long (up[top] and
 * down[0] are all -1).  Cells that do not exist get -1 in both. */
void oracle_gradient(const ocx *cx, const float *h, int64_t *up[4], int64_t *down[4]);

/* Morse-Smale complex of h: critical cells, separatrix branches, manifold labels. */
omsc *oracle_msc(const ocx *cx, const float *h);
enum {
    OMSC_CRIT0 = 0, OMSC_CRIT1 = 1, OMSC_CRIT2 = 2, OMSC_CRIT3 = 3,
    OMSC_DESC_SADDLE = 10, OMSC_DESC_OFFSETS = 11, OMSC_DESC_CELLS = 12, OMSC_DESC_TERMINAL = 13,
    OMSC_ASC_SADDLE = 20, OMSC_ASC_OFFSETS = 21, OMSC_ASC_CELLS = 22, OMSC_ASC_TERMINAL = 23,
    OMSC_MIN_LABEL = 30, OMSC_MAX_LABEL = 31
};
int64_t omsc_count(const omsc *m, int what);
void omsc_copy(const omsc *m, int what, int64_t *dst);
void omsc_free(omsc *m);

/* Smallest fp32 >= f[i] - xi and largest fp32 <= f[i] + xi, in exact arithmetic. */
void oracle_bounds(const float *f, int64_t n, float xi, float *lo, float *hi);

/* Full correction.  ss != 0 adds the saddle-saddle connectors of a 3D complex to the separatrix
 * step at tier 4.  stats[0..9] = iterations, c_iterations, s_iterations, n_edited,
 * n_quantized, n_lossless, residual_violations, converged, stalled, status.
 * log (may be NULL) receives up to log_cap records of 16 int64:
 *   kind (1 = C, 2 = S), FP0, FN0, FP1, FN1, FP2, FN2, FP3, FN3, TM_desc, TM_asc,
 *   |R|, changed, TM_ss (saddle-saddle troublemakers), 0, 0.
 * status: 0 ok, 1 not converged (stalled or max_iters), -1 invalid, -2 bound, -3 nonfinite. */
int oracle_correct(const ocx *cx, const float *f, const float *g_hat, float xi, int tier, int ss,
                   int q_max, int64_t max_iters, float *g_out, uint8_t *q_out, int64_t *stats,
                   int64_t *log, int64_t log_cap);

/* Violations of g against f as the correction loop sees them: cells whose criticality differs,
 * else (tier >= 3) the first differing cell of each separatrix branch the tier checks (and, with
 * ss at tier 4, the saddle-saddle troublemaker edges).  Writes up to cap (dimension, id) pairs
 * and returns the total. */
int64_t oracle_residual(const ocx *cx, const float *f, const float *g, int tier, int ss, int64_t *dims,
                        int64_t *ids, int64_t cap);

/* Decoder: g = lossless ? stored value : (g_hat - q*Delta) rounded once, Delta = xi*2^-q_max. */
void oracle_decode(const float *g_hat, const uint8_t *q, int64_t n, const int64_t *idx,
                   const float *val, int64_t n_lossless, float xi, int q_max, float *g_out);

#ifdef __cplusplus
}
#endif
#endif
