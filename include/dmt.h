/* dmt.h - C ABI of the MI355X (gfx950) library for the Morse-Smale-complex-preserving
 * correction stage of error-bounded lossy compression (DMTz, arXiv 2409.17346).
 *
 * Problem (Section 4.1, "Problem Statement"): given an original scalar field f and a
 * decompressed field g_hat on the same grid with |g_hat_i - f_i| <= xi, produce edits
 * delta_i and the corrected field g = g_hat + delta with |f_i - g_i| <= xi for every vertex
 * and a discrete Morse-Smale complex identical to that of f.
 *
 * Grid and complex.  Scalars live on the vertices of an nx*ny*nz regular grid (nz == 1 for
 * 2D), x fastest: vertex id v = x + nx*(y + ny*z).  The grid is triangulated by the
 * Freudenthal/Kuhn rule (two triangles per square along the (1,1) diagonal, six tetrahedra
 * per cube along the (1,1,1) diagonal; the paper's "regular grid-based triangulation" with
 * "six tetrahedra per cube", Section 4.8.1).
 *
 * Cell ids.  A cell is {a, a+c1, ..., a+cd} with a its componentwise-minimum vertex (the
 * anchor) and 0 < c1 < ... < cd a chain of direction bit sets (bit 0 = +x, bit 1 = +y,
 * bit 2 = +z, strict bitwise inclusion).  The chains of each dimension are sorted
 * lexicographically by their bit values and numbered 0..T_d-1:
 *   2D: T = {1, 3, 2}       (vertices, edges, triangles)
 *   3D: T = {1, 7, 12, 6}   (vertices, edges, triangles, tetrahedra)
 * Cell id = a * T_d + type, one id space per dimension; ids whose cell leaves the grid are
 * holes ("does not exist").  Ids are int64.
 *
 * Vertex order (Section 4.1, "Degeneracy handling"): a precedes b iff h_a < h_b, or
 * h_a == h_b and a < b (simulation of simplicity; -0 == +0).  Non-finite values are rejected.
 *
 * Memory.  Every array argument is a DEVICE pointer owned by the caller unless its name ends
 * in _host.  Nothing is freed by the library except its own context.  Calls are ordered on
 * the given stream; a call returns after the results it reports on the host are known
 * (it synchronises that stream when it returns host values).
 *
 * Errors.  Functions return dmt_status; no exception crosses the ABI.  dmt_last_error gives
 * a message for the last failing call on a context.  Validation errors leave outputs
 * untouched.  Contexts are not thread safe: use one per host thread.
 */
#ifndef DMT_H
#define DMT_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DMT_OK = 0,
    DMT_W_NOT_CONVERGED = 1,   /* stalled or iteration cap hit; outputs valid and within bound */
    DMT_W_PENDING = 2,         /* dmt_server_poll: the job has not finished yet */
    DMT_E_INVALID = -1,        /* bad grid, options, xi or sizes */
    DMT_E_BOUND = -2,          /* some |g_hat_i - f_i| > xi */
    DMT_E_NONFINITE = -3,      /* NaN or Inf in an input field */
    DMT_E_NOMEM = -4,          /* device allocation failed */
    DMT_E_HIP = -5             /* other HIP runtime error */
} dmt_status;

/* Preservation tiers (Section 4.1, "Multitier preservation targets"). */
typedef enum {
    DMT_T1_EXTREMA = 1,        /* minima and maxima */
    DMT_T2_CRITICAL = 2,       /* all critical cells */
    DMT_T3_CONNECTIVITY = 3,   /* + each separatrix reaches the same extremum */
    DMT_T4_GEOMETRY = 4        /* + each separatrix follows the same cells */
} dmt_tier;

typedef struct dmt_context dmt_context;

typedef struct {
    int32_t ndim;              /* 2 or 3; ndim == 2 requires nz == 1 */
    int64_t nx, ny, nz;        /* every used extent >= 2; nx*ny*nz < 2^31 */
} dmt_grid;

typedef struct {
    int32_t tier;              /* dmt_tier */
    int32_t q_max;             /* 0..7: edit step xi / 2^q_max (Equation 2); the paper uses 6 */
    int64_t max_iters;         /* cap on edit iterations (C + S); < 0 means no cap */
    uint32_t flags;            /* 0, or DMT_F_DENSE / DMT_F_PHASES, and DMT_F_SADDLE_SADDLE */
} dmt_options;

/* Option flags.  The first two choose how the loop runs (results are bit-identical in every
 * form; they exist for testing):
 * DMT_F_DENSE   recompute the whole gradient and every violation each iteration instead of only
 *               around the vertices edited in the previous iteration;
 * DMT_F_PHASES  run every iteration as full-grid kernel launches, one per phase, instead of
 *               inside one workgroup that stays resident for the whole loop.
 * DMT_F_SADDLE_SADDLE  (3D, tier 4) also preserve the saddle-saddle connectors (Section 3.1;
 *               Section 4.4, 1-dimensional troublemakers): the separatrix step walks f's 1-2 V-paths
 *               down from every 2-saddle through edges paired alike in f and g, and an edge paired
 *               differently in g is a troublemaker (edge ij paired with ijk in f: lower k).  Every
 *               edge these walks reach then pairs as in f, so g's connectors equal f's.  No effect
 *               in 2D or below tier 4. */
#define DMT_F_DENSE 1u
#define DMT_F_PHASES 2u
#define DMT_F_SADDLE_SADDLE 4u

typedef struct {
    int64_t iterations;        /* edit iterations applied (C + S) */
    int64_t c_iterations;      /* iterations fixing false critical cells (Section 4.3) */
    int64_t s_iterations;      /* iterations fixing separatrix troublemakers (Section 4.4) */
    int64_t n_edited;          /* vertices with q_out != 0 */
    int64_t n_quantized;       /* vertices with 1 <= q_out <= q_max */
    int64_t n_lossless;        /* vertices with q_out == 0xFF */
    int64_t residual_violations; /* violations left when not converged, else 0 */
    int32_t converged;
    int32_t stalled;           /* requests existed but every requested vertex was final */
} dmt_stats;

/* Per-iteration log record (int64 each): kind (1 = C, 2 = S), FP0, FN0, FP1, FN1, FP2, FN2,
 * FP3, FN3 (false positive / negative critical cells by dimension), TM_desc, TM_asc
 * (troublemaker branches fixed), n_req (vertices requested), changed (vertices edited), then
 * the work of the frontier forms in that iteration (0 in the dense form): dirty vertices,
 * affected anchors, listed violating anchors, branches whose first differing cell was
 * settled, branch cells examined while settling them, branch cells touched (on dirty vertices
 * whose own or top-cell pairing changed), the duration
 * of the iteration in the resident loop in 10 ns ticks (0 elsewhere; timing, not a result), and
 * TM_ss (saddle-saddle troublemaker edges, DMT_F_SADDLE_SADDLE). */
#define DMT_LOG_WORDS 21

/* ---- context ----------------------------------------------------------------------------- */

/* Creates a context bound to HIP device hip_device.  The context owns device scratch (grown on
 * demand, freed by dmt_context_destroy) and the results of the last MSC extraction /
 * correction. */
dmt_status dmt_context_create(dmt_context **ctx, int hip_device);
dmt_status dmt_context_destroy(dmt_context *ctx);
const char *dmt_last_error(const dmt_context *ctx);

/* Sizes of the per-dimension cell id spaces (N * T_d; 0 above ndim).  Host only. */
dmt_status dmt_cell_id_space(const dmt_grid *grid, int64_t counts_host[4]);

/* ---- setup (Section 4.2, Equation 2; Section 5 "relative error bound") ------------------ */

/* xi = fl32(rel * (max f - min f)), the range taken in double precision. */
dmt_status dmt_xi_from_relative(dmt_context *ctx, const dmt_grid *grid, const float *f, double rel,
                                float *xi_host, hipStream_t stream);

/* lo[i] = smallest fp32 >= f[i] - xi, hi[i] = largest fp32 <= f[i] + xi (exact arithmetic).
 * lo is the floor Equation 2 drops a vertex to ("f_i - xi").  n elements. */
dmt_status dmt_bounds(dmt_context *ctx, const float *f, int64_t n, float xi, float *lo, float *hi,
                      hipStream_t stream);

/* ---- discrete gradient and Morse-Smale complex (Section 3.1) ------------------------------ */

/* Discrete gradient of field (Section 3.1 pairing of Shivashankar-Natarajan as spelled out in
 * Section 4.2): for every cell id of every dimension d, up[off_d + id] = paired cofacet id (dim
 * d+1) or -1, down[off_d + id] = paired facet id (dim d-1) or -1, where off_d is the sum of the
 * id-space sizes of lower dimensions.  up and down hold sum_d counts[d] int64 each. */
dmt_status dmt_gradient_pairs(dmt_context *ctx, const dmt_grid *grid, const float *field,
                              int64_t *up, int64_t *down, hipStream_t stream);

/* Items of an extracted MSC (all int64):
 *  CRITd          ids of critical d-cells, ascending.
 *  DESC_*         descending separatrices: for each critical edge (1-saddle) in id order, one
 *                 branch per endpoint (endpoint id order): SADDLE[b], the vertex sequence
 *                 CELLS[OFFSETS[b] .. OFFSETS[b+1]) from the endpoint to the minimum, and
 *                 TERMINAL[b] (the minimum's vertex id).  OFFSETS has n_desc + 1 entries.
 *  ASC_*          ascending separatrices: for each critical (n-1)-cell in id order, one branch
 *                 per top-dimensional cofacet (id order): the top-cell sequence and TERMINAL =
 *                 the maximum's id, or -1 if the path leaves through the domain boundary.
 *  MIN_LABEL[v]   terminal of v's descending path (N entries).
 *  MAX_LABEL[T]   terminal of top cell T's ascending path, -1 boundary, -2 for ids that do not
 *                 exist (counts[ndim] entries). */
enum {
    DMT_MSC_CRIT0 = 0, DMT_MSC_CRIT1 = 1, DMT_MSC_CRIT2 = 2, DMT_MSC_CRIT3 = 3,
    DMT_MSC_DESC_SADDLE = 10, DMT_MSC_DESC_OFFSETS = 11, DMT_MSC_DESC_CELLS = 12, DMT_MSC_DESC_TERMINAL = 13,
    DMT_MSC_ASC_SADDLE = 20, DMT_MSC_ASC_OFFSETS = 21, DMT_MSC_ASC_CELLS = 22, DMT_MSC_ASC_TERMINAL = 23,
    DMT_MSC_MIN_LABEL = 30, DMT_MSC_MAX_LABEL = 31
};

/* Extracts the MSC of field into the context (kept until the next extraction) and writes the
 * length of every item to counts_host[item] (an array of 32 int64). */
dmt_status dmt_extract_msc(dmt_context *ctx, const dmt_grid *grid, const float *field,
                           int64_t counts_host[32], hipStream_t stream);
/* Copies item of the last extraction into dst (device, cap int64 entries). */
dmt_status dmt_msc_copy(dmt_context *ctx, int item, int64_t *dst, int64_t cap, hipStream_t stream);

/* Agreement of the MSC of g with that of f (Section 5.1, "Evaluation Metrics": critical and
 * separatrix recall = common / f's, precision = common / g's).  All counts are of the complexes
 * as dmt_extract_msc defines them:
 *   crit_f[d], crit_g[d]  critical d-cells of f and of g (0 above the grid's dimension);
 *   crit_common[d]        d-cells critical in both;
 *   sep_f[k], sep_g[k]    separatrix branches, k = 0 descending (1-saddle -> minimum), k = 1
 *                         ascending ((n-1)-saddle -> maximum or boundary);
 *   sep_same_ends[k]      branches of f whose counterpart in g (same saddle, same first cell)
 *                         ends at the same extremum (connectivity, tier 3);
 *   sep_same_cells[k]     those whose whole cell sequence is equal (geometry, tier 4).
 * f, g: N floats on the device.  Results on the host; the call synchronises the stream. */
typedef struct {
    int64_t crit_f[4], crit_g[4], crit_common[4];
    int64_t sep_f[2], sep_g[2], sep_same_ends[2], sep_same_cells[2];
} dmt_msc_agreement;
dmt_status dmt_compare_msc(dmt_context *ctx, const dmt_grid *grid, const float *f, const float *g,
                           dmt_msc_agreement *agreement_host, hipStream_t stream);

/* ---- correction (Sections 4.2-4.7) ------------------------------------------------------- */

/* Runs the C-loop / S-loop correction until f's MSC (at the requested tier) is restored.
 * f, g_hat: N floats.  Outputs: g_out (N floats, the corrected field) and q_out (N bytes:
 * the quantized edit count 0..q_max, or 0xFF where the vertex was set to its floor and is
 * stored losslessly).  Returns DMT_OK when converged, DMT_W_NOT_CONVERGED otherwise (outputs
 * still valid and within bound).  The lossless edits and the per-iteration log of this call
 * stay in the context for dmt_lossless_edits / dmt_iteration_log. */
dmt_status dmt_correct(dmt_context *ctx, const dmt_grid *grid, const float *f, const float *g_hat,
                       float xi, const dmt_options *opts, float *g_out, uint8_t *q_out,
                       dmt_stats *stats_host, hipStream_t stream);

/* Allocation-free variant of dmt_correct, for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid hipMalloc).  Same inputs,
 * outputs, statuses and results as dmt_correct, bit for bit; it makes no device allocation or
 * free of any kind.  Every device buffer it needs besides the caller's comes from one scratch
 * array of DMT_NOALLOC_SCRATCH_BYTES per GPU, part of the library's code object (so each GPU
 * the library runs on holds it until the process ends); its address is resolved when a
 * context is created on that device.
 * The lossless edits are written here instead of staying in the context: lossless_idx /
 * lossless_val are device arrays of lossless_cap entries (int64 vertex ids ascending, fp32
 * values); lossless_count_host receives the number of entries, and a count above lossless_cap
 * returns DMT_E_INVALID (g_out and q_out are still written).  The per-iteration log stays in the
 * context as for dmt_correct; dmt_lossless_edits reports no entries after this call, and kernel
 * timing (dmt_profile_enable) is not recorded for it.
 * Limits: DMT_E_NOMEM, before any work, when dmt_workspace_bytes of the grid exceeds
 * DMT_NOALLOC_SCRATCH_BYTES (about 0.92 M vertices in 2D, 0.50 M in 3D), or during the call if a
 * field's separatrices need more scratch than is left (outputs then undefined).
 * Concurrency: all calls on one GPU share its scratch array, which keeps the last call's
 * contents (each call initialises what it reads).  Calls that overlap in time on one GPU, from
 * any context or stream, race and corrupt each other's results: serialise them, e.g. on one
 * stream. */
#define DMT_NOALLOC_SCRATCH_BYTES 134217728LL
dmt_status dmt_correct_noalloc(dmt_context *ctx, const dmt_grid *grid, const float *f, const float *g_hat,
                               float xi, const dmt_options *opts, float *g_out, uint8_t *q_out,
                               int64_t *lossless_idx, float *lossless_val, int64_t lossless_cap,
                               int64_t *lossless_count_host, dmt_stats *stats_host, hipStream_t stream);

/* Launch shapes of the correction loop (Section 4.8: the GPU form of the C/S loops).  They change
 * speed only: every setting gives bit-identical results.  Index 0 is for 2D jobs, 1 for 3D jobs,
 * except grid_iterations: 0 for calls that run one job (dmt_correct), 1 for calls that run
 * several (batches, server rounds).
 *   loop_threads     threads of the workgroup that runs one job's loop: 512 or 1024 for 2D,
 *                    256 or 512 for 3D (fewer threads leave more registers per lane);
 *   handoff_anchors  in calls that run one job, an iteration with more affected plus listed
 *                    anchors than this (or a troublemaker pass over more candidate branches)
 *                    leaves the workgroup and runs as full-grid launches, one per phase; 0 never
 *                    hands off;
 *   grid_iterations  iterations run as full-grid launches per hand-off (1..4096);
 *   batch_handoff_anchors  the hand-off limit of calls that run several jobs (a paused job waits
 *                    for the other workgroups, so batches favour fewer, larger hand-offs).
 * Defaults: {1024, 512}, {8192, 1024}, {4, 64}, {8192, 8192}.  The autotuner of the Python
 * package picks them per workload by timing candidates. */
typedef struct {
    int32_t loop_threads[2];
    int32_t handoff_anchors[2];
    int32_t grid_iterations[2];
    int32_t batch_handoff_anchors[2];
} dmt_tuning;

/* Sets the launch shapes of later calls on ctx (NULL restores the defaults).  DMT_E_INVALID for
 * values outside the ranges above (the context keeps its setting). */
dmt_status dmt_set_tuning(dmt_context *ctx, const dmt_tuning *tuning);
/* Reads the launch shapes of ctx into tuning_host. */
dmt_status dmt_get_tuning(const dmt_context *ctx, dmt_tuning *tuning_host);

/* One job of a batch (Section 5.7: every field of a time series is corrected on its own).
 * Inputs: grid, device pointers f and g_hat, xi, options (flags must be 0), output device
 * pointers g_out and q_out, as for dmt_correct.  Filled by the call: status and stats. */
typedef struct {
    dmt_grid grid;
    const float *f, *g_hat;
    float xi;
    dmt_options opts;
    float *g_out;
    uint8_t *q_out;
    dmt_status status;
    dmt_stats stats;
} dmt_job;

/* Corrects n_jobs independent fields of any sizes (2D and 3D mixed) together: after each
 * field's setup and dense first iteration, one launch runs the C/S loops, each field inside one
 * workgroup taken from a queue, so fields proceed concurrently on different compute units.
 * Every job's outputs equal those of dmt_correct on the same inputs.  A job
 * that fails validation gets its error status and is skipped; the others still run.  Returns
 * the first job error, else DMT_W_NOT_CONVERGED if any job did not converge, else DMT_OK.  The
 * lossless edits of a job are the vertices whose q_out is 0xFF, with values g_out; no
 * per-iteration log is kept. */
dmt_status dmt_correct_batch(dmt_context *ctx, int32_t n_jobs, dmt_job *jobs_host, hipStream_t stream);

/* ---- served form: a request stream of corrections --------------------------------------- */

/* Estimated device workspace (bytes) of correcting one field of this grid: the unit of the
 * server's admission.  An upper estimate (the separatrix branches are data-dependent); -1 for an
 * invalid grid. */
int64_t dmt_workspace_bytes(const dmt_grid *grid, const dmt_options *opts);

typedef struct dmt_server dmt_server;

/* Starts a server on HIP device hip_device: min(max_jobs, 4) worker lanes, each a thread with its
 * own context and stream, among which the max_jobs slots (1..4096) are dealt out.  Jobs are
 * admitted in submission order while the summed footprints of all jobs in flight (the larger of
 * a job's estimate and the workspace it holds, plus what idle slots still hold) stay within
 * hbm_budget_bytes; a job always starts on an idle server.  An idle lane takes the next queued job
 * at once, so a job that arrives while others run starts on another stream and overlaps them on
 * the device; a busy lane admits more only when every lane is busy.  Each lane advances its jobs
 * together in rounds of one loop launch (at most 512 iterations per job), so its later jobs join
 * at the next round and finished ones leave after theirs.  Each job's results equal those of
 * dmt_correct. */
dmt_status dmt_server_create(dmt_server **srv, int hip_device, int64_t hbm_budget_bytes, int32_t max_jobs);

/* Waits for every submitted job to finish, then stops the worker and frees the server. */
dmt_status dmt_server_destroy(dmt_server *srv);

/* Queues one job (the descriptor is copied; flags must be 0).  Its device buffers must hold the
 * inputs when this is called (the server works on its own stream) and stay valid, untouched by
 * the caller, until dmt_server_poll returns DMT_OK for the ticket.  Invalid descriptors are
 * rejected here with DMT_E_INVALID.  Thread-safe. */
dmt_status dmt_server_submit(dmt_server *srv, const dmt_job *job, int64_t *ticket);

/* Result of a ticket: DMT_OK once the job has finished (result gets the descriptor with status
 * and stats filled; the ticket is then released), DMT_W_PENDING while it runs (wait = 0) or
 * after waiting for it (wait != 0, never returns pending), DMT_E_INVALID for an unknown ticket.
 * The lossless edits are the vertices with q_out == 0xFF, with values g_out.  Thread-safe. */
dmt_status dmt_server_poll(dmt_server *srv, int64_t ticket, int32_t wait, dmt_job *result);

/* Accounting of a server (host values; any pointer may be NULL): inflight_bytes = the bytes
 * admission counts (each job in flight at the larger of its estimate and the workspace it holds,
 * each idle slot at the workspace it still holds, plus the shared buffers), held_bytes = device
 * bytes held by the server's workspaces when last accounted, free_slots / pending = idle slots and
 * queued jobs, distinct_free_slots = idle slots counted once each (equal to free_slots unless
 * the slot list is corrupt).  The workspace of a finished job is kept for reuse; admission
 * releases idle slots' workspaces when a job would not fit the budget otherwise.
 * Setting DMT_FAULT_OUTPUTS=k in the environment before dmt_server_create makes the output step
 * of the k-th finished job fail with DMT_E_NOMEM (a test of the server's error path).
 * Thread-safe. */
dmt_status dmt_server_info(dmt_server *srv, int64_t *inflight_bytes, int64_t *held_bytes, int32_t *free_slots,
                           int32_t *pending, int32_t *distinct_free_slots);

/* Lossless edits of a finished batch or served job, read from its outputs (Section 4.7: the
 * vertices whose edit is stored as a value): the vertex ids with q_out == 0xFF in ascending
 * order and their values g_out.  n = vertices.  count_host receives the number of entries; with
 * cap == 0 nothing else is written, otherwise cap must be >= that count (else DMT_E_INVALID).
 * idx_out and val_out are device arrays of cap entries. */
dmt_status dmt_lossless_list(dmt_context *ctx, const uint8_t *q_out, const float *g_out, int64_t n,
                             int64_t *idx_out, float *val_out, int64_t cap, int64_t *count_host,
                             hipStream_t stream);

/* Lossless edits of the last dmt_correct: vertex ids ascending and their final values.
 * Writes min(count, cap) entries, returns the full count in count_host. */
dmt_status dmt_lossless_edits(dmt_context *ctx, int64_t *idx_out, float *val_out, int64_t cap,
                              int64_t *count_host, hipStream_t stream);

/* Per-iteration log of the last dmt_correct (host memory, DMT_LOG_WORDS int64 per record). */
dmt_status dmt_iteration_log(dmt_context *ctx, int64_t *log_host, int64_t cap, int64_t *count_host);

/* Decoder (Section 4.7, Figure 5 decompression side): g = g_hat - q * xi/2^q_max rounded once,
 * then the n_lossless (idx, val) pairs overwrite their vertices.  q == 0xFF entries must be
 * listed in idx.  All arrays on the device. */
dmt_status dmt_apply_edits(dmt_context *ctx, const float *g_hat, const uint8_t *q, int64_t n,
                           const int64_t *idx, const float *val, int64_t n_lossless, float xi,
                           int32_t q_max, float *g_out, hipStream_t stream);

/* ---- edit stream (Section 4.7, "Quantized Representation of Edits") ----------------------- */

/* Bits per vertex of the edit stream for q_max (0..7): the least b with 2^b >= q_max + 2 (codes
 * 0..q_max are edit counts, q_max + 1 marks a lossless vertex); q_max 6 -> 3.  -1 for a bad q_max. */
int32_t dmt_edit_bits(int32_t q_max);

/* Encodes a correction's edits as the paper's fixed-bit stream: code k = q_out[k] (0xFF -> q_max + 1)
 * in bits [k*b, (k+1)*b) of stream, little-endian within uint32 words (stream: device, at least
 * ceil(n*b/32) words, unused high bits of the last word zero), and the values g_out[k] of the
 * lossless vertices in vertex order into lossless_val (device, lossless_cap floats; no index is
 * stored, the stream marks the positions).  n_lossless_host receives their number; with
 * lossless_cap == 0 only the stream and the count are written, otherwise lossless_cap must be >= the
 * count.  DMT_E_INVALID for q_out entries above q_max other than 0xFF.  Synchronises the stream.
 * The stream is what a dictionary coder compresses next (the paper uses ZSTD). */
dmt_status dmt_pack_edits(dmt_context *ctx, const uint8_t *q_out, const float *g_out, int64_t n, int32_t q_max,
                          uint32_t *stream, int64_t stream_words, float *lossless_val, int64_t lossless_cap,
                          int64_t *n_lossless_host, hipStream_t stream_hip);

/* Decoder of dmt_pack_edits (decompression side of Section 4.7): g_out[k] = g_hat[k] - q * xi/2^q_max
 * rounded once for codes q <= q_max, else the next lossless value; q_out (device, optional) gets
 * the edit counts as dmt_correct wrote them.  DMT_E_INVALID for codes above q_max + 1 or a lossless
 * count different from n_lossless.  Synchronises the stream. */
dmt_status dmt_unpack_edits(dmt_context *ctx, const uint32_t *stream, int64_t stream_words, int64_t n,
                            int32_t q_max, const float *g_hat, const float *lossless_val, int64_t n_lossless,
                            float xi, float *g_out, uint8_t *q_out, hipStream_t stream_hip);

/* ---- kernel timing (roofline measurement) ------------------------------------------------ */

/* Kernel families timed by dmt_profile_*: */
enum {
    DMT_PROF_GRADIENT = 0,  /* lower-star gradient pass, units = vertices */
    DMT_PROF_CLASSIFY = 1,  /* critical-cell classification over every anchor (iteration 0), units = anchors */
    DMT_PROF_APPLY = 2,     /* Equation 2 edits: the dense form's pass (units = vertices), or the requests
                               and edits of iteration 0's listed violations (units 0) */
    DMT_PROF_SSTEP = 3,     /* separatrix troublemaker pass, units = branch cells */
    DMT_PROF_SETUP = 4,     /* floors and validation, units = vertices */
    DMT_PROF_MSC = 5,       /* critical cells + separatrix branches of f, units = vertices */
    DMT_PROF_LOOP = 6,      /* the frontier correction loop (resident kernel or its phases) */
    /* phases inside the resident loop kernel during the last correction call, summed over jobs
     * (wall clock of each job's workgroup, including the workgroup barrier that ends each phase;
     * launches and units read 0): the troublemaker pass, the gradient pass and the violation pass */
    DMT_PROF_LOOP_SAPPLY = 7, DMT_PROF_LOOP_GRAD = 8, DMT_PROF_LOOP_VR = 9,
    DMT_PROF_KERNELS = 10
};

/* Turns event timing of the kernel families on (1) or off (0) for later calls on ctx and
 * clears what was recorded.  Events are recorded on the stream each kernel is launched on. */
dmt_status dmt_profile_enable(dmt_context *ctx, int enable);
/* Launch count, summed duration (ms) and summed work units of family kernel since the last
 * dmt_profile_enable.  Waits for the recorded events. */
dmt_status dmt_profile_read(dmt_context *ctx, int kernel, int64_t *launches_host, double *ms_total_host,
                            int64_t *units_host);

#ifdef __cplusplus
}
#endif
#endif /* DMT_H */
