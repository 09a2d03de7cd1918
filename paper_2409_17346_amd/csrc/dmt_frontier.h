// Frontier form of the C/S correction loop (Sections 4.3-4.6), run on the device.
//
// The iteration is Jacobi: on g^(k), collect every violation's target vertex, then give each
// requested vertex one Equation 2 step.  Between iterations only the edited vertices change,
// so only a neighbourhood of them needs new work:
//   * a cell's pairing depends on the values on the closed 1-ring of its highest vertex, so
//     the gradient is recomputed for the closed 1-ring of every edited vertex (dirty vertices);
//   * a cell's violation (and its target) depends on its own codes and vertex values, so the
//     violation masks are recomputed for the anchors of cells touching a dirty vertex;
//   * every current violation requests its target again each iteration, so the anchors with a
//     non-zero violation mask are kept in a list that is rebuilt every iteration.
// g is double buffered: iteration k reads g^(k) from gb[k&1] and writes g^(k+1) into gb[(k+1)&1],
// which already holds g^(k) except on the vertices edited in iteration k-1 (copied across when
// those vertices are revisited as dirty).  Detection never sees an edit of its own iteration,
// so the thread that first requests a vertex can edit it at once: requests are deduplicated
// with per-iteration stamps (atomicMax) and each requested vertex takes exactly one step.
// Critical-cell targets are edited as they are found.  Separatrix troublemakers count only when
// no critical-cell violation exists, so f's branches are scanned speculatively in the same pass
// and their targets are edited after one grid-wide synchronisation.  Lists are filled with
// wave-aggregated appends.  The output is bit-identical to the dense form and to the oracle.
#pragma once
#include <cstddef>

#include "dmt_kernels.h"

namespace dmt {

// A full-grid iteration is dense when its lists cover more than 1/DENSE_DIV of the grid; a dense
// violation pass after an iteration that edited more than 1/NOMARK_DIV of the vertices marks no
// neighbourhoods.
constexpr int DENSE_DIV = 4;
constexpr int NOMARK_DIV = 32;

// The dirty-vertex, affected-anchor (two parities) and request stamps of a vertex are one
// 16-byte record: vstamp, astamp[0], astamp[1] and rstamp point at its words 0..3.
constexpr int STAMP_STRIDE = 4;

// Per-iteration counters live in slot it % 3: iteration it fills its own slot and the list
// lengths of slot (it+1) % 3; slot (it+1) % 3 is cleared when iteration it begins (its last
// readers belong to iteration it-2).  List buffers alternate by iteration parity.
struct Slot {
    unsigned long long cnt[CNT_WORDS];  // log record layout
    // n_dv and n_da are adjacent and 8-byte aligned: both are reserved with one 64-bit atomic
    int n_dv, n_da, n_vl;   // dirty vertices, affected anchors, violation list of this iteration
    int n_tc;               // branch cells of f on a dirty vertex whose codes changed (touched)
    int n_db;               // branches with a touched cell
    int n_scan;             // branch cells examined to settle those branches
    int n_frz;              // listed anchors frozen by this iteration (freeze list length)
};

static_assert(offsetof(Slot, n_dv) % 8 == 0 && offsetof(Slot, n_da) == offsetof(Slot, n_dv) + 4,
              "n_dv, n_da reserved as one 64-bit word");

struct Ctl {
    int it;                 // current iteration
    int done;               // 0 running, 1 converged, 2 iteration cap, 3 stalled
    int paused;             // 1: the resident loop stopped before a large iteration (host runs it)
    int cand_sel;           // current troublemaker candidate list (cand[cand_sel])
    int n_cand[2];
    int c_it, s_it;
    long long residual;
    unsigned long long ph[3];   // wall-clock ticks in the resident loop: troublemaker, gradient, violation passes
    // frozen anchors (violations whose every target is floored, see freeze_pass): their
    // violations by type, the number of distinct vertices they request, ftgt entries in use
    unsigned long long dead_cnt[8];
    unsigned long long dead_distinct;
    int n_ftgt;
    int n_dead;             // frozen anchors (in LDS while the resident loop runs)
    int n_v0;               // violating anchors listed by a classification pass: iteration 0's in
                            // vl[0], a later dense iteration's in vl[it & 1]
    // full-grid form: the current iteration is dense (every vertex and anchor, see phase_grad);
    // nomark: the last violation pass made no dirty/affected lists, so the next iteration is dense
    int dense, nomark;
    Slot slot[3];
};

// Buffers of one job.  The host fills FrontierBufs (plain pointers); device code reads the same
// bytes as a FrontierView, whose pointers carry the global address space in the device pass, so
// accesses through them compile to global rather than flat instructions even when the structure
// is read from memory.  Both are generated from one field list and have one layout.
#if defined(__HIP_DEVICE_COMPILE__)
#define DMT_GPTR(T) __attribute__((address_space(1))) T*
#else
#define DMT_GPTR(T) T*
#endif
#define DMT_PTR(T) T*

#define DMT_FRONTIER_FIELDS(P)                                                                     \
    P(Ctl) ctl;                                                                                    \
    P(const float) f;                                                                              \
    P(const float) gh;                                                                             \
    P(const float) lo;                                                                             \
    P(float) gb[2];           /* g^(k) in gb[k & 1] */                                             \
    P(uint8_t) state;                                                                              \
    P(const uint8_t) fpl;                                                                          \
    P(uint8_t) gpl;                                                                                \
    P(uint32_t) vmask;        /* violating planes per anchor */                                    \
    P(int) vl[2];             /* violation anchor lists */                                         \
    P(int) dvl[2];            /* dirty vertex lists */                                             \
    P(int) dal[2];            /* affected anchor lists */                                          \
    /* per-vertex stamps, interleaved in one array (entry i of each at [STAMP_STRIDE * i]) so   \
       that the claims around one vertex touch one cache line and one page: */                    \
    P(unsigned) vstamp;       /* dirty-vertex stamps */                                            \
    /* affected-anchor stamps by iteration parity: iteration k's in [k & 1]; the edits of         \
       iteration k mark [(k+1) & 1] while [k & 1] is still read */                                 \
    P(unsigned) astamp[2];                                                                         \
    P(unsigned) rstamp;       /* request stamps */                                                 \
    /* frozen anchors: per anchor the offset of its targets in ftgt (ftgt_cap entries), per       \
       vertex the number of frozen violations requesting it, and an iteration's freeze list */     \
    P(int) fofs;                                                                                   \
    P(int) ftgt;                                                                                   \
    P(unsigned) dreq;                                                                              \
    P(int) frz;                                                                                    \
    int ftgt_cap;                                                                                  \
    P(long long) log;         /* DMT_LOG_WORDS per iteration */                                    \
    int log_cap;              /* records log can hold */                                           \
    int ndim;                 /* 2 or 3 */                                                         \
    Dims dm;                                                                                       \
    /* separatrix branches of f */                                                                 \
    P(const int) dcell;                                                                            \
    P(const int) dcbr;                                                                             \
    P(const int) dterm;                                                                            \
    P(const int) acell;                                                                            \
    P(const int) acbr;                                                                             \
    P(const int) aterm;                                                                            \
    P(const int64_t) doff;                                                                         \
    P(const int64_t) aoff;                                                                         \
    P(int) dfirst;            /* first cell of each branch whose g pairing differs (INF32: none) */ \
    P(int) afirst;                                                                                 \
    long long n_dcell, n_acell;                                                                    \
    int n_desc, n_asc;                                                                             \
    /* vertex -> branch cells containing it, CSR: entries vstart[v] .. vstart[v+1] of ecell, each \
       a branch cell index (descending k, ascending n_dcell + k); branch ids: descending b,        \
       ascending n_desc + b */                                                                     \
    P(const int) vstart;                                                                           \
    P(const int) ecell;                                                                            \
    P(unsigned) bstamp;       /* touched-branch stamps */                                          \
    P(int) tcl;               /* touched cells of the current iteration */                         \
    P(int) dbl;               /* touched branches of the current iteration */                      \
    /* per branch id: the first touched cell that differs, packed with its target (cell << 32 |   \
       target; all ones between), and the target of the branch's first differing cell */          \
    P(unsigned long long) newmin;                                                                  \
    P(int) btgt;                                                                                   \
    /* branches whose first differing cell may be set (a superset of them), for the separatrix    \
       step; inlist marks the members */                                                           \
    P(int) cand[2];                                                                                \
    P(uint8_t) inlist;                                                                             \
    /* saddle-saddle connectors (3D, tier 4, DMT_F_SADDLE_SADDLE): the edges of f's 2-saddles,    \
       two queues of edge ids for the walk down f's 1-2 V-paths, and per-edge stamps; edge id =  \
       (c - 1) * n + anchor for the edge from anchor to anchor + c (c: direction bits 1..7) */      \
    P(const int) ss_src;                                                                           \
    P(int) ss_q[2];                                                                                \
    P(unsigned) ss_stamp;                                                                          \
    int n_ss_src;                                                                                  \
    int ss_on;                                                                                     \
    float delta;                                                                                   \
    int q_max, tier;                                                                               \
    long long max_iters;

struct FrontierBufs {
    DMT_FRONTIER_FIELDS(DMT_PTR)
};

struct FrontierView {
    DMT_FRONTIER_FIELDS(DMT_GPTR)
};

static_assert(sizeof(FrontierView) == sizeof(FrontierBufs), "one layout");

__device__ __forceinline__ const FrontierView& view(const FrontierBufs& b) {
    return *reinterpret_cast<const FrontierView*>(&b);
}

__device__ __forceinline__ int ld_relaxed(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_relaxed(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Reserves one slot per lane with pred set, one atomic per wave; returns the lane's index.
__device__ __forceinline__ int wave_append(bool pred, int* counter) {
    const unsigned long long b = __ballot(pred);
    if (b == 0) return -1;
    const int lane = __lane_id();
    const int leader = __ffsll((long long)b) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, __popcll(b));
    base = __shfl(base, leader);
    return base + __popcll(b & ((1ull << lane) - 1ull));
}

// Reserves k slots per lane (k >= 0), one atomic per wave; whole waves call it.  Returns the
// lane's first index (unspecified when the wave reserves nothing).
__device__ __forceinline__ int wave_append_n(int k, int* counter) {
    const int lane = __lane_id();
    int incl = k;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    const int total = __shfl(incl, 63, 64);
    int base = 0;
    if (total != 0) {
        if (lane == 63) base = atomicAdd(counter, total);
        base = __shfl(base, 63, 64);
    }
    return base + incl - k;
}

// Two appends at once to a pair of adjacent counters (pair[0], pair[1], 8-byte aligned): k0 and
// k1 slots per lane (each below 2^10), one scan and one 64-bit atomic per wave; whole waves call
// it.  Returns the lane's first index in each list through i0 and i1.
__device__ __forceinline__ void wave_append_pair(int k0, int k1, int* pair, int& i0, int& i1) {
    const int lane = __lane_id();
    const int k = k0 | k1 << 16;
    int incl = k;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    const int total = __shfl(incl, 63, 64);
    unsigned long long base = 0;
    if (total != 0) {
        if (lane == 63)
            base = atomicAdd(reinterpret_cast<unsigned long long*>(pair),
                             (unsigned long long)(unsigned)(total & 0xffff) |
                                 (unsigned long long)(unsigned)(total >> 16) << 32);
        base = __shfl(base, 63, 64);
    }
    const int ex = incl - k;
    i0 = (int)(unsigned)base + (ex & 0xffff);
    i1 = (int)(base >> 32) + (ex >> 16);
}

// Lists are walked in rounds of gsize items, item base + gtid in a round; a wave whose first
// item lies past the end leaves the loop (a wave-uniform test, so wave-level collectives in the
// body stay safe), which keeps idle waves from competing with working ones for issue slots.
__device__ __forceinline__ bool wave_done(int base, int gtid, int n) {
    return base + (gtid & ~63) >= n;
}

// The counter slots of the workgroup-resident loop live in LDS while the loop runs (copied in
// from the job's control block when it starts and back when it stops); the full-grid phases
// use the control block itself.
__shared__ Slot wg_slots[3];
__shared__ int wg_n_dead;

// Control words the resident loop keeps in LDS while it runs, like the slots (copied in when it
// starts and back when it stops): the iteration, its outcome, the step counts and the
// troublemaker candidate lists' selector and lengths.
struct WgCtl {
    int it, done, c_it, s_it, cand_sel, n_cand[2];
};
__shared__ WgCtl wg_ctl;

template <bool WG = false>
__device__ __forceinline__ int* cand_sel_of(const FrontierView& B) {
    if constexpr (WG) return &wg_ctl.cand_sel;
    else return &B.ctl->cand_sel;
}

template <bool WG = false>
__device__ __forceinline__ int* n_cand_of(const FrontierView& B, int sel) {
    if constexpr (WG) return &wg_ctl.n_cand[sel];
    else return &B.ctl->n_cand[sel];
}

// Adds each thread's counts cnt[0, NC) to the slot counters cnt_out.  The resident loop's slots
// are in LDS, where a lane adds its non-zero counts directly; the full-grid form sums the block
// in LDS first and adds the block's totals to the slots in global memory.
template <bool WG, int NC>
__device__ __forceinline__ void add_counters(unsigned long long* cnt_out, const int* cnt) {
    if constexpr (WG) {
#pragma unroll
        for (int k = 0; k < NC; k++)
            if (cnt[k]) atomicAdd(&cnt_out[k], (unsigned long long)cnt[k]);
    } else {
        block_add_counters<NC>(cnt_out, cnt);
    }
}

template <bool WG = false>
__device__ __forceinline__ Slot& slot_of(const FrontierView& B, int it) {
    if constexpr (WG) return wg_slots[it % 3];
    else return B.ctl->slot[it % 3];
}

// Number of frozen anchors of the job (the resident loop keeps it in LDS).
template <bool WG = false>
__device__ __forceinline__ int* n_dead_of(const FrontierView& B) {
    if constexpr (WG) return &wg_n_dead;
    else return &B.ctl->n_dead;
}

__device__ __forceinline__ unsigned long long c_total(const Slot& s) {
    unsigned long long t = 0;
#pragma unroll
    for (int k = CNT_FP0; k < CNT_FP0 + 8; k++) t += ld_relaxed(&s.cnt[k]);
    return t;
}

// Violations of iteration it: critical-cell violations, else (tier >= 3) troublemakers.
__device__ __forceinline__ unsigned long long violations(const FrontierView& B, int it) {
    const Slot& s = slot_of(B, it);
    const unsigned long long ct = c_total(s);
    if (ct) return ct;
    return B.tier >= 3 ? ld_relaxed(&s.cnt[CNT_TM_DESC]) + ld_relaxed(&s.cnt[CNT_TM_ASC]) +
                             ld_relaxed(&s.cnt[CNT_TM_SS])
                       : 0ull;
}

// ---- Equation 2 on one vertex, and the neighbourhood an edit makes dirty -------------------

// Equation 2 on vertex v given its state byte st, g_hat and floor (loaded by the caller).
__device__ __forceinline__ bool apply_vertex(const FrontierView& B, int v, int it, uint8_t st, float ghv, float l) {
    if (st & 0x80) return false;
    const int q = st & 7;
    const float t = fmaf(-(float)(q + 1), B.delta, ghv);
    float* gn = B.gb[(it + 1) & 1];
    if (q < B.q_max && t >= l) {
        B.state[v] = (uint8_t)(q + 1);
        gn[v] = t;
    } else {
        B.state[v] = (uint8_t)(0x80 | q);
        gn[v] = l;
    }
    return true;
}

// Marks the closed 1-ring of an edited vertex as dirty and the anchors of cells touching it as
// affected, for iteration it + 1.  Lanes without an edit pass changed = false; whole waves
// call it.  Two forms, chosen per wave:
//  * few edits (all claims of the wave fit one round): the claims (edited vertex, slot) are
//    spread over the lanes, one stamp atomic per lane; winners appended with one atomic per list;
//  * otherwise each edited lane claims its NV ring slots and NA anchors itself, with no branches
//    between the atomics (a slot outside the grid issues a maximum with 0 on the vertex's own
//    entry, which changes nothing), so all are in flight at once.
template <int D, bool WG = false>
__device__ __forceinline__ void mark_neighbourhood(const FrontierView& B, const Dims& dm, bool changed, int v,
                                                   int it) {
    constexpr auto& g = G<D>::g;
    constexpr int NV = Geom<D>::NS + 1;
    constexpr int NA = g.naff;
    constexpr int PER = NV + NA;
    const unsigned long long mask = __ballot(changed);
    if (mask == 0) return;
    const int nxt = (it + 1) & 1;
    Slot& N1 = slot_of<WG>(B, it + 1);
    const unsigned stamp = (unsigned)it + 1u;
    int x = 0, y = 0, z = 0;
    if (changed) coords(dm, v, x, y, z);
    const int total = __popcll(mask) * PER;
    if (total <= 64) {
        const int cl = __lane_id();
        const bool valid = cl < total;
        const int k = valid ? cl / PER : 0;      // k-th edited lane of the wave
        const int slot = valid ? cl - k * PER : 0;
        unsigned long long m = mask;
        for (int r = 0; r < k; r++) m &= m - 1ull;
        const int src = __ffsll((long long)m) - 1;
        const int vv = __shfl(v, src, 64);
        const int sx = __shfl(x, src, 64), sy = __shfl(y, src, 64), sz = __shfl(z, src, 64);
        int dx = 0, dy = 0, dz = 0;
        const bool ring = slot < NV;
        if (ring) {
            if (slot > 0) { dx = g.slot_d[slot - 1][0]; dy = g.slot_d[slot - 1][1]; dz = g.slot_d[slot - 1][2]; }
        } else {
            dx = g.aff_d[slot - NV][0]; dy = g.aff_d[slot - NV][1]; dz = g.aff_d[slot - NV][2];
        }
        const bool ok = valid && (unsigned)(sx + dx) < (unsigned)dm.nx && (unsigned)(sy + dy) < (unsigned)dm.ny &&
                        (unsigned)(sz + dz) < (unsigned)dm.nz;
        const int t = vv + dx + dm.nx * dy + dm.nxy * dz;
        bool won = false;
        if (ok) won = atomicMax((ring ? B.vstamp : B.astamp[nxt]) + (size_t)STAMP_STRIDE * t, stamp) < stamp;
        // both appends with one 64-bit atomic on the adjacent counters n_dv, n_da
        const unsigned long long bv = __ballot(won && ring), ba = __ballot(won && !ring);
        unsigned long long base = 0;
        if (__lane_id() == 0 && (bv | ba))
            base = atomicAdd(reinterpret_cast<unsigned long long*>(&N1.n_dv),
                             (unsigned long long)__popcll(bv) | (unsigned long long)__popcll(ba) << 32);
        base = __shfl(base, 0, 64);
        const unsigned long long below = (1ull << __lane_id()) - 1ull;
        const int iv = (int)(unsigned)base + __popcll(bv & below);
        const int ia = (int)(base >> 32) + __popcll(ba & below);
        if (won) {
            if (ring) B.dvl[nxt][iv] = t;
            else B.dal[nxt][ia] = t;
        }
        return;
    }
    uint32_t mv = 0;
    uint64_t ma = 0;
    if (changed) {
        unsigned* vs = B.vstamp;
        unsigned* as = B.astamp[nxt];
        unsigned ov[NV];
        unsigned oa[NA];
        uint32_t okv = 0;
        uint64_t oka = 0;
#pragma unroll
        for (int s = 0; s < NV; s++) {
            const int dx = s == 0 ? 0 : g.slot_d[s == 0 ? 0 : s - 1][0];
            const int dy = s == 0 ? 0 : g.slot_d[s == 0 ? 0 : s - 1][1];
            const int dz = s == 0 ? 0 : g.slot_d[s == 0 ? 0 : s - 1][2];
            const bool ok = (unsigned)(x + dx) < (unsigned)dm.nx && (unsigned)(y + dy) < (unsigned)dm.ny &&
                            (unsigned)(z + dz) < (unsigned)dm.nz;
            okv |= (uint32_t)ok << s;
            ov[s] = atomicMax(vs + (size_t)STAMP_STRIDE * (ok ? v + dx + dm.nx * dy + dm.nxy * dz : v), ok ? stamp : 0u);
        }
#pragma unroll
        for (int j = 0; j < NA; j++) {
            const int dx = g.aff_d[j][0], dy = g.aff_d[j][1], dz = g.aff_d[j][2];
            const bool ok = x + dx >= 0 && y + dy >= 0 && z + dz >= 0 && x + dx < dm.nx && y + dy < dm.ny &&
                            z + dz < dm.nz;
            oka |= (uint64_t)ok << j;
            oa[j] = atomicMax(as + (size_t)STAMP_STRIDE * (ok ? v + dx + dm.nx * dy + dm.nxy * dz : v), ok ? stamp : 0u);
        }
#pragma unroll
        for (int s = 0; s < NV; s++)
            if (((okv >> s) & 1u) && ov[s] < stamp) mv |= 1u << s;
#pragma unroll
        for (int j = 0; j < NA; j++)
            if (((oka >> j) & 1ull) && oa[j] < stamp) ma |= 1ull << j;
    }
    int iv, ia;
    wave_append_pair(__popc(mv), __popcll(ma), &N1.n_dv, iv, ia);
    if (!changed) return;
    int* dv = B.dvl[nxt];
    int* da = B.dal[nxt];
#pragma unroll
    for (int s = 0; s < NV; s++) {
        if (mv & (1u << s)) {
            const int dx = s == 0 ? 0 : g.slot_d[s == 0 ? 0 : s - 1][0];
            const int dy = s == 0 ? 0 : g.slot_d[s == 0 ? 0 : s - 1][1];
            const int dz = s == 0 ? 0 : g.slot_d[s == 0 ? 0 : s - 1][2];
            dv[iv++] = v + dx + dm.nx * dy + dm.nxy * dz;
        }
    }
#pragma unroll
    for (int j = 0; j < NA; j++) {
        if (ma & (1ull << j)) da[ia++] = v + g.aff_d[j][0] + dm.nx * g.aff_d[j][1] + dm.nxy * g.aff_d[j][2];
    }
}

// Request of vertex v (v < 0: none) in iteration it: the first requester counts it in rc[0]
// and, when edits are allowed, edits it (counted in rc[1]) and marks its neighbourhood.
// With floored, *floored is cleared unless v is already at its floor (final).  With frozen (the
// job has frozen anchors), a vertex that frozen violations request (dreq[v] > 0) is counted among
// their distinct targets instead.
// Without mark (a violation pass whose next iteration is dense), the neighbourhood is not marked.
template <int D, bool WG = false>
__device__ __forceinline__ void request_apply(const FrontierView& B, const Dims& dm, int v, int it, bool edit,
                                              int* rc, bool* floored = nullptr, bool frozen = false,
                                              bool mark = true) {
    const unsigned stamp = (unsigned)it + 1u;
    bool changed = false;
    if (v >= 0) {
        // the vertex's state, g_hat and floor are read while the stamp atomic is in flight (only
        // the stamp winner edits v, so they are current whenever they are used)
        const uint8_t st = B.state[v];
        const float ghv = B.gh[v], l = B.lo[v];
        const unsigned dq = frozen ? B.dreq[v] : 0u;
        if (floored) *floored &= (st & 0x80) != 0;
        if (atomicMax(&B.rstamp[(size_t)STAMP_STRIDE * v], stamp) < stamp) {
            if (dq == 0) rc[0]++;
            if (edit) changed = apply_vertex(B, v, it, st, ghv, l);
            if (changed) rc[1]++;
        }
    }
    if (mark) mark_neighbourhood<D, WG>(B, dm, changed, v, it);   // mark is uniform over the wave
}

// ---- violation mask of one anchor: planes whose criticality differs between f and g --------

// vmask word: bits 0..25 the violating planes; VM_QUIET: every target of the anchor's violations
// was at its floor when last requested; VM_DEAD: the anchor is frozen (its targets are in ftgt).
constexpr uint32_t VM_PLANES = (1u << 26) - 1u;
constexpr uint32_t VM_QUIET = 1u << 30;
constexpr uint32_t VM_DEAD = 1u << 31;

// Violation mask of anchor a.  The anchor's codes are read as whole 8-byte words (its group is
// 8-byte aligned and in bounds for every anchor), all loads in flight together; planes whose
// cell does not exist, or that the tier ignores, are masked afterwards.  With fpk
// (2D), its f codes are also returned packed (plane P in byte P) with bit 63 set, so its targets
// need not load them again.
template <int D>
__device__ __forceinline__ uint32_t vmask_anchor(const Dims& dm, int a, int x, int y, int z,
                                                 const uint8_t* __restrict__ fpl, const uint8_t* __restrict__ gpl,
                                                 int tier, uint64_t* fpk = nullptr) {
    constexpr int W = plane_stride<D>() / 8;
    uint64_t fw[W], gw[W];
    const uint64_t* fp = reinterpret_cast<const uint64_t*>(fpl + pidx<D>(0, a));
    const uint64_t* gp = reinterpret_cast<const uint64_t*>(gpl + pidx<D>(0, a));
#pragma unroll
    for (int k = 0; k < W; k++) {
        fw[k] = fp[k];
        gw[k] = gp[k];
    }
    uint8_t fc[Geom<D>::NB], gc[Geom<D>::NB];
    static_for<0, Geom<D>::NB>([&](auto pc) {
        constexpr int P = decltype(pc)::value;
        fc[P] = (uint8_t)(fw[P / 8] >> (8 * (P % 8)));
        gc[P] = (uint8_t)(gw[P / 8] >> (8 * (P % 8)));
    });
    if constexpr (D == 2) {
        if (fpk) *fpk = fw[0] | (1ull << 63);   // byte 7 is padding
    }
    uint32_t m = 0;
    static_for<0, Geom<D>::NB>([&](auto pc) {
        constexpr int P = decltype(pc)::value;
        constexpr int dim = G<D>::g.bdim[P];
        const bool use = !(tier == 1 && dim != 0 && dim != D) && cell_exists<D, P>(dm, x, y, z);
        m |= (uint32_t)(use && ((fc[P] == CODE_CRIT) != (gc[P] == CODE_CRIT))) << P;
    });
    return m;
}

// ---- target of one violating plane (Rules A and B, as classify_plane) ---------------------

template <int D, int P>
__device__ __forceinline__ int plane_target(const FrontierView& B, const Dims& dm, int a, const float* gcur, int* cnt) {
    constexpr auto& g = G<D>::g;
    constexpr int dim = g.bdim[P];
    const uint8_t fc = B.fpl[pidx<D>(P, a)];
    const uint8_t gc = B.gpl[pidx<D>(P, a)];
    if (fc != CODE_CRIT) {
        cnt[2 * dim]++;
        return a + c27_lin(dm, fc & 63);
    }
    const int gx = gc & 63;
    const int xv = a + c27_lin(dm, gx);
    const float fx = B.f[xv];
    const bool up = (gc & CODE_UP) != 0;
    int best = -1;
    float gbest = 0.0f;
    int kx = 0;
    static_for<0, g.bnv[P]>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        constexpr int bx = G<D>::g.bvert[P][k][0], by = G<D>::g.bvert[P][k][1], bz = G<D>::g.bvert[P][k][2];
        constexpr int ck = c27_of(bx, by, bz);
        if (!up && ck == gx) { kx = k; return; }
        const int w = a + bx + dm.nx * by + dm.nxy * bz;
        if (!prec(B.f[w], w, fx, xv)) return;
        const float gw = gcur[w];
        if (best < 0 || prec(gw, w, gbest, best)) { best = w; gbest = gw; }
    });
    if (best < 0) {
        int fa = a, fp = 0;
        static_for<0, g.bnv[P]>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            if (k == kx) {
                fa = a + G<D>::g.facet_anchor[P][k][0] + dm.nx * G<D>::g.facet_anchor[P][k][1] +
                     dm.nxy * G<D>::g.facet_anchor[P][k][2];
                fp = G<D>::g.facet_plane[P][k];
            }
        });
        best = fa + c27_lin(dm, B.fpl[pidx<D>(fp, fa)] & 63);
    }
    cnt[2 * dim + 1]++;
    return best;
}

// plane p chosen at run time
template <int D, int P>
__device__ __forceinline__ int plane_target_dyn(int p, const FrontierView& B, const Dims& dm, int a, const float* gcur,
                                                int* cnt) {
    if (p == P) return plane_target<D, P>(B, dm, a, gcur, cnt);
    if constexpr (P + 1 < Geom<D>::NB) return plane_target_dyn<D, P + 1>(p, B, dm, a, gcur, cnt);
    return -1;
}

// Target of violating plane p (chosen at run time) of anchor a: a false positive (the cell is
// paired in f) takes the apex of its f-pair on one code path for every plane, so a wave whose
// lanes hold different planes does not run one path per plane; false negatives (rare) go through
// the per-plane code.
template <int D>
__device__ __forceinline__ int plane_target_any(int p, const FrontierView& B, const Dims& dm, int a, const float* gcur,
                                                int* cnt, uint64_t fpk = 0) {
    constexpr auto& g = G<D>::g;
    const uint8_t fc = (fpk >> 63) ? (uint8_t)(fpk >> (8 * p)) : B.fpl[pidx<D>(p, a)];
    if (fc != CODE_CRIT) {
        int dim = (p >= g.base[1]) + (p >= g.base[2]);
        if constexpr (D == 3) dim += (p >= g.base[3]);
        static_for<0, D + 1>([&](auto dc) {
            constexpr int d = decltype(dc)::value;
            if (dim == d) cnt[2 * d]++;
        });
        return a + c27_lin(dm, fc & 63);
    }
    return plane_target_dyn<D, 0>(p, B, dm, a, gcur, cnt);
}

// Requests (and, with edit, edits) the targets of the violating planes m of anchor a.  Whole
// waves call it; lanes without an anchor pass m = 0.  One plane per lane per round.
// quiet is cleared unless every target is already at its floor.
template <int D, bool WG = false>
__device__ __forceinline__ void anchor_requests(const FrontierView& B, const Dims& dm, int a, uint32_t m, int it,
                                                bool edit, int* cnt, int* rc, bool& quiet, bool frozen,
                                                bool track_quiet, uint64_t fpk = 0, bool mark = true) {
    const float* gcur = B.gb[it & 1];
    for (;;) {
        if (__ballot(m != 0) == 0) break;
        int target = -1;
        if (m != 0) {
            const int p = __ffs(m) - 1;
            m &= m - 1u;
            target = plane_target_any<D>(p, B, dm, a, gcur, cnt, fpk);
        }
        request_apply<D, WG>(B, dm, target, it, edit, rc, track_quiet ? &quiet : nullptr, frozen, mark);
    }
}

// ---- frozen anchors ------------------------------------------------------------------------
//
// A violation whose target is at its floor requests it again every iteration and nothing
// changes; near fp32 floor collisions hundreds of thousands of such violations can outlive every
// other edit.  An anchor that stays listed (not affected) for a second iteration with every target
// at its floor is frozen: it leaves the violation list, its targets are kept in ftgt, and its
// violations are counted through per-type totals (dead_cnt) and the per-vertex request counts
// (dreq, whose non-zero entries make up dead_distinct), which every iteration adds to its
// counters exactly as if the anchor had requested its targets again.  When an edit affects a
// frozen anchor, the gradient pass of the next iteration revives it (its counts are removed)
// and the violation pass examines it afresh.  The log, the statistics and the output are those
// of processing every violation every iteration.

// dimension of the cells of plane p
template <int D>
__device__ __forceinline__ int plane_dim(int p) {
    constexpr auto& g = G<D>::g;
    int d = (p >= g.base[1]) + (p >= g.base[2]);
    if constexpr (D == 3) d += (p >= g.base[3]);
    return d;
}

// Revives the frozen anchors among iteration it's affected anchors.
template <int D, bool WG = false>
__device__ __forceinline__ void revive_pass(const FrontierView& B, const Dims& dm, int it, int gtid, int gsize) {
    if (ld_relaxed(n_dead_of<WG>(B)) == 0) return;
    const Slot& S = slot_of<WG>(B, it);
    const int na = ld_relaxed(&S.n_da);
    const int* alist = B.dal[it & 1];
    int dc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int dd = 0, nr = 0;
    for (int i = gtid; i < na; i += gsize) {
        const int a = alist[i];
        const uint32_t mv = B.vmask[a];
        if (!(mv & VM_DEAD)) continue;
        uint32_t m = mv & VM_PLANES;
        B.vmask[a] = m;
        nr++;
        const int o = B.fofs[a];
        for (int k = 0; m != 0; k++) {
            const int p = __ffs(m) - 1;
            m &= m - 1u;
            const int d = plane_dim<D>(p);
            dc[2 * d + (B.fpl[pidx<D>(p, a)] == CODE_CRIT ? 1 : 0)]++;
            if (atomicSub(&B.dreq[B.ftgt[o + k]], 1u) == 1u) dd++;
        }
    }
    for (int k = 0; k < 8; k++)
        if (dc[k]) atomicAdd(&B.ctl->dead_cnt[k], (unsigned long long)(-(long long)dc[k]));
    if (dd) atomicAdd(&B.ctl->dead_distinct, (unsigned long long)(-(long long)dd));
    if (nr) atomicSub(n_dead_of<WG>(B), nr);
}

// Freezes the anchors the violation pass of iteration it listed for freezing: records their
// targets (the same this iteration requested) and adds their violations to the frozen counts,
// which iteration it + 1 onward uses.  With ftgt full the anchor stays in the violation list.
template <int D, bool WG = false>
__device__ __forceinline__ void freeze_pass(const FrontierView& B, const Dims& dm, int it, int gtid, int gsize) {
    const Slot& S = slot_of<WG>(B, it);
    const int nf = ld_relaxed(&S.n_frz);
    const float* gcur = B.gb[it & 1];
    int dc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int dd = 0, nz = 0;
    for (int i = gtid; i < nf; i += gsize) {
        const int a = B.frz[i];
        uint32_t m = B.vmask[a] & VM_PLANES;
        const int k = __popc(m);
        // once ftgt is full no more space is taken (the counter stays far below 2^31)
        int o = -1;
        if (ld_relaxed(&B.ctl->n_ftgt) + k <= B.ftgt_cap) o = atomicAdd(&B.ctl->n_ftgt, k);
        if (o < 0 || o + k > B.ftgt_cap) {
            const int idx = atomicAdd(&slot_of<WG>(B, it + 1).n_vl, 1);
            B.vl[(it + 1) & 1][idx] = a;
            continue;
        }
        B.fofs[a] = o;
        for (int j = 0; m != 0; j++) {
            const int p = __ffs(m) - 1;
            m &= m - 1u;
            const int t = plane_target_any<D>(p, B, dm, a, gcur, dc);
            B.ftgt[o + j] = t;
            if (atomicAdd(&B.dreq[t], 1u) == 0u) dd++;
        }
        B.vmask[a] = (B.vmask[a] & VM_PLANES) | VM_DEAD;
        nz++;
    }
    for (int k = 0; k < 8; k++)
        if (dc[k]) atomicAdd(&B.ctl->dead_cnt[k], (unsigned long long)dc[k]);
    if (dd) atomicAdd(&B.ctl->dead_distinct, (unsigned long long)dd);
    if (nz) atomicAdd(n_dead_of<WG>(B), nz);
}

// ---- phases ------------------------------------------------------------------------------

// Gradient of g^(it) for the dirty vertices (every vertex at iteration 0); brings the write
// buffer up to date on them; lists the cells of f's branches that contain a dirty vertex (the
// only branch cells whose pairing can have changed); clears the next slot.
template <int D, bool WG = false>
__device__ __forceinline__ void phase_grad(const FrontierView& B, const Dims& dm, int it, int gtid, int gsize) {
    if (gtid == 0) {
        Slot& s = slot_of<WG>(B, it + 1);
        for (int k = 0; k < CNT_WORDS; k++) s.cnt[k] = 0;
        s.n_dv = s.n_da = s.n_vl = s.n_tc = s.n_db = s.n_scan = s.n_frz = 0;
    }
    const float* gcur = B.gb[it & 1];
    float* gnext = B.gb[(it + 1) & 1];
    if (it == 0) {
        for (int i = gtid; i < dm.n; i += gsize) grad_vertex<D>(i, gcur, B.gpl, dm);
        return;
    }
    Slot& S = slot_of<WG>(B, it);
    if constexpr (!WG) {
        // Dense iteration (full-grid form): when the last violation pass made no lists, or its
        // lists cover more than 1/DENSE_DIV of the grid, every vertex's gradient is recomputed and
        // copied across, and a classification pass (k_fr_classify_dense) classifies every anchor
        // and lists the violating ones for the violation pass, as at iteration 0.  The
        // frozen anchors are all revived (their masks are recomputed) and the first differing
        // cell of every branch is found afresh.  It is the frontier iteration with every vertex
        // dirty and every anchor affected, which gives the same result.
        Ctl* c = B.ctl;
        const bool dense = ld_relaxed(&c->nomark) != 0 ||
                           (long long)ld_relaxed(&S.n_dv) + ld_relaxed(&S.n_da) > (long long)dm.n / DENSE_DIV;
        if (gtid == 0) c->dense = dense;
        if (dense) {
            if (gtid == 0) {
                c->n_v0 = 0;
                c->cand_sel = 0;
                c->n_cand[0] = c->n_cand[1] = 0;
                c->n_dead = 0;
                for (int k = 0; k < 8; k++) c->dead_cnt[k] = 0;
                c->dead_distinct = 0;
                c->n_ftgt = 0;
            }
            for (int i = gtid; i < dm.n; i += gsize) {
                grad_vertex<D>(i, gcur, B.gpl, dm);
                gnext[i] = gcur[i];
                if (B.dreq) B.dreq[i] = 0u;
            }
            if (B.tier >= 3) {
                for (int k = gtid; k < B.n_desc; k += gsize) B.dfirst[k] = INF32;
                for (int k = gtid; k < B.n_asc; k += gsize) B.afirst[k] = INF32;
            }
            return;
        }
    }
    const int n = ld_relaxed(&S.n_dv);
    const int* list = B.dvl[it & 1];
    // With branch tracking, the branch cells on each dirty vertex whose vertex or top-cell codes
    // changed are listed as touched (each dirty vertex is listed once per iteration, so each cell
    // appears at most D + 1 times).  A cell's code is written only by the vertex whose lower star
    // holds it, which is one of the cell's vertices: a changed cell is always listed.
    const bool track = B.vstart != nullptr;
    for (int base = 0; base < n; base += gsize) {
        if (wave_done(base, gtid, n)) break;
        const int i = base + gtid;
        int e0 = 0, e1 = 0;
        if (i < n) {
            const int t = list[i];
            // the vertex's branch-cell range is loaded with its neighbourhood, before the code
            // stores, so a changed vertex does not wait for it afterwards
            const int s0 = track ? B.vstart[t] : 0, s1 = track ? B.vstart[t + 1] : 0;
            const bool ch = grad_vertex<D, true>(t, gcur, B.gpl, dm);
            gnext[t] = gcur[t];
            if (track && ch) {
                e0 = s0;
                e1 = s1;
            }
        }
        if (track) {
            int pos = wave_append_n(e1 - e0, &S.n_tc);
            for (int e = e0; e < e1; e++) B.tcl[pos++] = B.ecell[e];
        }
    }
    revive_pass<D, WG>(B, dm, it, gtid, gsize);
}

// Whether branch cell k (descending: a vertex, ascending: a top cell) is paired differently in
// g than in f; with tgt, also the troublemaker target it would have as its branch's first
// differing cell: the apex of its f-pair, read from the same f code.
template <int D>
__device__ __forceinline__ bool branch_cell_differs(const FrontierView& B, const Dims& dm, bool asc, long long k,
                                                    int* tgt = nullptr) {
    constexpr auto& g = G<D>::g;
    if (!asc) {
        const int v = B.dcell[k];
        const uint8_t fc = B.fpl[pidx<D>(0, v)];
        if (tgt) *tgt = v + c27_lin(dm, fc & 63);
        return fc != B.gpl[pidx<D>(0, v)];
    }
    const int T = B.acell[k];
    const int a = T / g.ntypes[D];
    const int tp = T - a * g.ntypes[D] + g.base[D];
    const size_t o = pidx<D>(tp, a);
    const uint8_t fc = B.fpl[o];
    if (tgt) *tgt = a + c27_lin(dm, fc & 63);
    return fc != B.gpl[o];
}

// Dense scan for the first differing cell of every branch (first[] at INF32 before): lane k of
// a wave takes cell base + k, so a wave covers consecutive cells, and the cells of one branch are
// consecutive; only the first differing cell of each branch run within the wave lowers first[]
// (one atomic per run instead of one per differing cell, which on a field where most cells
// differ put many atomics on one address).
template <int D>
__device__ __forceinline__ void dense_first_scan(const FrontierView& B, const Dims& dm, bool asc, int gtid,
                                                 int gsize) {
    const long long n = asc ? B.n_acell : B.n_dcell;
    const int* cbr = asc ? B.acbr : B.dcbr;
    int* first = asc ? B.afirst : B.dfirst;
    const int lane = __lane_id();
    const unsigned long long below = (1ull << lane) - 1ull;
    for (long long k0 = gtid - lane; k0 < n; k0 += gsize) {   // k0: the wave's first cell
        const long long k = k0 + lane;
        const bool in = k < n;
        const int br = in ? cbr[k] : -1;
        const bool d = in && branch_cell_differs<D>(B, dm, asc, k);
        const int prev = __shfl_up(br, 1, 64);
        const unsigned long long starts = __ballot(lane == 0 || br != prev);   // first lane of each run
        const unsigned long long diff = __ballot(d);
        if (d) {
            // this lane's run starts at the highest start at or below it; an earlier differing
            // lane of the same run holds the run's minimum
            const int run0 = 63 - __clzll(starts & (below | (1ull << lane)));
            const unsigned long long earlier = diff & below;
            const int prevd = earlier ? 63 - __clzll(earlier) : -1;
            if (prevd < run0) atomicMin(&first[br], (int)k);
        }
    }
}

constexpr unsigned long long NEWMIN_NONE = ~0ull;

__device__ __forceinline__ unsigned long long newmin_pack(long long k, int target) {
    return (unsigned long long)k << 32 | (unsigned)target;
}

// Keeping first[] (each f-branch's first cell whose g pairing differs) current, in two passes
// separated by a synchronisation.  Before iteration it, no cell of branch b before first[b]
// differed, and only the touched cells can have changed since.
// Pass A (touched_cells): each touched cell marks its branch and, if it differs now, lowers
// newmin[branch] to it.
template <int D, bool WG = false>
__device__ __forceinline__ void touched_cells(const FrontierView& B, const Dims& dm, int it, int gtid, int gsize) {
    Slot& S = slot_of<WG>(B, it);
    const int n = ld_relaxed(&S.n_tc);
    const unsigned stamp = (unsigned)it + 1u;
    for (int base = 0; base < n; base += gsize) {
        if (wave_done(base, gtid, n)) break;
        const int i0 = base + gtid;
        bool mine = false;
        int bb = 0;
        if (i0 < n) {
            const int kk = B.tcl[i0];
            const bool asc = kk >= B.n_dcell;
            const int k = asc ? kk - (int)B.n_dcell : kk;
            bb = asc ? B.n_desc + B.acbr[k] : B.dcbr[k];
            mine = atomicMax(&B.bstamp[bb], stamp) < stamp;
            int t;
            if (branch_cell_differs<D>(B, dm, asc, k, &t)) atomicMin(&B.newmin[bb], newmin_pack(k, t));
        }
        const int idx = wave_append(mine, &S.n_db);
        if (mine) B.dbl[idx] = bb;
    }
}

template <int D>
__device__ __forceinline__ void cand_rebuild(const FrontierView& B, int gtid, int gsize);

// Pass B (phase_bscan): for each marked branch, if its old first cell still differs the new
// first is the smaller of it and newmin; otherwise the first differing cell after the old first
// (searched only up to newmin), else newmin.  One wave per branch, 64 cells per step.  The
// target of the new first cell (btgt) comes from the code that decided it.
template <int D, bool WG = false>
__device__ __forceinline__ void phase_bscan(const FrontierView& B, const Dims& dm, int it, int gtid, int gsize) {
    if (it == 0 || B.tier < 3) return;
    if constexpr (!WG) {
        if (ld_relaxed(&B.ctl->dense)) {   // first[] was found afresh by the dense scan
            cand_rebuild<D>(B, gtid, gsize);
            return;
        }
    }
    Slot& S = slot_of<WG>(B, it);
    const int n = ld_relaxed(&S.n_db);
    const int lane = __lane_id();
    const int sel = ld_relaxed(cand_sel_of<WG>(B));
    int scanned = 0;
    for (int i = gtid >> 6; i < n; i += gsize >> 6) {
        const int bb = B.dbl[i];
        const bool asc = bb >= B.n_desc;
        const int b = asc ? bb - B.n_desc : bb;
        int* first = asc ? B.afirst : B.dfirst;
        const int64_t* off = asc ? B.aoff : B.doff;
        const int old = first[b];
        const unsigned long long nmp = B.newmin[bb];
        const int nm = nmp == NEWMIN_NONE ? INF32 : (int)(nmp >> 32);
        const int nmt = (int)(unsigned)nmp;
        int res, rt;
        int ot = 0;
        if (old != INF32 && branch_cell_differs<D>(B, dm, asc, old, &ot)) {
            res = old < nm ? old : nm;
            rt = old < nm ? ot : nmt;
        } else {
            res = nm;
            rt = nmt;
            const long long hi = off[b + 1];
            const long long end = nm < hi ? nm : hi;
            long long k0 = old == INF32 ? end : (long long)old + 1;
            for (; k0 < end; k0 += 64) {
                const long long k = k0 + lane;
                int t = 0;
                const bool d = k < end && branch_cell_differs<D>(B, dm, asc, k, &t);
                const unsigned long long m = __ballot(d);
                scanned += 64;
                if (m) {
                    const int l = __ffsll((long long)m) - 1;
                    res = (int)(k0 + l);
                    rt = __shfl(t, l, 64);
                    break;
                }
            }
        }
        if (lane == 0) {
            first[b] = res;
            B.btgt[bb] = rt;
            B.newmin[bb] = NEWMIN_NONE;
            if (res != INF32 && !B.inlist[bb]) {
                B.inlist[bb] = 1;
                B.cand[sel][atomicAdd(n_cand_of<WG>(B, sel), 1)] = bb;
            }
        }
    }
    if (lane == 0 && scanned) atomicAdd(&S.n_scan, scanned);
}

// Violation masks of the affected anchors (every anchor at iteration 0), the targets of every
// violating anchor (edited at once when edit is set), the violation list of the next iteration,
// and the speculative first-difference scan along f's branches.
// Freezing (FREEZE) is done by the full-grid form, which runs the large iterations where many
// violations are listed, and by the 3D resident loop (3D density fields collide at their floors
// by the hundred thousand); the 2D resident loop keeps frozen anchors frozen and revives them but
// freezes none (its violation pass is the critical path of most 2D iterations), and a quiet bit it
// leaves on a listed anchor stays true (its targets are unchanged and final).
template <int D, bool WG = false, bool FREEZE = !WG || D == 3>
__device__ __forceinline__ void phase_vr(const FrontierView& B, const Dims& dm, int it, bool edit, int gtid,
                                         int gsize) {
    Slot& S = slot_of<WG>(B, it);
    int* n_next = &slot_of<WG>(B, it + 1).n_vl;
    int* next = B.vl[(it + 1) & 1];
    int cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int rc[2] = {0, 0};
    // One index space: the affected anchors get new masks; the anchors listed by the previous
    // iteration and not affected since keep theirs.  Iteration 0, and a dense iteration after it
    // (full-grid form, see phase_grad: every anchor affected), take the violating anchors that
    // the classification pass listed in vl[it & 1], with their masks computed there.
    const bool first = it == 0;
    bool all = false;
    if constexpr (!WG) all = !first && ld_relaxed(&B.ctl->dense) != 0;
    const bool dense = first || all;
    const int na = dense ? ld_relaxed(&B.ctl->n_v0) : ld_relaxed(&S.n_da);
    const int nl = dense ? 0 : ld_relaxed(&S.n_vl);
    const int ntot = na + nl;
    // a dense iteration after the first, whose previous iteration edited more than 1/NOMARK_DIV
    // of the vertices, marks no neighbourhoods (its own edits will be about as many): its next
    // iteration is dense too, and the full-grid form runs it.  Violations at floored targets edit
    // nothing, so a field stalled at its floors goes back to frontier iterations, which freeze them.
    const bool mark = !(dense && it > 0 &&
                        (long long)ld_relaxed(&slot_of<WG>(B, it - 1).cnt[CNT_CHANGED]) > (long long)dm.n / NOMARK_DIV);
    if (!WG && gtid == 0) B.ctl->nomark = !mark;
    const int* alist = B.dal[it & 1];
    const int* vlist = B.vl[it & 1];
    const unsigned astamp_it = (unsigned)it;
    const unsigned* astamp = B.astamp[it & 1];
    // the frozen violations (revived ones already removed by the gradient pass) count in this
    // iteration as they are
    const bool frozen = ld_relaxed(n_dead_of<WG>(B)) != 0;
    if (gtid == 0 && frozen) {
        for (int k = 0; k < 8; k++) {
            const unsigned long long d = ld_relaxed(&B.ctl->dead_cnt[k]);
            if (d) atomicAdd(&S.cnt[CNT_FP0 + k], d);
        }
        const unsigned long long dd = ld_relaxed(&B.ctl->dead_distinct);
        if (dd) atomicAdd(&S.cnt[CNT_NREQ], dd);
    }
    int* n_frz = &S.n_frz;
    for (int base = 0; base < ntot; base += gsize) {
        if (wave_done(base, gtid, ntot)) break;
        const int i0 = base + gtid;
        uint32_t m = 0, old_quiet = 0;
        uint64_t fpk = 0;   // the anchor's f codes, when loaded here (2D)
        int a = 0;
        bool listed = false;
        if (i0 < na && dense) {
            a = vlist[i0];
            m = B.vmask[a];
        } else if (i0 < na) {
            a = alist[i0];
            int x, y, z;
            coords(dm, a, x, y, z);
            m = vmask_anchor<D>(dm, a, x, y, z, B.fpl, B.gpl, B.tier, &fpk);
            B.vmask[a] = m;
        } else if (i0 < ntot) {
            a = vlist[i0 - na];
            if (astamp[(size_t)STAMP_STRIDE * a] != astamp_it) {
                const uint32_t mv = B.vmask[a];
                m = mv & VM_PLANES;
                old_quiet = mv & VM_QUIET;
                listed = true;
            }
        }
        // a listed anchor (not affected since it was last examined, so its targets are the same)
        // whose targets were all at their floor then is frozen after this pass
        const bool frz = FREEZE && listed && m != 0 && old_quiet;
        const int idx = wave_append(m != 0 && !frz, n_next);
        if (m != 0 && !frz) next[idx] = a;
        const int fi = wave_append(frz, n_frz);
        if (frz) B.frz[fi] = a;
        bool quiet = true;
        anchor_requests<D, WG>(B, dm, a, m, it, edit, cnt, rc, quiet, frozen, FREEZE, fpk, mark);
        // the quiet bit is rewritten only when it changes (rarely)
        if constexpr (FREEZE) {
            const uint32_t qb = (m != 0 && quiet) ? VM_QUIET : 0u;
            if ((i0 < na || (listed && !frz)) && qb != old_quiet) B.vmask[a] = m | qb;
        }
    }
    // first differing cell of the f-branches, kept up to date for the separatrix step: every
    // branch at iteration 0 (first[] starts at INF32), afterwards the branches listed by the
    // gradient pass (a later dense iteration's classification pass scans every branch)
    if (B.tier >= 3) {
        if (first) {
            dense_first_scan<D>(B, dm, false, gtid, gsize);
            dense_first_scan<D>(B, dm, true, gtid, gsize);
        } else if (!all) {
            touched_cells<D, WG>(B, dm, it, gtid, gsize);
        }
    }
    add_counters<WG, 8>(S.cnt + CNT_FP0, cnt);
    add_counters<WG, 2>(S.cnt + CNT_NREQ, rc);
}

// Troublemaker targets (apex of the f-pair of each branch's first differing cell), edited at
// once.  Only called when iteration it has no critical-cell violation.
template <int D, bool WG = false>
__device__ __forceinline__ void phase_sapply(const FrontierView& B, const Dims& dm, int it, bool edit, int gtid,
                                             int gsize) {
    constexpr auto& g = G<D>::g;
    int c[2] = {0, 0};
    int rc[2] = {0, 0};
    // the candidate list: members whose first differing cell is unset leave it, the others are
    // kept in the other buffer (the decision of this iteration makes it current)
    const int sel = ld_relaxed(cand_sel_of<WG>(B));
    const int nb = ld_relaxed(n_cand_of<WG>(B, sel));
    const int* cl = B.cand[sel];
    int* keep = B.cand[sel ^ 1];
    const bool mark = WG || ld_relaxed(&B.ctl->nomark) == 0;   // set by this iteration's violation pass
    for (int base = 0; base < nb; base += gsize) {
        if (wave_done(base, gtid, nb)) break;
        const int i0 = base + gtid;
        int target = -1;
        bool kept = false;
        int bb = 0;
        if (i0 < nb) {
            bb = cl[i0];
            const bool asc = bb >= B.n_desc;
            const int b = asc ? bb - B.n_desc : bb;
            const int* first = asc ? B.afirst : B.dfirst;
            const int* cells = asc ? B.acell : B.dcell;
            const int* term = asc ? B.aterm : B.dterm;
            const int k = first[b];
            const int tgt = B.btgt[bb];   // loaded beside first[b]; valid when it is set
            kept = k != INF32;
            if (!kept) B.inlist[bb] = 0;
            if (k != INF32) {
                bool ok = true;
                if (B.tier == 3) {
                    // cells before k are paired alike in f and g, so g's path from the branch's
                    // start passes through cell k: its walk starts there
                    int gt;
                    if (!asc) {
                        int v = cells[k];
                        for (int step = 0; step < dm.n; step++) {
                            const uint8_t cc = B.gpl[pidx<D>(0, v)];
                            if (cc == CODE_CRIT) break;
                            v += c27_lin(dm, cc & 63);
                        }
                        gt = v;
                    } else {
                        const int T0 = cells[k];
                        int a = T0 / g.ntypes[D];
                        int tp = T0 - a * g.ntypes[D] + g.base[D];
                        gt = -1;
                        for (int step = 0; step < dm.n * g.ntypes[D]; step++) {
                            const int id = top_id<D>(a, tp);
                            if (!asc_step<D>(dm, B.gpl, a, tp)) { gt = id; break; }
                            if (a < 0) { gt = -1; break; }
                        }
                    }
                    ok = gt != term[b];
                }
                if (ok) {
                    target = tgt;
                    c[asc ? 1 : 0]++;
                }
            }
        }
        const int idx = wave_append(kept, n_cand_of<WG>(B, sel ^ 1));
        if (kept) keep[idx] = bb;
        request_apply<D, WG>(B, dm, target, it, edit, rc, nullptr, false, mark);
    }
    add_counters<WG, 2>(slot_of<WG>(B, it).cnt + CNT_TM_DESC, c);
    add_counters<WG, 2>(slot_of<WG>(B, it).cnt + CNT_NREQ, rc);
}

// ---- saddle-saddle connectors (3D) --------------------------------------------------------

// Id of the edge between adjacent vertices p and q: (c - 1) * n + anchor, with anchor the lower
// of the two and c the direction bits of the step to the other.
__device__ __forceinline__ int ss_edge_id(const Dims& dm, int p, int q) {
    int px, py, pz, qx, qy, qz;
    coords(dm, p, px, py, pz);
    coords(dm, q, qx, qy, qz);
    if (qx < px || qy < py || qz < pz) {
        const int t = p; p = q; q = t;
        const int dx = px - qx, dy = py - qy, dz = pz - qz;
        return ((dx + 2 * dy + 4 * dz) - 1) * dm.n + p;
    }
    return ((qx - px + 2 * (qy - py) + 4 * (qz - pz)) - 1) * dm.n + p;
}

// Breadth-first walk of f's 1-2 V-paths from the edges of f's 2-saddles, by one workgroup of nt
// threads (tid = thread index): an edge paired alike in f and g and with a triangle in f leads on
// to the triangle's two other edges; an edge paired differently in g is a troublemaker, and
// emit(target) gets the apex of its f-pair (edge ij paired with triangle ijk in f: k; edge ij
// paired with vertex i in f: j); critical edges (1-saddles) and edges paired with a vertex end a
// path.  Each edge is claimed once per walk by raising its stamp to `stamp`; the level queues
// hold edge ids.  Whole waves call emit (target -1: none).  Returns this thread's troublemakers.
template <class Emit>
__device__ __forceinline__ int ss_walk(const uint8_t* fpl, const uint8_t* gpl, const Dims& dm, const int* src,
                                       int n_src, int* q0, int* q1, unsigned* stamps, unsigned stamp, int tid,
                                       int nt, Emit emit) {
    __shared__ int ss_len[2];
    int* q[2] = {q0, q1};
    const int n = dm.n;
    int found = 0;
    if (tid == 0) { ss_len[0] = 0; ss_len[1] = 0; }
    __syncthreads();
    for (int base = 0; base < n_src; base += nt) {
        if (wave_done(base, tid, n_src)) break;
        const int i = base + tid;
        int e = 0;
        bool won = false;
        if (i < n_src) {
            e = src[i];
            won = atomicMax(&stamps[e], stamp) < stamp;
        }
        const int k = wave_append(won, &ss_len[0]);
        if (won) q0[k] = e;
    }
    __syncthreads();
    int cur = 0;
    for (;;) {
        const int ncur = ss_len[cur];
        if (ncur == 0) break;
        if (tid == 0) ss_len[cur ^ 1] = 0;
        __syncthreads();
        for (int base = 0; base < ncur; base += nt) {
            if (wave_done(base, tid, ncur)) break;
            const int i = base + tid;
            int target = -1, p0 = -1, p1 = -1;
            if (i < ncur) {
                const int e = q[cur][i];
                const int c = e / n + 1;            // the edge's direction bits = its code plane
                const int a = e - (c - 1) * n;
                const uint8_t fc = fpl[pidx<3>(c, a)], gc = gpl[pidx<3>(c, a)];
                if (fc != gc) {
                    if (fc != CODE_CRIT) {
                        target = a + c27_lin(dm, fc & 63);
                        found++;
                    }
                } else if (fc & 0x40) {
                    const int x = a + c27_lin(dm, fc & 63);
                    const int w = a + (c & 1) + dm.nx * ((c >> 1) & 1) + dm.nxy * ((c >> 2) & 1);
                    p0 = ss_edge_id(dm, a, x);
                    p1 = ss_edge_id(dm, w, x);
                }
            }
            const bool w0 = p0 >= 0 && atomicMax(&stamps[p0], stamp) < stamp;
            const bool w1 = p1 >= 0 && atomicMax(&stamps[p1], stamp) < stamp;
            const int k0 = wave_append(w0, &ss_len[cur ^ 1]);
            if (w0) q[cur ^ 1][k0] = p0;
            const int k1 = wave_append(w1, &ss_len[cur ^ 1]);
            if (w1) q[cur ^ 1][k1] = p1;
            emit(target);
        }
        __syncthreads();
        cur ^= 1;
    }
    return found;
}

// The saddle-saddle part of the separatrix step of iteration it (called by one whole workgroup
// after phase_sapply): troublemakers are requested and edited at once, like the branches'.
template <bool WG>
__device__ __forceinline__ void phase_ss(const FrontierView& B, const Dims& dm, int it, bool edit, int tid, int nt) {
    int rc[2] = {0, 0};
    const bool mark = WG || ld_relaxed(&B.ctl->nomark) == 0;
    int c = ss_walk(B.fpl, B.gpl, dm, B.ss_src, B.n_ss_src, B.ss_q[0], B.ss_q[1], B.ss_stamp, (unsigned)it + 1u,
                    tid, nt, [&](int target) { request_apply<3, WG>(B, dm, target, it, edit, rc, nullptr, false, mark); });
    add_counters<WG, 1>(slot_of<WG>(B, it).cnt + CNT_TM_SS, &c);
    add_counters<WG, 2>(slot_of<WG>(B, it).cnt + CNT_NREQ, rc);
}

// Edges of f's 2-saddles (critical triangles, ids a * 12 + type): three per triangle into src.
__global__ void __launch_bounds__(256) k_ss_sources(const int* __restrict__ crit2, int n2, Dims dm,
                                                    int* __restrict__ src) {
    constexpr auto& g = G<3>::g;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n2) return;
    const int T = crit2[k];
    const int a = T / g.ntypes[2];
    const int p = g.base[2] + (T - a * g.ntypes[2]);
    int v[3];
    for (int j = 0; j < 3; j++) v[j] = a + g.bvert[p][j][0] + dm.nx * g.bvert[p][j][1] + dm.nxy * g.bvert[p][j][2];
    src[3 * k] = ss_edge_id(dm, v[0], v[1]);
    src[3 * k + 1] = ss_edge_id(dm, v[0], v[2]);
    src[3 * k + 2] = ss_edge_id(dm, v[1], v[2]);
}

// The dense form's saddle-saddle walk: troublemaker targets into req, their count into cnt.
__global__ void __launch_bounds__(1024) k_ss_dense(const uint8_t* __restrict__ fpl, const uint8_t* __restrict__ gpl,
                                                   Dims dm, const int* __restrict__ src, int n_src, int* q0, int* q1,
                                                   unsigned* stamps, unsigned stamp, uint8_t* __restrict__ req,
                                                   unsigned long long* __restrict__ cnt) {
    int c = ss_walk(fpl, gpl, dm, src, n_src, q0, q1, stamps, stamp, threadIdx.x, blockDim.x, [&](int target) {
        if (target >= 0) req[target] = 1;
    });
    block_add_counters<1>(cnt + CNT_TM_SS, &c);
}

// ---- iteration bookkeeping ----------------------------------------------------------------

// End state of iteration it from its counters (all threads agree): 0 go on, 1 converged,
// 2 iteration cap, 3 stalled.  The cap is tested before the stall, as no edit is made at the cap.
__device__ __forceinline__ int iteration_state(const FrontierView& B, int it) {
    const unsigned long long viol = violations(B, it);
    if (viol == 0) return 1;
    if ((long long)it == B.max_iters) return 2;
    if (ld_relaxed(&slot_of(B, it).cnt[CNT_CHANGED]) == 0) return 3;
    return 0;
}

// Log record, step counters and residual of iteration it (one thread).
__device__ __forceinline__ void record_iteration(const FrontierView& B, int it, int state) {
    Ctl* c = B.ctl;
    const Slot& S = slot_of(B, it);
    if (state == 2 || state == 3) c->residual = (long long)violations(B, it);
    if (state != 0) return;
    const bool cstep = c_total(S) != 0;
    if (B.log) {
        long long* rec = B.log + (size_t)it * DMT_LOG_WORDS;
        rec[0] = cstep ? 1 : 2;
        for (int k = 1; k < CNT_NREQ; k++) rec[k] = (long long)ld_relaxed(&S.cnt[k]);
        rec[CNT_NREQ] = (long long)ld_relaxed(&S.cnt[CNT_NREQ]);
        rec[CNT_CHANGED] = (long long)ld_relaxed(&S.cnt[CNT_CHANGED]);
        // a dense iteration's passes took every vertex as dirty and every anchor as affected
        const bool dense = it > 0 && ld_relaxed(&c->dense) != 0;
        rec[13] = it == 0 ? 0 : dense ? B.dm.n : ld_relaxed(&S.n_dv);
        rec[14] = it == 0 ? 0 : dense ? B.dm.n : ld_relaxed(&S.n_da);
        rec[15] = it == 0 || dense ? 0 : ld_relaxed(&S.n_vl);
        rec[16] = ld_relaxed(&S.n_db);
        rec[17] = ld_relaxed(&S.n_scan) + (dense && B.tier >= 3 ? B.n_dcell + B.n_acell : 0);   // dense: every branch cell
        rec[18] = it == 0 ? 0 : ld_relaxed(&S.n_tc);
        rec[19] = 0;
        rec[20] = (long long)ld_relaxed(&S.cnt[CNT_TM_SS]);
    }
    if (cstep) c->c_it++; else c->s_it++;
}

// The first candidate list (list 0): the branches whose first differing cell the dense scan of
// iteration 0 set.  ctl->n_cand[0] must be 0 before the launch.
// The troublemaker candidate list rebuilt from first[] (after a dense scan): the branches whose
// first differing cell is set, with their targets, into list 0 (ctl->n_cand[0] = 0 and
// ctl->cand_sel = 0 before).  Whole blocks of 256 threads call it (gtid, gsize: the grid's
// thread id and size); a thread takes CAND_PER_THREAD consecutive branch ids per round and the
// block reserves its list slots with one atomic (one per wave made the list counter the
// bottleneck on large fields: 45 ms for the branches of a 384^3 field).
constexpr int CAND_PER_THREAD = 8;

template <int D>
__device__ __forceinline__ void cand_rebuild(const FrontierView& B, int gtid, int gsize) {
    const long long nb = (long long)B.n_desc + B.n_asc;
    const long long per_round = (long long)gsize * CAND_PER_THREAD;
    __shared__ int cand_base_sh;
    for (long long base = 0; base < nb; base += per_round) {   // the same rounds for every thread
        const long long i0 = base + (long long)gtid * CAND_PER_THREAD;
        unsigned mask = 0;
        int c = 0;
#pragma unroll
        for (int j = 0; j < CAND_PER_THREAD; j++) {
            const long long i = i0 + j;
            if (i < nb) {
                const bool asc = i >= B.n_desc;
                const int k = asc ? B.afirst[i - B.n_desc] : B.dfirst[i];
                const bool set = k != INF32;
                B.inlist[i] = set;
                if (set) {
                    int t;
                    (void)branch_cell_differs<D>(B, B.dm, asc, k, &t);
                    B.btgt[i] = t;
                    mask |= 1u << j;
                    c++;
                }
            }
        }
        int total;
        int o = block_exclusive_scan(c, total);
        if (threadIdx.x == 0 && total) cand_base_sh = atomicAdd(&B.ctl->n_cand[0], total);
        __syncthreads();
        o += cand_base_sh;
#pragma unroll
        for (int j = 0; j < CAND_PER_THREAD; j++)
            if ((mask >> j) & 1u) B.cand[0][o++] = (int)(i0 + j);
        __syncthreads();   // cand_base_sh is written again in the next round
    }
}

// The first candidate list, after the dense scan of iteration 0.
template <int D>
__global__ void __launch_bounds__(256) k_fr_cand_init(FrontierBufs hb, Ctl* c) {
    cand_rebuild<D>(view(hb), blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

__global__ void k_fr_init(Ctl* c) {
    c->it = 0;
    c->done = 0;
    c->paused = 0;
    c->cand_sel = 0;
    c->n_cand[0] = c->n_cand[1] = 0;
    c->c_it = c->s_it = 0;
    c->residual = 0;
    c->ph[0] = c->ph[1] = c->ph[2] = 0;
    for (int k = 0; k < 8; k++) c->dead_cnt[k] = 0;
    c->dead_distinct = 0;
    c->n_ftgt = 0;
    c->n_dead = 0;
    c->n_v0 = 0;
    c->dense = c->nomark = 0;
    for (int i = 0; i < 3; i++) {
        for (int k = 0; k < CNT_WORDS; k++) c->slot[i].cnt[k] = 0;
        c->slot[i].n_dv = c->slot[i].n_da = c->slot[i].n_vl = c->slot[i].n_db = 0;
        c->slot[i].n_scan = c->slot[i].n_tc = c->slot[i].n_frz = 0;
    }
}

// ---- workgroup-resident form: each job's loop runs inside one workgroup ---------------------

// After a separatrix step: the list its troublemaker pass kept becomes current (one thread).
__device__ __forceinline__ void cand_flip(Ctl* c) {
    const int sel = c->cand_sel;
    c->n_cand[sel] = 0;
    c->cand_sel = sel ^ 1;
}

// iteration_state and record_iteration of the resident loop for a whole wave (wave 0 of the
// workgroup): lane k loads counter k, so the loads are issued together, and returns log word k in
// *rec (the caller stores the record while the next iteration's gradient pass runs).  The step
// counts and the candidate-list selector are the LDS copies (wg_ctl).
__device__ __forceinline__ unsigned long long c_total_wg(const Slot& S) {
    unsigned long long t = 0;
#pragma unroll
    for (int k = CNT_FP0; k < CNT_FP0 + 8; k++) t += S.cnt[k];
    return t;
}

// ct: the iteration's critical-cell violations (c_total_wg of its slot).  Every lane reads the
// counters it needs from LDS itself (the slot is final: the passes that fill it are behind a
// barrier).
// dense: the iteration's passes ran densely on the full grid (the loop's first decision only).
__device__ __forceinline__ int wave_decide(const FrontierView& B, int it, int lane, unsigned long long ct,
                                           long long* rec, bool dense = false) {
    const Slot& S = wg_slots[it % 3];
    const unsigned long long v = lane < CNT_WORDS ? S.cnt[lane] : 0ull;
    const unsigned long long tm_ss = S.cnt[CNT_TM_SS];
    const unsigned long long tt = S.cnt[CNT_TM_DESC] + S.cnt[CNT_TM_ASC] + tm_ss;
    const unsigned long long changed = S.cnt[CNT_CHANGED];
    const unsigned long long viol = ct ? ct : (B.tier >= 3 ? tt : 0ull);
    int st = 0;
    if (viol == 0) st = 1;
    else if ((long long)it == B.max_iters) st = 2;
    else if (changed == 0) st = 3;
    long long r = 0;
    if (lane == 0) r = ct ? 1 : 2;
    else if (lane <= CNT_CHANGED) r = (long long)v;
    else if (lane == 13) r = dense ? B.dm.n : S.n_dv;
    else if (lane == 14) r = dense ? B.dm.n : S.n_da;
    else if (lane == 15) r = dense ? 0 : S.n_vl;
    else if (lane == 16) r = S.n_db;
    else if (lane == 17) r = S.n_scan + (dense && B.tier >= 3 ? B.n_dcell + B.n_acell : 0);
    else if (lane == 18) r = S.n_tc;
    else if (lane == 20) r = (long long)tm_ss;
    *rec = r;
    if (lane == 0) {
        if (st == 2 || st == 3) B.ctl->residual = (long long)viol;
        if (st == 0) {
            if (ct) wg_ctl.c_it++;
            else wg_ctl.s_it++;
        }
        if (ct == 0 && B.tier >= 3) {   // the list the troublemaker pass kept becomes current
            const int sel = wg_ctl.cand_sel;
            wg_ctl.n_cand[sel] = 0;
            wg_ctl.cand_sel = sel ^ 1;
        }
        wg_ctl.it = st ? it : it + 1;
        wg_ctl.done = st;
    }
    return st;
}

// The loop of one job from the end of its iteration ctl->it's violation pass (the
// precondition: that iteration's gradient, violation and branch passes are done), in one
// workgroup, synchronised by workgroup barriers only.  Returns when the job ends, when its log
// is full, after max_passes iterations, or (big > 0) before a large step: ctl->paused = 1 before
// an iteration with more than big affected and listed anchors (ctl->it that iteration, whose
// passes have not started), ctl->paused = 2 before a troublemaker pass over more than big
// candidates (ctl->it the iteration it belongs to); the host runs those as full-grid launches.
// An iteration with critical-cell violations is decided as soon as its passes end; one without
// runs its troublemaker pass first.
template <int D>
__device__ __forceinline__ void run_job_wg(const FrontierView& B, int max_passes, int big) {
    const Dims dm = B.dm;
    Ctl* c = B.ctl;
    const int tid = threadIdx.x, nt = blockDim.x;
    if (ld_relaxed(&c->done)) return;
    int it = ld_relaxed(&c->it);
    // the full-grid violation pass before this launch made no lists: the next iteration is dense
    // and is left to the grid
    const bool nomark_in = ld_relaxed(&c->nomark) != 0;
    // the passes of iteration it (the one decided first) ran densely on the full grid
    const bool dense_in = it > 0 && ld_relaxed(&c->dense) != 0;
    const int it_in = it;
    constexpr int SLOT_WORDS = (int)(3 * sizeof(Slot) / sizeof(int));
    static_assert(sizeof(Slot) % sizeof(int) == 0, "slots copied as ints");
    {
        const int* src = reinterpret_cast<const int*>(c->slot);
        int* dst = reinterpret_cast<int*>(wg_slots);
        for (int k = tid; k < SLOT_WORDS; k += nt) dst[k] = src[k];
        if (tid == 0) {
            wg_n_dead = ld_relaxed(&c->n_dead);
            wg_ctl.it = it;
            wg_ctl.done = 0;
            wg_ctl.c_it = c->c_it;
            wg_ctl.s_it = c->s_it;
            wg_ctl.cand_sel = c->cand_sel;
            wg_ctl.n_cand[0] = c->n_cand[0];
            wg_ctl.n_cand[1] = c->n_cand[1];
        }
    }
    __syncthreads();
    unsigned long long ph[3] = {0, 0, 0};
    unsigned long long t = tid == 0 ? wall_clock64() : 0;
    unsigned long long t_it = tid < 64 ? wall_clock64() : 0;   // start of the current iteration's gradient pass
    auto tick = [&](int k) {
        if (tid == 0) { const unsigned long long t1 = wall_clock64(); ph[k] += t1 - t; t = t1; }
    };
    // decisions are taken by wave 0 and shared through LDS; each variable is written again only
    // after several more workgroup barriers, when every wave has read it
    __shared__ int sstep_sh, state_sh;
    // wave 0 holds the log record of the last decided iteration (lane k: word k) until it is stored
    long long rec = 0;
    int rec_it = -1;
    auto flush = [&]() {
        if (tid < 64 && rec_it >= 0) {
            if (tid < DMT_LOG_WORDS) B.log[(size_t)rec_it * DMT_LOG_WORDS + tid] = rec;
            rec_it = -1;
        }
    };
    // wave 0: decides iteration it (state_sh: 0 go on, 1-3 done, 4 pause before the next one)
    auto decide = [&](unsigned long long ct) {
        const int st = wave_decide(B, it, tid, ct, &rec, dense_in && it == it_in);
        if (tid == 19) rec = (long long)(wall_clock64() - t_it);
        int act = st;
        // a large next iteration is left to full-grid launches: pause before its gradient pass
        if (st == 0 && big > 0) {
            const Slot& N = wg_slots[(it + 1) % 3];
            if (N.n_da + N.n_vl > big || nomark_in) {
                if (tid == 0) c->paused = 1;
                act = 4;
            }
        }
        if (st == 0 && B.log) rec_it = it;
        if (tid == 0) state_sh = act;
    };
    for (int pass = 0; pass < max_passes; pass++) {
        if (B.log && it >= B.log_cap) break;
        if (tid < 64) {
            const unsigned long long ct = c_total_wg(wg_slots[it % 3]);
            const bool s_step = B.tier >= 3 && ct == 0;
            int act = 0;
            if (!s_step) {
                decide(ct);
            } else if (big > 0 && wg_ctl.n_cand[wg_ctl.cand_sel] > big) {
                // a troublemaker pass over more than `big` candidates is left to the grid too
                if (tid == 0) c->paused = 2;
                act = 2;
            } else {
                act = 1;
            }
            if (tid == 0) sstep_sh = act;
        }
        __syncthreads();
        const int ss = sstep_sh;
        if (ss == 2) break;
        if (ss) {
            phase_sapply<D, true>(B, dm, it, (long long)it != B.max_iters, tid, nt);
            __syncthreads();
            if constexpr (D == 3) {
                if (B.ss_on && B.tier == 4) {
                    phase_ss<true>(B, dm, it, (long long)it != B.max_iters, tid, nt);
                    __syncthreads();
                }
            }
            if (tid < 64) decide(0ull);
            __syncthreads();
        }
        const int st = state_sh;
        tick(0);
        if (st) break;
        it++;
        if (tid < 64) t_it = wall_clock64();
        flush();
        phase_grad<D, true>(B, dm, it, tid, nt);
        __syncthreads();
        tick(1);
        phase_vr<D, true>(B, dm, it, (long long)it != B.max_iters, tid, nt);
        __syncthreads();
        if constexpr (D == 3) freeze_pass<D, true>(B, dm, it, tid, nt);
        if (B.tier >= 3) phase_bscan<D, true>(B, dm, it, tid, nt);
        if (D == 3 || B.tier >= 3) __syncthreads();
        tick(2);
    }
    flush();
    __syncthreads();
    {
        const int* src = reinterpret_cast<const int*>(wg_slots);
        int* dst = reinterpret_cast<int*>(c->slot);
        for (int k = tid; k < SLOT_WORDS; k += nt) dst[k] = src[k];
        if (tid == 0) {
            c->n_dead = wg_n_dead;
            c->it = wg_ctl.it;
            c->done = wg_ctl.done;
            c->c_it = wg_ctl.c_it;
            c->s_it = wg_ctl.s_it;
            c->cand_sel = wg_ctl.cand_sel;
            c->n_cand[0] = wg_ctl.n_cand[0];
            c->n_cand[1] = wg_ctl.n_cand[1];
            for (int k = 0; k < 3; k++) c->ph[k] += ph[k];
        }
    }
    __syncthreads();
}

// Workgroups of NT threads take jobs (all of dimension D) from a queue (an atomic counter
// starting at 0) until none is left.  NT is a tuning choice (512 or 1024 threads in 2D, 256 or
// 512 in 3D): fewer threads give each lane more registers (the 3D passes need about twice those
// of the 2D ones), more threads cover larger frontiers per step; results do not depend on it.
template <int D, int NT>
__global__ void __launch_bounds__(NT) k_fr_loop_wg(const FrontierBufs* __restrict__ jobs, int n_jobs, int* queue,
                                                   int max_passes, int big) {
    __shared__ int job_sh;
    for (;;) {
        if (threadIdx.x == 0) job_sh = atomicAdd(queue, 1);
        __syncthreads();
        const int j = __builtin_amdgcn_readfirstlane(job_sh);   // uniform: job fields load as scalars
        __syncthreads();
        if (j >= n_jobs) return;
        run_job_wg<D>(view(jobs[j]), max_passes, big);
    }
}

// Vertex -> branch cells of f: one entry per (vertex, cell) of every branch cell (descending
// cells are vertices; an ascending top cell contributes each of its D + 1 vertices).  Pass 0
// counts entries per vertex into pos; pass 1 (pos = exclusive offsets) fills ecell.  The order
// of entries within a vertex depends on scheduling; their use (marking branches) does not.
template <int D>
__global__ void __launch_bounds__(256) k_fr_branch_map(FrontierBufs hb, int pass, int* __restrict__ pos,
                                                       int* __restrict__ ecell) {
    const FrontierView& B = view(hb);
    constexpr auto& g = G<D>::g;
    const Dims dm = B.dm;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long ne = B.n_dcell + (long long)(D + 1) * B.n_acell;
    if (e >= ne) return;
    int v, kk;
    if (e < B.n_dcell) {
        v = B.dcell[e];
        kk = (int)e;
    } else {
        const long long k = (e - B.n_dcell) / (D + 1);
        const int j = (int)(e - B.n_dcell - k * (D + 1));
        const int T = B.acell[k];
        const int a = T / g.ntypes[D];
        const int tp = T - a * g.ntypes[D] + g.base[D];
        v = a;
        static_for<g.base[D], g.base[D] + g.ntypes[D]>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            if (q != tp) return;
            static_for<0, D + 1>([&](auto rc) {
                constexpr int r = decltype(rc)::value;
                constexpr auto& gg = G<D>::g;
                if (r == j) v = a + gg.bvert[q][r][0] + dm.nx * gg.bvert[q][r][1] + dm.nxy * gg.bvert[q][r][2];
            });
        });
        kk = (int)(B.n_dcell + k);
    }
    if (pass == 0) atomicAdd(&pos[v], 1);
    else ecell[atomicAdd(&pos[v], 1)] = kk;
}

// ---- launch-per-phase form: one full-grid launch per phase --------------------------------

__device__ __forceinline__ bool running(const Ctl* c) { return ld_relaxed(&c->done) == 0; }

template <int D>
__global__ void __launch_bounds__(256) k_fr_grad(FrontierBufs hb, Dims dm) {
    const FrontierView& B = view(hb);
    if (!running(B.ctl)) return;
    phase_grad<D>(B, dm, ld_relaxed(&B.ctl->it), blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

// The critical-cell classification as a streaming pass (a4): every anchor's violation mask from
// its f and g codes in every plane (each plane a byte array, read once, coalesced) and the list of
// violating anchors, compacted by wave ballot and a block-wide prefix sum with one atomic per
// chunk (count in ctl->n_v0, 0 before).  A block takes chunks of CLASSIFY_APB consecutive anchors
// (chunk c0, c0 + cstep, ...); thread t takes those at t + k * 256 of a chunk (coalesced).  The
// violation pass then requests targets for the listed anchors only.
constexpr int CLASSIFY_APB = 1024;   // anchors per chunk
template <int D>
__device__ __forceinline__ void classify_chunks(const FrontierView& B, const Dims& dm, int* list, int c0, int cstep) {
    const int nchunks = (int)((dm.n + CLASSIFY_APB - 1) / CLASSIFY_APB);
    __shared__ int base_sh;
    for (int ch = c0; ch < nchunks; ch += cstep) {
        const int a0 = ch * CLASSIFY_APB;
        uint32_t m[CLASSIFY_APB / 256];
        int c = 0;
#pragma unroll
        for (int k = 0; k < CLASSIFY_APB / 256; k++) {
            const int a = a0 + k * 256 + (int)threadIdx.x;
            m[k] = 0;
            if (a < dm.n) {
                int x, y, z;
                coords(dm, a, x, y, z);
                m[k] = vmask_anchor<D>(dm, a, x, y, z, B.fpl, B.gpl, B.tier);
                B.vmask[a] = m[k];
            }
            c += m[k] != 0;
        }
        int total;
        int off = block_exclusive_scan(c, total);
        if (threadIdx.x == 0 && total) base_sh = atomicAdd(&B.ctl->n_v0, total);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < CLASSIFY_APB / 256; k++)
            if (m[k] != 0) list[base_sh + off++] = a0 + k * 256 + (int)threadIdx.x;
        __syncthreads();   // base_sh is written again for the next chunk
    }
}

// Iteration 0's classification: one chunk per block, the list in vl[0].
template <int D>
__global__ void __launch_bounds__(256) k_fr_classify0(FrontierBufs hb, Dims dm) {
    const FrontierView& B = view(hb);
    classify_chunks<D>(B, dm, B.vl[0], blockIdx.x, gridDim.x);
}

// The classification of a dense iteration after the first (full-grid form, see phase_grad), as
// at iteration 0: the list goes to vl[it & 1], which a dense iteration's violation pass does not
// otherwise read (it has no anchors listed by the previous iteration).  The violation pass keeps
// its heavy per-anchor code, with few waves per SIMD, for the violating anchors alone.  Then the
// first differing cell of every branch (first[] reset by the gradient pass).  Returns at once
// when the iteration is not dense; launched on a capped grid, so that costs little.
template <int D>
__global__ void __launch_bounds__(256) k_fr_classify_dense(FrontierBufs hb, Dims dm) {
    const FrontierView& B = view(hb);
    if (!running(B.ctl) || ld_relaxed(&B.ctl->dense) == 0) return;
    const int it = ld_relaxed(&B.ctl->it);
    classify_chunks<D>(B, dm, B.vl[it & 1], blockIdx.x, gridDim.x);
    if (B.tier >= 3) {
        const int gtid = blockIdx.x * blockDim.x + threadIdx.x, gsize = gridDim.x * blockDim.x;
        dense_first_scan<D>(B, dm, false, gtid, gsize);
        dense_first_scan<D>(B, dm, true, gtid, gsize);
    }
}

template <int D>
__global__ void __launch_bounds__(256) k_fr_vr(FrontierBufs hb, Dims dm) {
    const FrontierView& B = view(hb);
    if (!running(B.ctl)) return;
    const int it = ld_relaxed(&B.ctl->it);
    phase_vr<D>(B, dm, it, (long long)it != B.max_iters, blockIdx.x * blockDim.x + threadIdx.x,
                gridDim.x * blockDim.x);
}

template <int D>
__global__ void __launch_bounds__(256) k_fr_bscan(FrontierBufs hb, Dims dm) {
    const FrontierView& B = view(hb);
    if (!running(B.ctl)) return;
    const int it = ld_relaxed(&B.ctl->it);
    const int gtid = blockIdx.x * blockDim.x + threadIdx.x, gsize = gridDim.x * blockDim.x;
    freeze_pass<D>(B, dm, it, gtid, gsize);
    phase_bscan<D>(B, dm, it, gtid, gsize);
}

template <int D>
__global__ void __launch_bounds__(256) k_fr_sapply(FrontierBufs hb, Dims dm) {
    const FrontierView& B = view(hb);
    const int it = ld_relaxed(&B.ctl->it);
    if (!running(B.ctl) || B.tier < 3 || c_total(slot_of(B, it)) != 0) return;
    phase_sapply<D>(B, dm, it, (long long)it != B.max_iters, blockIdx.x * blockDim.x + threadIdx.x,
                    gridDim.x * blockDim.x);
}

// The saddle-saddle walk of a job's separatrix step as one workgroup (phase and hand-off forms).
__global__ void __launch_bounds__(1024) k_fr_ss(FrontierBufs hb, Dims dm) {
    const FrontierView& B = view(hb);
    const int it = ld_relaxed(&B.ctl->it);
    if (!running(B.ctl) || B.tier < 4 || !B.ss_on || c_total(slot_of(B, it)) != 0) return;
    phase_ss<false>(B, dm, it, (long long)it != B.max_iters, threadIdx.x, blockDim.x);
}

__global__ void k_fr_finish(FrontierBufs hb) {
    const FrontierView& B = view(hb);
    Ctl* c = B.ctl;
    if (c->done) return;
    const int it = c->it;
    const int state = iteration_state(B, it);
    record_iteration(B, it, state);
    if (B.tier >= 3 && c_total(slot_of(B, it)) == 0) cand_flip(c);
    if (state) { c->done = state; return; }
    c->it = it + 1;
}

}  // namespace dmt
