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
#include "dmt_kernels.h"

namespace dmt {

// Per-iteration counters live in slot it % 3: iteration it fills its own slot and the list
// lengths of slot (it+1) % 3; slot (it+1) % 3 is cleared when iteration it begins (its last
// readers belong to iteration it-2).  List buffers alternate by iteration parity.
struct Slot {
    unsigned long long cnt[CNT_WORDS];  // log record layout
    int n_req;              // distinct vertices requested in this iteration
    int n_dv, n_da, n_vl;   // dirty vertices, affected anchors, violation list of this iteration
};

struct Ctl {
    int it;                 // current iteration
    int done;               // 0 running, 1 converged, 2 iteration cap, 3 stalled, 4 paused (log full)
    int c_it, s_it;
    long long residual;
    Slot slot[3];
};

struct FrontierBufs {
    Ctl* ctl;
    const float *f, *gh, *lo;
    float* gb[2];           // g^(k) in gb[k & 1]
    uint8_t* state;
    const uint8_t* fpl;
    uint8_t* gpl;
    uint32_t* vmask;        // violating planes per anchor
    int* vl[2];             // violation anchor lists
    int* dvl[2];            // dirty vertex lists
    int* dal[2];            // affected anchor lists
    unsigned* vstamp;       // dirty-vertex stamps
    unsigned* astamp[2];    // affected-anchor stamps by iteration parity (iteration k's in [k & 1]: the
                            // edits of iteration k mark [(k+1) & 1] while [k & 1] is still read)
    unsigned* rstamp;       // request stamps
    long long* log;         // DMT_LOG_WORDS per iteration
    // separatrix branches of f
    const int *dcell, *dcbr, *dterm, *acell, *acbr, *aterm;
    const int64_t *doff, *aoff;
    int* dfirst;
    int* afirst;
    long long n_dcell, n_acell;
    int n_desc, n_asc;
    float delta;
    int q_max, tier;
    long long max_iters;
};

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

__device__ __forceinline__ Slot& slot_of(const FrontierBufs& B, int it) { return B.ctl->slot[it % 3]; }

__device__ __forceinline__ unsigned long long c_total(const Slot& s) {
    unsigned long long t = 0;
#pragma unroll
    for (int k = CNT_FP0; k < CNT_FP0 + 8; k++) t += ld_relaxed(&s.cnt[k]);
    return t;
}

// Violations of iteration it: critical-cell violations, else (tier >= 3) troublemakers.
__device__ __forceinline__ unsigned long long violations(const FrontierBufs& B, int it) {
    const Slot& s = slot_of(B, it);
    const unsigned long long ct = c_total(s);
    if (ct) return ct;
    return B.tier >= 3 ? ld_relaxed(&s.cnt[CNT_TM_DESC]) + ld_relaxed(&s.cnt[CNT_TM_ASC]) : 0ull;
}

// ---- Equation 2 on one vertex, and the neighbourhood an edit makes dirty -------------------

__device__ __forceinline__ bool apply_vertex(const FrontierBufs& B, int v, int it) {
    const uint8_t st = B.state[v];
    if (st & 0x80) return false;
    const int q = st & 7;
    const float t = fmaf(-(float)(q + 1), B.delta, B.gh[v]);
    const float l = B.lo[v];
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
// affected, for iteration it + 1.  Lanes without an edit pass changed = false.
template <int D>
__device__ __noinline__ void mark_neighbourhood(const FrontierBufs& B, const Dims& dm, bool changed, int v,
                                                   int it) {
    constexpr auto& g = G<D>::g;
    if (__ballot(changed) == 0) return;
    const int nxt = (it + 1) & 1;
    Slot& N1 = slot_of(B, it + 1);
    const unsigned stamp = (unsigned)it + 1u;
    int x = 0, y = 0, z = 0;
    if (changed) coords(dm, v, x, y, z);
#pragma unroll
    for (int s = -1; s < Geom<D>::NS; s++) {
        const int dx = s < 0 ? 0 : g.slot_d[s < 0 ? 0 : s][0];
        const int dy = s < 0 ? 0 : g.slot_d[s < 0 ? 0 : s][1];
        const int dz = s < 0 ? 0 : g.slot_d[s < 0 ? 0 : s][2];
        bool mine = false;
        int t = 0;
        if (changed && (unsigned)(x + dx) < (unsigned)dm.nx && (unsigned)(y + dy) < (unsigned)dm.ny &&
            (unsigned)(z + dz) < (unsigned)dm.nz) {
            t = v + dx + dm.nx * dy + dm.nxy * dz;
            mine = atomicMax(&B.vstamp[t], stamp) < stamp;
        }
        const int idx = wave_append(mine, &N1.n_dv);
        if (mine) B.dvl[nxt][idx] = t;
    }
#pragma unroll
    for (int j = 0; j < g.naff; j++) {
        const int dx = g.aff_d[j][0], dy = g.aff_d[j][1], dz = g.aff_d[j][2];
        bool mine = false;
        int a = 0;
        if (changed && x + dx >= 0 && y + dy >= 0 && z + dz >= 0 && x + dx < dm.nx && y + dy < dm.ny &&
            z + dz < dm.nz) {
            a = v + dx + dm.nx * dy + dm.nxy * dz;
            mine = atomicMax(&B.astamp[nxt][a], stamp) < stamp;
        }
        const int idx = wave_append(mine, &N1.n_da);
        if (mine) B.dal[nxt][idx] = a;
    }
}

// Request of vertex v (v < 0: none) in iteration it: the first requester counts it and, when
// edits are allowed, edits it and marks its neighbourhood.
template <int D>
__device__ __noinline__ void request_apply(const FrontierBufs& B, const Dims& dm, int v, int it, bool edit,
                                              int* changed_cnt) {
    const unsigned stamp = (unsigned)it + 1u;
    const bool mine = v >= 0 && atomicMax(&B.rstamp[v], stamp) < stamp;
    wave_append(mine, &slot_of(B, it).n_req);
    bool changed = false;
    if (mine && edit) changed = apply_vertex(B, v, it);
    if (changed) (*changed_cnt)++;
    mark_neighbourhood<D>(B, dm, changed, v, it);
}

// ---- violation mask of one anchor: planes whose criticality differs between f and g --------

template <int D, int P>
__device__ __forceinline__ void vmask_plane(const Dims& dm, int a, int x, int y, int z, const uint8_t* fpl,
                                            const uint8_t* gpl, int tier, uint32_t& m) {
    constexpr auto& g = G<D>::g;
    constexpr int dim = g.bdim[P];
    if (!(tier == 1 && dim != 0 && dim != D) && cell_exists<D, P>(dm, x, y, z)) {
        const bool fc = fpl[(size_t)P * dm.n + a] == CODE_CRIT;
        const bool gc = gpl[(size_t)P * dm.n + a] == CODE_CRIT;
        if (fc != gc) m |= 1u << P;
    }
    if constexpr (P + 1 < Geom<D>::NB) vmask_plane<D, P + 1>(dm, a, x, y, z, fpl, gpl, tier, m);
}

// ---- target of one violating plane (Rules A and B, as classify_plane) ---------------------

template <int D, int P>
__device__ __forceinline__ int plane_target(const FrontierBufs& B, const Dims& dm, int a, const float* gcur, int* cnt) {
    constexpr auto& g = G<D>::g;
    constexpr int dim = g.bdim[P];
    const uint8_t fc = B.fpl[(size_t)P * dm.n + a];
    const uint8_t gc = B.gpl[(size_t)P * dm.n + a];
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
#pragma unroll
    for (int k = 0; k < g.bnv[P]; k++) {
        const int ck = c27_of(g.bvert[P][k][0], g.bvert[P][k][1], g.bvert[P][k][2]);
        if (!up && ck == gx) { kx = k; continue; }
        const int w = a + g.bvert[P][k][0] + dm.nx * g.bvert[P][k][1] + dm.nxy * g.bvert[P][k][2];
        if (!prec(B.f[w], w, fx, xv)) continue;
        const float gw = gcur[w];
        if (best < 0 || prec(gw, w, gbest, best)) { best = w; gbest = gw; }
    }
    if (best < 0) {
        int fa = a, fp = 0;
#pragma unroll
        for (int k = 0; k < g.bnv[P]; k++) {
            if (k == kx) {
                fa = a + g.facet_anchor[P][k][0] + dm.nx * g.facet_anchor[P][k][1] + dm.nxy * g.facet_anchor[P][k][2];
                fp = g.facet_plane[P][k];
            }
        }
        best = fa + c27_lin(dm, B.fpl[(size_t)fp * dm.n + fa] & 63);
    }
    cnt[2 * dim + 1]++;
    return best;
}

// plane p chosen at run time
template <int D, int P>
__device__ __forceinline__ int plane_target_dyn(int p, const FrontierBufs& B, const Dims& dm, int a, const float* gcur,
                                                int* cnt) {
    if (p == P) return plane_target<D, P>(B, dm, a, gcur, cnt);
    if constexpr (P + 1 < Geom<D>::NB) return plane_target_dyn<D, P + 1>(p, B, dm, a, gcur, cnt);
    return -1;
}

// Requests (and, with edit, edits) the targets of the violating planes m of anchor a.  Whole
// waves call it; lanes without an anchor pass m = 0.  One plane per lane per round.
template <int D>
__device__ __forceinline__ void anchor_requests(const FrontierBufs& B, const Dims& dm, int a, uint32_t m, int it,
                                                bool edit, int* cnt, int* changed_cnt) {
    const float* gcur = B.gb[it & 1];
    for (;;) {
        if (__ballot(m != 0) == 0) break;
        int target = -1;
        if (m != 0) {
            const int p = __ffs(m) - 1;
            m &= m - 1u;
            target = plane_target_dyn<D, 0>(p, B, dm, a, gcur, cnt);
        }
        request_apply<D>(B, dm, target, it, edit, changed_cnt);
    }
}

// ---- phases ------------------------------------------------------------------------------

// Gradient of g^(it) for the dirty vertices (every vertex at iteration 0); brings the write
// buffer up to date on them; clears the branch scan results and the next slot.
template <int D>
__device__ __forceinline__ void phase_grad(const FrontierBufs& B, const Dims& dm, int it, int gtid, int gsize) {
    if (gtid == 0) {
        Slot& s = slot_of(B, it + 1);
        for (int k = 0; k < CNT_WORDS; k++) s.cnt[k] = 0;
        s.n_req = s.n_dv = s.n_da = s.n_vl = 0;
    }
    for (int b = gtid; b < B.n_desc; b += gsize) B.dfirst[b] = INF32;
    for (int b = gtid; b < B.n_asc; b += gsize) B.afirst[b] = INF32;
    const float* gcur = B.gb[it & 1];
    float* gnext = B.gb[(it + 1) & 1];
    if (it == 0) {
        for (int i = gtid; i < dm.n; i += gsize) grad_vertex<D>(i, gcur, B.gpl, dm);
        return;
    }
    const int n = ld_relaxed(&slot_of(B, it).n_dv);
    const int* list = B.dvl[it & 1];
    for (int i = gtid; i < n; i += gsize) {
        const int t = list[i];
        grad_vertex<D>(t, gcur, B.gpl, dm);
        gnext[t] = gcur[t];
    }
}

// Violation masks of the affected anchors (every anchor at iteration 0), the targets of every
// violating anchor (edited at once when edit is set), the violation list of the next iteration,
// and the speculative first-difference scan along f's branches.
template <int D>
__device__ __forceinline__ void phase_vr(const FrontierBufs& B, const Dims& dm, int it, bool edit, int gtid,
                                         int gsize) {
    Slot& S = slot_of(B, it);
    int* n_next = &slot_of(B, it + 1).n_vl;
    int* next = B.vl[(it + 1) & 1];
    int cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int changed = 0;
    // affected anchors: new masks
    const int na = it == 0 ? dm.n : ld_relaxed(&S.n_da);
    const int* alist = B.dal[it & 1];
    for (int i0 = gtid; i0 - (int)threadIdx.x < na; i0 += gsize) {
        uint32_t m = 0;
        int a = 0;
        if (i0 < na) {
            a = it == 0 ? i0 : alist[i0];
            int x, y, z;
            coords(dm, a, x, y, z);
            vmask_plane<D, 0>(dm, a, x, y, z, B.fpl, B.gpl, B.tier, m);
            B.vmask[a] = m;
        }
        const int idx = wave_append(m != 0, n_next);
        if (m != 0) next[idx] = a;
        anchor_requests<D>(B, dm, a, m, it, edit, cnt, &changed);
    }
    // anchors listed from the previous iteration and not affected since: unchanged masks
    const int nl = ld_relaxed(&S.n_vl);
    const int* vlist = B.vl[it & 1];
    const unsigned astamp_it = (unsigned)it;
    const unsigned* astamp = B.astamp[it & 1];
    for (int i0 = gtid; i0 - (int)threadIdx.x < nl; i0 += gsize) {
        uint32_t m = 0;
        int a = 0;
        if (i0 < nl) {
            a = vlist[i0];
            if (astamp[a] != astamp_it) m = B.vmask[a];
        }
        const int idx = wave_append(m != 0, n_next);
        if (m != 0) next[idx] = a;
        anchor_requests<D>(B, dm, a, m, it, edit, cnt, &changed);
    }
    // speculative separatrix scan: first cell of each f-branch whose g pairing differs
    if (B.tier >= 3) {
        constexpr auto& g = G<D>::g;
        for (long long k = gtid; k < B.n_dcell; k += gsize) {
            const int v = B.dcell[k];
            if (B.fpl[v] != B.gpl[v]) atomicMin(&B.dfirst[B.dcbr[k]], (int)k);
        }
        for (long long k = gtid; k < B.n_acell; k += gsize) {
            const int T = B.acell[k];
            const int a = T / g.ntypes[D];
            const int tp = T - a * g.ntypes[D] + g.base[D];
            const size_t o = (size_t)tp * dm.n + a;
            if (B.fpl[o] != B.gpl[o]) atomicMin(&B.afirst[B.acbr[k]], (int)k);
        }
    }
    block_add_counters<8>(S.cnt + CNT_FP0, cnt);
    block_add_counters<1>(S.cnt + CNT_CHANGED, &changed);
}

// Troublemaker targets (apex of the f-pair of each branch's first differing cell), edited at
// once.  Only called when iteration it has no critical-cell violation.
template <int D>
__device__ __forceinline__ void phase_sapply(const FrontierBufs& B, const Dims& dm, int it, bool edit, int gtid,
                                             int gsize) {
    constexpr auto& g = G<D>::g;
    int c[2] = {0, 0};
    int changed = 0;
    const int nb = B.n_desc + B.n_asc;
    for (int i0 = gtid; i0 - (int)threadIdx.x < nb; i0 += gsize) {
        int target = -1;
        if (i0 < nb) {
            const bool asc = i0 >= B.n_desc;
            const int b = asc ? i0 - B.n_desc : i0;
            const int* first = asc ? B.afirst : B.dfirst;
            const int* cells = asc ? B.acell : B.dcell;
            const int64_t* off = asc ? B.aoff : B.doff;
            const int* term = asc ? B.aterm : B.dterm;
            const int k = first[b];
            if (k != INF32) {
                bool ok = true;
                if (B.tier == 3) {
                    int gt;
                    if (!asc) {
                        int v = cells[off[b]];
                        for (int step = 0; step < dm.n; step++) {
                            const uint8_t cc = B.gpl[v];
                            if (cc == CODE_CRIT) break;
                            v += c27_lin(dm, cc & 63);
                        }
                        gt = v;
                    } else {
                        const int T0 = cells[off[b]];
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
                    if (!asc) {
                        const int v = cells[k];
                        target = v + c27_lin(dm, B.fpl[v] & 63);
                    } else {
                        const int T = cells[k];
                        const int a = T / g.ntypes[D];
                        const int tp = T - a * g.ntypes[D] + g.base[D];
                        target = a + c27_lin(dm, B.fpl[(size_t)tp * dm.n + a] & 63);
                    }
                    c[asc ? 1 : 0]++;
                }
            }
        }
        request_apply<D>(B, dm, target, it, edit, &changed);
    }
    block_add_counters<2>(slot_of(B, it).cnt + CNT_TM_DESC, c);
    block_add_counters<1>(slot_of(B, it).cnt + CNT_CHANGED, &changed);
}

// ---- iteration bookkeeping ----------------------------------------------------------------

// End state of iteration it from its counters (all threads agree): 0 go on, 1 converged,
// 2 iteration cap, 3 stalled.  The cap is tested before the stall, as no edit is made at the cap.
__device__ __forceinline__ int iteration_state(const FrontierBufs& B, int it) {
    const unsigned long long viol = violations(B, it);
    if (viol == 0) return 1;
    if ((long long)it == B.max_iters) return 2;
    if (ld_relaxed(&slot_of(B, it).cnt[CNT_CHANGED]) == 0) return 3;
    return 0;
}

// Log record, step counters and residual of iteration it (one thread).
__device__ __forceinline__ void record_iteration(const FrontierBufs& B, int it, int state) {
    Ctl* c = B.ctl;
    const Slot& S = slot_of(B, it);
    if (state == 2 || state == 3) c->residual = (long long)violations(B, it);
    if (state != 0) return;
    const bool cstep = c_total(S) != 0;
    if (B.log) {
        long long* rec = B.log + (size_t)it * DMT_LOG_WORDS;
        rec[0] = cstep ? 1 : 2;
        for (int k = 1; k < CNT_NREQ; k++) rec[k] = (long long)ld_relaxed(&S.cnt[k]);
        rec[CNT_NREQ] = ld_relaxed(&S.n_req);
        rec[CNT_CHANGED] = (long long)ld_relaxed(&S.cnt[CNT_CHANGED]);
        for (int k = CNT_CHANGED + 1; k < DMT_LOG_WORDS; k++) rec[k] = 0;
    }
    if (cstep) c->c_it++; else c->s_it++;
}

__global__ void k_fr_init(Ctl* c) {
    c->it = 0;
    c->done = 0;
    c->c_it = c->s_it = 0;
    c->residual = 0;
    for (int i = 0; i < 3; i++) {
        for (int k = 0; k < CNT_WORDS; k++) c->slot[i].cnt[k] = 0;
        c->slot[i].n_req = c->slot[i].n_dv = c->slot[i].n_da = c->slot[i].n_vl = 0;
    }
}

// ---- persistent form: the loops of a batch of jobs in one cooperative launch ----------------

// Loop state of one job in the persistent kernel, indexed by pass parity: pass p reads [p & 1]
// (written by the previous pass's decision, several barriers earlier) and the decision of pass
// p writes [(p + 1) & 1], so the single writer never races with readers.
struct JobRun {
    int itp[2];             // iteration the job is at
    int donep[2];           // end state (0 = running)
    int log_cap;            // records the job's log can hold (ignored when it has no log)
    int ndim;               // 2 or 3
};

struct BatchCtl {
    unsigned bar_count, bar_gen;  // grid barrier
    int err;                      // 1: a grid barrier timed out
    int parity;                   // pass parity to resume from
    unsigned long long ph[4];     // wall-clock ticks (100 MHz) per phase, seen from block 0
};

__device__ __forceinline__ bool batch_barrier(BatchCtl* c, unsigned nblocks, unsigned& gen,
                                              unsigned long long timeout) {
    __shared__ int ok_sh;
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        const unsigned arrived = __hip_atomic_fetch_add(&c->bar_count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == nblocks - 1) {
            __hip_atomic_store(&c->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&c->bar_gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const unsigned long long t0 = wall_clock64();
            while (__hip_atomic_load(&c->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(2);
                if (wall_clock64() - t0 > timeout) { ok = 0; break; }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (!ok || __hip_atomic_load(&c->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            ok = 0;
            __hip_atomic_store(&c->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        ok_sh = ok;
    }
    __syncthreads();
    gen++;
    return ok_sh != 0;
}

// The frontier loops of n_jobs fields (2D and 3D mixed), advanced in lockstep: one pass runs
// one iteration of every unfinished job, so each grid barrier is shared by all of them.
// Precondition: the gradient and violation passes of each job's current iteration are done
// (iteration 0's run as full-grid launches before the first launch of this kernel).
// Per pass: troublemaker passes [barrier], decisions, gradient passes, barrier, violation
// passes, barrier.  Pauses (and can be launched again) when a job's log is full or after
// max_passes passes, so every launch ends.
__global__ void __launch_bounds__(256) k_fr_loop_batch(const FrontierBufs* __restrict__ jobs,
                                                       const Dims* __restrict__ dims, JobRun* __restrict__ run,
                                                       int n_jobs, BatchCtl* bc, unsigned long long timeout,
                                                       int max_passes) {
    const unsigned nblocks = gridDim.x;
    const int gtid = blockIdx.x * blockDim.x + threadIdx.x;
    const int gsize = gridDim.x * blockDim.x;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    unsigned gen = __hip_atomic_load(&bc->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int p = __hip_atomic_load(&bc->parity, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!batch_barrier(bc, nblocks, gen, timeout)) return;   // every block starts from one generation
    unsigned long long ph[3] = {0, 0, 0};
    unsigned long long t = lead ? wall_clock64() : 0;
    auto tick = [&](int k) {
        if (lead) { const unsigned long long t1 = wall_clock64(); ph[k] += t1 - t; t = t1; }
    };
    for (int pass = 0; pass < max_passes; pass++) {
        const int q = p & 1;
        bool any = false, pause = false;
        for (int j = 0; j < n_jobs; j++) {
            if (ld_relaxed(&run[j].donep[q])) continue;
            any = true;
            if (jobs[j].log && ld_relaxed(&run[j].itp[q]) >= run[j].log_cap) pause = true;
        }
        if (!any || pause) break;
        // troublemaker passes of the jobs without critical-cell violations
        bool any_s = false;
        for (int j = 0; j < n_jobs; j++) {
            if (ld_relaxed(&run[j].donep[q])) continue;
            const FrontierBufs& B = jobs[j];
            const int it = ld_relaxed(&run[j].itp[q]);
            if (B.tier < 3 || c_total(slot_of(B, it)) != 0) continue;
            any_s = true;
            const bool edit = (long long)it != B.max_iters;
            if (run[j].ndim == 2) phase_sapply<2>(B, dims[j], it, edit, gtid, gsize);
            else phase_sapply<3>(B, dims[j], it, edit, gtid, gsize);
        }
        if (any_s) {
            if (!batch_barrier(bc, nblocks, gen, timeout)) return;
            tick(0);
        }
        // decisions (every thread reaches the same ones) and the next iteration's gradient pass;
        // a finished job's state is carried to the other parity too, or the next pass would
        // read the stale entry and take the job up again
        for (int j = 0; j < n_jobs; j++) {
            const int dq = ld_relaxed(&run[j].donep[q]);
            if (dq) {
                if (lead) {
                    run[j].itp[q ^ 1] = ld_relaxed(&run[j].itp[q]);
                    run[j].donep[q ^ 1] = dq;
                }
                continue;
            }
            const FrontierBufs& B = jobs[j];
            const int it = ld_relaxed(&run[j].itp[q]);
            const int st = iteration_state(B, it);
            if (lead) {
                record_iteration(B, it, st);
                run[j].itp[q ^ 1] = st ? it : it + 1;
                run[j].donep[q ^ 1] = st;
                B.ctl->it = st ? it : it + 1;
                B.ctl->done = st;
            }
            if (st) continue;
            if (run[j].ndim == 2) phase_grad<2>(B, dims[j], it + 1, gtid, gsize);
            else phase_grad<3>(B, dims[j], it + 1, gtid, gsize);
        }
        if (!batch_barrier(bc, nblocks, gen, timeout)) return;
        tick(1);
        for (int j = 0; j < n_jobs; j++) {
            if (ld_relaxed(&run[j].donep[q])) continue;
            const FrontierBufs& B = jobs[j];
            const int it = ld_relaxed(&run[j].itp[q]);
            if (iteration_state(B, it)) continue;
            const bool edit = (long long)(it + 1) != B.max_iters;
            if (run[j].ndim == 2) phase_vr<2>(B, dims[j], it + 1, edit, gtid, gsize);
            else phase_vr<3>(B, dims[j], it + 1, edit, gtid, gsize);
        }
        if (!batch_barrier(bc, nblocks, gen, timeout)) return;
        tick(2);
        p++;
    }
    if (lead) {
        for (int k = 0; k < 3; k++) bc->ph[k] += ph[k];
        bc->parity = p;
    }
}

// ---- launch-per-phase form (when a cooperative launch is not available) --------------------

__device__ __forceinline__ bool running(const Ctl* c) { return ld_relaxed(&c->done) == 0; }

template <int D>
__global__ void __launch_bounds__(256) k_fr_grad(FrontierBufs B, Dims dm) {
    if (!running(B.ctl)) return;
    phase_grad<D>(B, dm, ld_relaxed(&B.ctl->it), blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

template <int D>
__global__ void __launch_bounds__(256) k_fr_vr(FrontierBufs B, Dims dm) {
    if (!running(B.ctl)) return;
    const int it = ld_relaxed(&B.ctl->it);
    phase_vr<D>(B, dm, it, (long long)it != B.max_iters, blockIdx.x * blockDim.x + threadIdx.x,
                gridDim.x * blockDim.x);
}

template <int D>
__global__ void __launch_bounds__(256) k_fr_sapply(FrontierBufs B, Dims dm) {
    const int it = ld_relaxed(&B.ctl->it);
    if (!running(B.ctl) || B.tier < 3 || c_total(slot_of(B, it)) != 0) return;
    phase_sapply<D>(B, dm, it, (long long)it != B.max_iters, blockIdx.x * blockDim.x + threadIdx.x,
                    gridDim.x * blockDim.x);
}

__global__ void k_fr_finish(FrontierBufs B) {
    Ctl* c = B.ctl;
    if (c->done) return;
    const int it = c->it;
    const int state = iteration_state(B, it);
    record_iteration(B, it, state);
    if (state) { c->done = state; return; }
    c->it = it + 1;
}

}  // namespace dmt
