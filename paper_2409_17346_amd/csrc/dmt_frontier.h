// Frontier form of the C/S correction loop (Sections 4.3-4.6), device-controlled.
//
// The iteration is Jacobi: on g^(k), collect every violation's target vertex, then give each
// requested vertex one Equation 2 step.  Between iterations only the edited vertices change,
// so only a neighbourhood of them needs new work:
//   * a cell's pairing depends on the values on the closed 1-ring of its highest vertex, so
//     the gradient is recomputed for the closed 1-ring of every edited vertex (dirty vertices);
//   * a cell's violation (and its target) depends on its own codes and vertex values, so the
//     violation masks are recomputed for the anchors of cells touching a dirty vertex;
//   * every current violation requests its target again each iteration, so the anchors with a
//     non-zero violation mask are kept in a list that is compacted as masks clear.
// Lists are deduplicated with per-iteration stamps (atomicMax) and filled with wave-aggregated
// appends.  All control decisions live in a device control block, so the host only has to
// look at it once per batch of iterations.  The result is the same set arithmetic as the
// dense form, hence bit-identical output.
#pragma once
#include "dmt_kernels.h"

namespace dmt {

// Per-iteration counters live in slot it % 3: iteration it fills its own slot and the list
// lengths of slot (it+1) % 3, and slot (it+1) % 3 is cleared at the start of iteration it (its
// last readers belong to iteration it-2, so no reader can race with the clear).  List buffers
// alternate by iteration parity.
struct Slot {
    unsigned long long cnt[CNT_WORDS];  // log record layout
    int n_req;              // requests of this iteration
    int n_dv, n_da, n_vl;   // dirty vertices, affected anchors, violation list of this iteration
};

struct Ctl {
    int it;                 // next iteration to execute
    int done;               // 0 running, 1 converged, 2 iteration cap, 3 stalled, 4 paused (log full)
    int c_it, s_it;
    long long residual;
    unsigned bar_count, bar_gen;  // grid barrier of the persistent kernel
    int err;                      // 1: a grid barrier timed out
    int pad;
    unsigned long long ph[8];     // wall-clock ticks (100 MHz) per loop phase, seen from block 0
    Slot slot[3];
};

struct FrontierBufs {
    Ctl* ctl;
    const float *f, *gh, *lo;
    float* g;
    uint8_t* state;
    const uint8_t* fpl;
    uint8_t* gpl;
    uint32_t* vmask;        // violating planes per anchor
    uint8_t* inlist;        // anchor is in the violation list
    int* vl[2];             // violation anchor lists
    int* dvl[2];            // dirty vertex lists
    int* dal[2];            // affected anchor lists
    unsigned* vstamp;       // dirty-vertex stamps
    unsigned* astamp;       // affected-anchor stamps
    unsigned* rstamp;       // request stamps
    int* reql;              // request list
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

__device__ __forceinline__ void request(const FrontierBufs& B, int v, unsigned stamp, int* n_req) {
    const bool mine = atomicMax(&B.rstamp[v], stamp) < stamp;
    const int idx = wave_append(mine, n_req);
    if (mine) B.reql[idx] = v;
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

// ---- targets of the violating planes of one anchor (same rules as classify_plane) ---------

template <int D, int P>
__device__ __forceinline__ void target_plane(const FrontierBufs& B, const Dims& dm, int a, uint32_t m,
                                             unsigned stamp, int* cnt, int* n_req) {
    constexpr auto& g = G<D>::g;
    constexpr int dim = g.bdim[P];
    if ((m >> P) & 1u) {
        const uint8_t fc = B.fpl[(size_t)P * dm.n + a];
        const uint8_t gc = B.gpl[(size_t)P * dm.n + a];
        int target;
        if (fc != CODE_CRIT) {
            target = a + c27_lin(dm, fc & 63);
            cnt[2 * dim]++;
        } else {
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
                const float gw = B.g[w];
                if (best < 0 || prec(gw, w, gbest, best)) { best = w; gbest = gw; }
            }
            if (best < 0) {
                int fa = a, fp = 0;
#pragma unroll
                for (int k = 0; k < g.bnv[P]; k++) {
                    if (k == kx) {
                        fa = a + g.facet_anchor[P][k][0] + dm.nx * g.facet_anchor[P][k][1] +
                             dm.nxy * g.facet_anchor[P][k][2];
                        fp = g.facet_plane[P][k];
                    }
                }
                best = fa + c27_lin(dm, B.fpl[(size_t)fp * dm.n + fa] & 63);
            }
            target = best;
            cnt[2 * dim + 1]++;
        }
        request(B, target, stamp, n_req);
    }
    if constexpr (P + 1 < Geom<D>::NB) target_plane<D, P + 1>(B, dm, a, m, stamp, cnt, n_req);
}

// ---- phases ------------------------------------------------------------------------------

// Phase 1: gradient of g for the dirty vertices (every vertex at iteration 0).
template <int D>
__device__ __forceinline__ void phase_grad(const FrontierBufs& B, const Dims& dm, int it, int gtid, int gsize) {
    const int n = it == 0 ? dm.n : ld_relaxed(&slot_of(B, it).n_dv);
    const int* list = B.dvl[it & 1];
    for (int i = gtid; i < n; i += gsize) grad_vertex<D>(it == 0 ? i : list[i], B.g, B.gpl, dm);
}

// Phase 2: violation masks of the affected anchors; new violators join the list.
template <int D>
__device__ __forceinline__ void phase_vmask(const FrontierBufs& B, const Dims& dm, int it, int gtid, int gsize) {
    const int n = it == 0 ? dm.n : ld_relaxed(&slot_of(B, it).n_da);
    const int* list = B.dal[it & 1];
    int* vl = B.vl[it & 1];
    int* n_vl = &slot_of(B, it).n_vl;
    for (int i0 = gtid; i0 - (int)threadIdx.x < n; i0 += gsize) {   // whole blocks iterate together
        const bool act = i0 < n;
        bool add = false;
        int a = 0;
        if (act) {
            a = it == 0 ? i0 : list[i0];
            int x, y, z;
            coords(dm, a, x, y, z);
            uint32_t m = 0;
            vmask_plane<D, 0>(dm, a, x, y, z, B.fpl, B.gpl, B.tier, m);
            B.vmask[a] = m;
            add = m != 0 && !B.inlist[a];
            if (add) B.inlist[a] = 1;
        }
        const int idx = wave_append(add, n_vl);
        if (add) vl[idx] = a;
    }
}

// Phase 3: every listed anchor with violations requests its targets; cleared anchors leave.
template <int D>
__device__ __forceinline__ void phase_requests(const FrontierBufs& B, const Dims& dm, int it, int gtid, int gsize) {
    Slot& S = slot_of(B, it);
    const int n = ld_relaxed(&S.n_vl);
    const int* list = B.vl[it & 1];
    int* out = B.vl[(it + 1) & 1];
    int* n_out = &slot_of(B, it + 1).n_vl;
    const unsigned stamp = (unsigned)it + 1u;
    int cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int i0 = gtid; i0 - (int)threadIdx.x < n; i0 += gsize) {
        const bool act = i0 < n;
        int a = 0;
        uint32_t m = 0;
        if (act) {
            a = list[i0];
            m = B.vmask[a];
            if (m == 0) B.inlist[a] = 0;
        }
        const bool keep = act && m != 0;
        const int idx = wave_append(keep, n_out);
        if (keep) {
            out[idx] = a;
        }
        if (keep) target_plane<D, 0>(B, dm, a, m, stamp, cnt, &S.n_req);
    }
    block_add_counters<8>(S.cnt + CNT_FP0, cnt);
}

// Phase 4 (S-step, only when no critical-cell violation remains and tier >= 3): first cell
// along each f-branch whose g pairing differs.
template <int D>
__device__ __forceinline__ void phase_scheck(const FrontierBufs& B, const Dims& dm, int gtid, int gsize) {
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

// Phase 5: troublemaker targets (apex of the f-pair of the first differing cell).
template <int D>
__device__ __forceinline__ void phase_stargets(const FrontierBufs& B, const Dims& dm, int it, int gtid, int gsize) {
    constexpr auto& g = G<D>::g;
    const unsigned stamp = (unsigned)it + 1u;
    int c[2] = {0, 0};
    const int nb = B.n_desc + B.n_asc;
    for (int i0 = gtid; i0 - (int)threadIdx.x < nb; i0 += gsize) {
        int target = -1;
        int fam = 0;
        if (i0 < nb) {
            const bool asc = i0 >= B.n_desc;
            const int b = asc ? i0 - B.n_desc : i0;
            int* first = asc ? B.afirst : B.dfirst;
            const int* cells = asc ? B.acell : B.dcell;
            const int64_t* off = asc ? B.aoff : B.doff;
            const int* term = asc ? B.aterm : B.dterm;
            const int k = first[b];
            if (k != INF32) {
                first[b] = INF32;
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
                    fam = asc ? 1 : 0;
                    c[fam]++;
                }
            }
        }
        if (target >= 0) request(B, target, stamp, &slot_of(B, it).n_req);
    }
    block_add_counters<2>(slot_of(B, it).cnt + CNT_TM_DESC, c);
}

// Phase 6: decision and Equation 2 for every requested vertex; edited vertices mark the next
// iteration's dirty vertices and affected anchors.  Returns false when the loop ends here.
template <int D>
__device__ __forceinline__ void phase_apply(const FrontierBufs& B, const Dims& dm, int it, int gtid, int gsize) {
    constexpr auto& g = G<D>::g;
    Slot& S = slot_of(B, it);
    Slot& N1 = slot_of(B, it + 1);
    const int n = ld_relaxed(&S.n_req);
    const int nxt = (it + 1) & 1;
    const unsigned stamp = (unsigned)it + 1u;
    int c = 0;
    for (int i0 = gtid; i0 - (int)threadIdx.x < n; i0 += gsize) {
        bool changed = false;
        int v = 0;
        if (i0 < n) {
            v = B.reql[i0];
            const uint8_t st = B.state[v];
            if (!(st & 0x80)) {
                const int q = st & 7;
                const float t = fmaf(-(float)(q + 1), B.delta, B.gh[v]);
                const float l = B.lo[v];
                if (q < B.q_max && t >= l) {
                    B.state[v] = (uint8_t)(q + 1);
                    B.g[v] = t;
                } else {
                    B.state[v] = (uint8_t)(0x80 | q);
                    B.g[v] = l;
                }
                changed = true;
                c++;
            }
        }
        // mark the closed 1-ring as dirty and the anchors of cells touching it as affected
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
                mine = atomicMax(&B.astamp[a], stamp) < stamp;
            }
            const int idx = wave_append(mine, &N1.n_da);
            if (mine) B.dal[nxt][idx] = a;
        }
    }
    block_add_counters<1>(S.cnt + CNT_CHANGED, &c);
}

// ---- iteration bookkeeping shared by both drivers ------------------------------------------

__device__ __forceinline__ void clear_slot(Slot& s) {
    for (int k = 0; k < CNT_WORDS; k++) s.cnt[k] = 0;
    s.n_req = s.n_dv = s.n_da = s.n_vl = 0;
}

// Stall test, log record and counters of a finished iteration (one thread).
// Returns the loop's end state (0 = go on).
__device__ __forceinline__ int finish_iteration(const FrontierBufs& B, int it) {
    Ctl* c = B.ctl;
    const Slot& S = c->slot[it % 3];
    const unsigned long long ct = c_total(S);
    const bool cstep = ct != 0;
    const unsigned long long viol = cstep ? ct : ld_relaxed(&S.cnt[CNT_TM_DESC]) + ld_relaxed(&S.cnt[CNT_TM_ASC]);
    if (ld_relaxed(&S.cnt[CNT_CHANGED]) == 0) { c->residual = (long long)viol; return 3; }
    long long* rec = B.log + (size_t)it * DMT_LOG_WORDS;
    rec[0] = cstep ? 1 : 2;
    for (int k = 1; k < CNT_NREQ; k++) rec[k] = (long long)ld_relaxed(&S.cnt[k]);
    rec[CNT_NREQ] = ld_relaxed(&S.n_req);
    rec[CNT_CHANGED] = (long long)ld_relaxed(&S.cnt[CNT_CHANGED]);
    for (int k = CNT_CHANGED + 1; k < DMT_LOG_WORDS; k++) rec[k] = 0;
    if (cstep) c->c_it++; else c->s_it++;
    return 0;
}

__global__ void k_fr_init(Ctl* c) {
    c->it = 0;
    c->done = 0;
    c->c_it = c->s_it = 0;
    c->residual = 0;
    c->bar_count = c->bar_gen = 0;
    c->err = 0;
    for (int i = 0; i < 8; i++) c->ph[i] = 0;
    for (int i = 0; i < 3; i++) clear_slot(c->slot[i]);
}

// ---- persistent form: the whole loop in one cooperative launch ----------------------------

// Grid-wide barrier on a generation counter.  Arrival is a release at agent scope (the block's
// writes become visible to every XCD); waiting polls with relaxed loads (an acquire per poll
// would invalidate the XCD's L2 each time) and ends with one acquire fence.  A block that waits
// longer than the timeout (wall clock, 100 MHz) reports it and the caller leaves the loop, so a
// lost block can never hang the device.
__device__ __forceinline__ bool grid_barrier(Ctl* c, unsigned nblocks, unsigned& gen, unsigned long long timeout) {
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

template <int D>
__global__ void __launch_bounds__(256) k_fr_loop(FrontierBufs B, Dims dm, int log_cap, unsigned long long timeout) {
    Ctl* c = B.ctl;
    const unsigned nblocks = gridDim.x;
    const int gtid = blockIdx.x * blockDim.x + threadIdx.x;
    const int gsize = gridDim.x * blockDim.x;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    unsigned gen = __hip_atomic_load(&c->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int it = __hip_atomic_load(&c->it, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // every block starts from the same generation
    if (!grid_barrier(c, nblocks, gen, timeout)) return;
    int state = 0;
    unsigned long long ph[6] = {0, 0, 0, 0, 0, 0};
    unsigned long long t = lead ? wall_clock64() : 0;
    auto tick = [&](int k) {
        if (lead) { const unsigned long long t1 = wall_clock64(); ph[k] += t1 - t; t = t1; }
    };
    for (;;) {
        // iteration 0's dense gradient and violation masks ran as full-grid launches
        if (it > 0) {
            if (lead) clear_slot(c->slot[(it + 1) % 3]);
            phase_grad<D>(B, dm, it, gtid, gsize);
            if (!grid_barrier(c, nblocks, gen, timeout)) return;
            tick(0);
            phase_vmask<D>(B, dm, it, gtid, gsize);
            if (!grid_barrier(c, nblocks, gen, timeout)) return;
            tick(1);
        }
        phase_requests<D>(B, dm, it, gtid, gsize);
        if (!grid_barrier(c, nblocks, gen, timeout)) return;
        tick(2);
        if (B.tier >= 3 && c_total(c->slot[it % 3]) == 0) {
            phase_scheck<D>(B, dm, gtid, gsize);
            if (!grid_barrier(c, nblocks, gen, timeout)) return;
            tick(3);
            phase_stargets<D>(B, dm, it, gtid, gsize);
            if (!grid_barrier(c, nblocks, gen, timeout)) return;
            tick(4);
        }
        const unsigned long long viol = violations(B, it);
        if (viol == 0) { state = 1; break; }
        if ((long long)it == B.max_iters) { state = 2; if (lead) c->residual = (long long)viol; break; }
        phase_apply<D>(B, dm, it, gtid, gsize);
        if (!grid_barrier(c, nblocks, gen, timeout)) return;
        tick(5);
        if (ld_relaxed(&c->slot[it % 3].cnt[CNT_CHANGED]) == 0) {
            state = 3;
            if (lead) finish_iteration(B, it);
            break;
        }
        if (lead) finish_iteration(B, it);
        it++;
        if (it >= log_cap) { state = 4; break; }
    }
    if (lead)
        for (int k = 0; k < 6; k++) c->ph[k] += ph[k];
    if (lead) {
        c->it = it;
        c->done = state;
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
__global__ void __launch_bounds__(256) k_fr_vmask(FrontierBufs B, Dims dm) {
    if (!running(B.ctl)) return;
    phase_vmask<D>(B, dm, ld_relaxed(&B.ctl->it), blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

template <int D>
__global__ void __launch_bounds__(256) k_fr_requests(FrontierBufs B, Dims dm) {
    if (!running(B.ctl)) return;
    phase_requests<D>(B, dm, ld_relaxed(&B.ctl->it), blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

template <int D>
__global__ void __launch_bounds__(256) k_fr_scheck(FrontierBufs B, Dims dm) {
    if (!running(B.ctl) || B.tier < 3 || c_total(slot_of(B, ld_relaxed(&B.ctl->it))) != 0) return;
    phase_scheck<D>(B, dm, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

template <int D>
__global__ void __launch_bounds__(256) k_fr_stargets(FrontierBufs B, Dims dm) {
    const int it = ld_relaxed(&B.ctl->it);
    if (!running(B.ctl) || B.tier < 3 || c_total(slot_of(B, it)) != 0) return;
    phase_stargets<D>(B, dm, it, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

// decision (converged / iteration cap) before the edits, then the edits
template <int D>
__global__ void __launch_bounds__(256) k_fr_apply(FrontierBufs B, Dims dm) {
    if (!running(B.ctl)) return;
    const int it = ld_relaxed(&B.ctl->it);
    const unsigned long long viol = violations(B, it);
    if (viol == 0 || (long long)it == B.max_iters) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            B.ctl->residual = viol == 0 ? 0 : (long long)viol;
            B.ctl->done = viol == 0 ? 1 : 2;
        }
        return;
    }
    phase_apply<D>(B, dm, it, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

__global__ void k_fr_finish(FrontierBufs B) {
    Ctl* c = B.ctl;
    if (c->done) return;
    const int it = c->it;
    const int st = finish_iteration(B, it);
    if (st) { c->done = st; return; }
    c->it = it + 1;
    clear_slot(c->slot[(it + 2) % 3]);
}

}  // namespace dmt
