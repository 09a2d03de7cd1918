// Host side of the C ABI declared in include/dmt.h: validation, workspaces, MSC extraction and
// the driver of the C-loop / S-loop correction (Sections 4.2-4.6 of the paper).  All arithmetic
// on field values happens in the kernels of dmt_kernels.h and dmt_frontier.h; the host only
// sequences launches, sizes buffers and reads counters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>
#include <atomic>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "dmt.h"
#include "dmt_frontier.h"
#include "dmt_verify.h"
#include "dmt_codec.h"

using namespace dmt;

// Scratch memory of the allocation-free correction (dmt_correct_noalloc): one array per device,
// loaded with the code object and held until the process ends.  Host code never uses this name
// as an address; its device address is resolved once per device (scratch_address below).
static __device__ __align__(256) unsigned char scratch[DMT_NOALLOC_SCRATCH_BYTES];

namespace {

// Device address of `scratch` on each device, resolved once with that device current.
std::mutex scratch_mu;
std::vector<int> scratch_state;         // 0 not yet resolved, 1 resolved, -1 failed
std::vector<char*> scratch_ptr;
std::vector<std::string> scratch_msg;

// Resolves (once) the scratch address of the current device `dev` of ndev; nullptr and a message
// when the runtime cannot give it.
char* scratch_address(int dev, int ndev, std::string& msg) {
    std::lock_guard<std::mutex> lk(scratch_mu);
    if ((int)scratch_state.size() < ndev) {
        scratch_state.resize(ndev, 0);
        scratch_ptr.resize(ndev, nullptr);
        scratch_msg.resize(ndev);
    }
    if (scratch_state[dev] == 0) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e == hipSuccess && p) {
            scratch_ptr[dev] = static_cast<char*>(p);
            scratch_state[dev] = 1;
        } else {
            (void)hipGetLastError();
            scratch_msg[dev] = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            scratch_state[dev] = -1;
        }
    }
    msg = scratch_msg[dev];
    return scratch_ptr[dev];
}

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
};

constexpr int TPB = 256;
constexpr int HAND_STREAMS = 4;  // streams for the grid iterations of paused batch jobs
constexpr int GRID_RUN_MAX = 16;  // longest doubled hand-off run (grid_iterations if that is more)
inline unsigned nblocks(int64_t n) { return (unsigned)((n + TPB - 1) / TPB); }
// blocks of a classification launch: one per chunk of CLASSIFY_APB anchors, at most cap
inline unsigned classify_blocks(int64_t n, unsigned cap = ~0u) {
    const unsigned b = (unsigned)((n + CLASSIFY_APB - 1) / CLASSIFY_APB);
    return b < cap ? b : cap;
}

// Critical cells and separatrix branches of one gradient (device arrays, int32 ids).
struct MscBufs {
    DevBuf crit[4];
    int64_t ncrit[4] = {0, 0, 0, 0};
    DevBuf dlen, dterm, doff, dfirst, dcell, dcbr;
    DevBuf asadcnt, asadoff, astart, asad, alen, aterm, aoff, afirst, acell, acbr;
    DevBuf vlab, tlab;
    int64_t n_desc = 0, n_desc_cells = 0, n_asc = 0, n_asc_cells = 0, n_vlab = 0, n_tlab = 0;
    bool valid = false;
    std::vector<DevBuf*> all() {
        return {&crit[0], &crit[1], &crit[2], &crit[3], &dlen, &dterm, &doff, &dfirst, &dcell, &dcbr, &asadcnt,
                &asadoff, &astart, &asad, &alen, &aterm, &aoff, &afirst, &acell, &acbr, &vlab, &tlab};
    }
};

// Device state of one correction job.
struct JobWs {
    DevBuf lo, g0, g1, state, fpl, gpl, vmask, vl0, vl1, dvl0, dvl1, dal0, dal1, stamps;
    DevBuf vpos, vstart, tsum, toff, ecell, bstamp, tcl, dbl, newmin, btgt, cand0, cand1, inlist;
    DevBuf ss_src, ss_q0, ss_q1, ss_stamp;
    DevBuf fofs, ftgt, dreq, frz;
    MscBufs msc;
    std::vector<DevBuf*> all() {
        std::vector<DevBuf*> v = {&lo,     &g0,     &g1,      &state,  &fpl,   &gpl,   &vmask,  &vl0,
                                  &vl1,    &dvl0,   &dvl1,    &dal0,   &dal1,  &stamps, &vpos,   &vstart,
                                  &tsum,   &toff,   &ecell,   &bstamp, &tcl,
                                  &dbl,    &newmin, &btgt,    &cand0,   &cand1,  &inlist, &ss_src, &ss_q0,  &ss_q1,
                                  &ss_stamp, &fofs, &ftgt,  &dreq,    &frz};
        for (DevBuf* b : msc.all()) v.push_back(b);
        return v;
    }
};

}  // namespace

namespace {
// The launch shapes the library uses unless dmt_set_tuning says otherwise.
dmt_tuning default_tuning() {
    dmt_tuning t;
    t.loop_threads[0] = 1024;
    t.loop_threads[1] = 512;
    t.handoff_anchors[0] = 8192;
    t.handoff_anchors[1] = 1024;
    t.grid_iterations[0] = 4;
    t.grid_iterations[1] = 64;
    t.batch_handoff_anchors[0] = 8192;
    t.batch_handoff_anchors[1] = 8192;
    return t;
}
}  // namespace

struct dmt_context {
    int device = 0;
    std::string err;
    std::vector<JobWs> ws;                 // one workspace per job of the last batch (ws[0]: single calls)
    MscBufs msc;                           // results of dmt_extract_msc
    MscBufs cmp[2];                        // the two complexes of dmt_compare_msc
    DevBuf gpl2, agree;                    // dmt_compare_msc: second field's planes, counters
    DevBuf gpl, req, cnt, flags, part, blk, blkoff, ll_idx, ll_val, dlog, jobs_dev, ctl_all, queue, scan_tsum, scan_toff;
    int64_t n_lossless = 0;
    std::vector<int64_t> log;
    unsigned long long* hcnt = nullptr;    // pinned
    int64_t* hscratch = nullptr;           // pinned
    std::vector<Ctl> hctl;                 // per-job control blocks read back after the loop
    hipStream_t side = nullptr;            // the 3D loop kernel of a mixed batch runs here
    hipEvent_t fork = nullptr, join = nullptr;
    // grid iterations of paused jobs of a batch run side by side on these, forked from the
    // launch stream and joined back into it
    hipStream_t hand[HAND_STREAMS] = {};
    hipEvent_t hand_join[HAND_STREAMS] = {};
    unsigned long long ph[3] = {0, 0, 0};  // loop phase ticks of the last correction call
    // kernel timing: event pairs per kernel family, recorded on the launch stream
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev[DMT_PROF_KERNELS];
    int64_t prof_units[DMT_PROF_KERNELS] = {0};
    dmt_tuning tune = default_tuning();
    // allocation-free calls: this device's scratch array (its device address, 0 if it could
    // not be resolved) and, while such a call runs, a bump arena over it that every buffer of
    // the call is carved from instead of hipMalloc
    char* scratch = nullptr;
    std::string scratch_err;
    bool arena_on = false;
    size_t arena_used = 0;
};

namespace {

dmt_status fail(dmt_context* c, dmt_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

#define HIPCHK(ctx, expr)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail((ctx), DMT_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));   \
    } while (0)

#define CHECK_LAUNCH(ctx) HIPCHK(ctx, hipGetLastError())

// Carves bytes (256-aligned) from the scratch arena of an allocation-free call.
dmt_status arena_take(dmt_context* c, DevBuf& b, size_t bytes) {
    const size_t off = (c->arena_used + 255) & ~(size_t)255;
    if (off + bytes > (size_t)DMT_NOALLOC_SCRATCH_BYTES)
        return fail(c, DMT_E_NOMEM, "the allocation-free path needs more than its " +
                                        std::to_string((long long)DMT_NOALLOC_SCRATCH_BYTES) +
                                        " bytes of scratch for this field");
    b.p = c->scratch + off;
    b.cap = bytes;
    c->arena_used = off + bytes;
    return DMT_OK;
}

dmt_status ensure(dmt_context* c, DevBuf& b, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (b.cap >= bytes) return DMT_OK;
    // in an allocation-free call every buffer was emptied at entry, so b (if set) is an
    // arena buffer of this call: carve a larger one and leave the old space unused
    if (c->arena_on) return arena_take(c, b, bytes);
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, DMT_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    b.cap = bytes;
    return DMT_OK;
}

#define ENSURE(ctx, buf, bytes)                        \
    do {                                               \
        dmt_status s_ = ensure((ctx), (buf), (bytes)); \
        if (s_ != DMT_OK) return s_;                   \
    } while (0)

#define TRY(expr)                         \
    do {                                  \
        dmt_status s_ = (expr);           \
        if (s_ != DMT_OK) return s_;      \
    } while (0)

template <typename T>
T* P(DevBuf& b) { return reinterpret_cast<T*>(b.p); }

// The context's shared device buffers (not those of job workspaces or of dmt_extract_msc).
std::vector<DevBuf*> context_bufs(dmt_context* c) {
    return {&c->gpl,    &c->req,      &c->cnt,   &c->flags, &c->part,      &c->blk,      &c->blkoff, &c->ll_idx,
            &c->ll_val, &c->dlog,     &c->jobs_dev, &c->ctl_all, &c->queue, &c->scan_tsum, &c->scan_toff};
}

dmt_status check_grid(dmt_context* c, const dmt_grid* gr, Dims& dm, int& D) {
    if (!gr) return fail(c, DMT_E_INVALID, "grid is NULL");
    if (gr->ndim != 2 && gr->ndim != 3) return fail(c, DMT_E_INVALID, "ndim must be 2 or 3");
    if (gr->nx < 2 || gr->ny < 2) return fail(c, DMT_E_INVALID, "nx and ny must be >= 2");
    if (gr->ndim == 2 && gr->nz != 1) return fail(c, DMT_E_INVALID, "2D grids need nz == 1");
    if (gr->ndim == 3 && gr->nz < 2) return fail(c, DMT_E_INVALID, "3D grids need nz >= 2");
    const int64_t n = gr->nx * gr->ny * gr->nz;
    // internal cell ids are int32: N * (cells per anchor of the largest dimension) < 2^31
    const int64_t tmax = gr->ndim == 2 ? 3 : 12;
    if (n > (int64_t)INT32_MAX / tmax) return fail(c, DMT_E_INVALID, "grid too large");
    D = gr->ndim;
    dm.nx = (int)gr->nx;
    dm.ny = (int)gr->ny;
    dm.nz = (int)gr->nz;
    dm.nxy = dm.nx * dm.ny;
    dm.n = (int)n;
    set_divisors(dm);
    return DMT_OK;
}

dmt_status check_options(dmt_context* c, const dmt_options* o, float xi) {
    if (!o) return fail(c, DMT_E_INVALID, "options are NULL");
    if (o->tier < 1 || o->tier > 4) return fail(c, DMT_E_INVALID, "tier must be 1..4");
    if (o->q_max < 0 || o->q_max > 7) return fail(c, DMT_E_INVALID, "q_max must be 0..7");
    if (o->flags & ~(uint32_t)(DMT_F_DENSE | DMT_F_PHASES | DMT_F_SADDLE_SADDLE))
        return fail(c, DMT_E_INVALID, "unknown flags");
    if (!(xi > 0.0f) || !std::isfinite(xi)) return fail(c, DMT_E_INVALID, "xi must be finite and > 0");
    if (!(ldexpf(xi, -o->q_max) >= FLT_MIN)) return fail(c, DMT_E_INVALID, "xi / 2^q_max is not a normal float");
    return DMT_OK;
}

// bytes of code planes per vertex (anchor-major, padded)
int plane_bytes(int D) { return D == 2 ? plane_stride<2>() : plane_stride<3>(); }
int ntypes(int D, int d) { return D == 2 ? G<2>::g.ntypes[d] : G<3>::g.ntypes[d]; }

hipEvent_t next_event(dmt_context* c) {
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->ev_pool.push_back(e);
    }
    return c->ev_pool[c->ev_used++];
}

// Brackets the launches of kernel family k with events when timing is on.
struct ProfScope {
    dmt_context* c;
    int k;
    hipStream_t st;
    hipEvent_t e0 = nullptr;
    ProfScope(dmt_context* c_, int k_, hipStream_t st_, int64_t units) : c(c_), k(k_), st(st_) {
        if (!c->prof) return;
        e0 = next_event(c);
        if (e0) (void)hipEventRecord(e0, st);
        c->prof_units[k] += units;
    }
    ~ProfScope() {
        if (!c->prof || !e0) return;
        hipEvent_t e1 = next_event(c);
        if (!e1) return;
        (void)hipEventRecord(e1, st);
        c->prof_ev[k].push_back({e0, e1});
    }
};

dmt_status launch_grad(dmt_context* c, int D, const float* h, uint8_t* pl, const Dims& dm, hipStream_t st) {
    ProfScope ps(c, DMT_PROF_GRADIENT, st, dm.n);
    if (D == 2) k_grad<2><<<nblocks(dm.n), TPB, 0, st>>>(h, pl, dm);
    else k_grad<3><<<nblocks(dm.n), TPB, 0, st>>>(h, pl, dm);
    CHECK_LAUNCH(c);
    return DMT_OK;
}

// exclusive scan of n ints into n+1 int64 (device); the total is returned on the host
dmt_status scan(dmt_context* c, const int* in, int64_t n, int64_t* out, int64_t* total, hipStream_t st) {
    if (n <= 65536) {
        k_scan_single<<<1, 1024, 0, st>>>(in, n, out);
    } else {
        // tiles of 1024: tile sums, a single-block scan of the sums, then each tile's prefix
        const int64_t ntiles = (n + 1023) / 1024;
        ENSURE(c, c->scan_tsum, sizeof(int) * (size_t)ntiles);
        ENSURE(c, c->scan_toff, sizeof(int64_t) * (size_t)(ntiles + 1));
        k_tile_sum<<<(unsigned)ntiles, TPB, 0, st>>>(in, (int)n, P<int>(c->scan_tsum));
        k_scan_single<<<1, 1024, 0, st>>>(P<int>(c->scan_tsum), ntiles, P<int64_t>(c->scan_toff));
        k_tile_scan64<<<(unsigned)ntiles, TPB, 0, st>>>(in, (int)n, P<int64_t>(c->scan_toff), out);
    }
    CHECK_LAUNCH(c);
    if (total) {
        HIPCHK(c, hipMemcpyAsync(c->hscratch, out + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        *total = c->hscratch[0];
    }
    return DMT_OK;
}

dmt_status fill_i32(dmt_context* c, int* p, int64_t n, int value, hipStream_t st) {
    if (n <= 0) return DMT_OK;
    HIPCHK(c, hipMemsetD32Async((hipDeviceptr_t)p, value, (size_t)n, st));
    return DMT_OK;
}

// Critical cells, separatrix branches and (optionally) manifold labels of the gradient in
// planes pl (Section 3.1).
template <int D>
dmt_status build_msc(dmt_context* c, MscBufs& m, const uint8_t* pl, const Dims& dm, bool labels, hipStream_t st) {
    constexpr auto& g = G<D>::g;
    const unsigned nb = nblocks(dm.n);
    m.valid = false;
    ENSURE(c, c->flags, 16);
    HIPCHK(c, hipMemsetAsync(c->flags.p, 0, sizeof(unsigned), st));
    unsigned* werr = P<unsigned>(c->flags);
    ENSURE(c, c->blk, sizeof(int) * (size_t)(D + 1) * nb);
    ENSURE(c, c->blkoff, sizeof(int64_t) * (size_t)(D + 1) * (nb + 1));
    k_crit_count<D><<<nb, TPB, 0, st>>>(pl, dm, P<int>(c->blk));
    CHECK_LAUNCH(c);
    for (int d = 0; d <= D; d++) {
        TRY(scan(c, P<int>(c->blk) + (size_t)d * nb, nb, P<int64_t>(c->blkoff) + (size_t)d * (nb + 1), &m.ncrit[d],
                 st));
        ENSURE(c, m.crit[d], sizeof(int) * (size_t)m.ncrit[d]);
    }
    for (int d = D + 1; d < 4; d++) m.ncrit[d] = 0;
    k_crit_write<D><<<nb, TPB, 0, st>>>(pl, dm, P<int64_t>(c->blkoff), (int)nb, P<int>(m.crit[0]), P<int>(m.crit[1]),
                                        P<int>(m.crit[2]), D == 3 ? P<int>(m.crit[3]) : nullptr);
    CHECK_LAUNCH(c);

    // descending branches: two per 1-saddle
    m.n_desc = 2 * m.ncrit[1];
    ENSURE(c, m.dlen, sizeof(int) * (size_t)m.n_desc);
    ENSURE(c, m.dterm, sizeof(int) * (size_t)m.n_desc);
    ENSURE(c, m.doff, sizeof(int64_t) * (size_t)(m.n_desc + 1));
    ENSURE(c, m.dfirst, sizeof(int) * (size_t)m.n_desc);
    if (m.n_desc) {
        k_desc_walk<D><<<nblocks(m.n_desc), TPB, 0, st>>>(pl, dm, P<int>(m.crit[1]), (int)m.n_desc, 0, P<int>(m.dlen),
                                                          P<int>(m.dterm), nullptr, nullptr, nullptr, werr);
        CHECK_LAUNCH(c);
    }
    TRY(scan(c, P<int>(m.dlen), m.n_desc, P<int64_t>(m.doff), &m.n_desc_cells, st));
    ENSURE(c, m.dcell, sizeof(int) * (size_t)m.n_desc_cells);
    ENSURE(c, m.dcbr, sizeof(int) * (size_t)m.n_desc_cells);
    if (m.n_desc) {
        k_desc_walk<D><<<nblocks(m.n_desc), TPB, 0, st>>>(pl, dm, P<int>(m.crit[1]), (int)m.n_desc, 1, nullptr, nullptr,
                                                          P<int64_t>(m.doff), P<int>(m.dcell), P<int>(m.dcbr), werr);
        CHECK_LAUNCH(c);
    }
    TRY(fill_i32(c, P<int>(m.dfirst), m.n_desc, INF32, st));

    // ascending branches: one per top cofacet of each (D-1)-saddle
    const int64_t nsad = m.ncrit[D - 1];
    ENSURE(c, m.asadcnt, sizeof(int) * (size_t)nsad);
    ENSURE(c, m.asadoff, sizeof(int64_t) * (size_t)(nsad + 1));
    if (nsad) {
        k_asc_starts<D><<<nblocks(nsad), TPB, 0, st>>>(dm, P<int>(m.crit[D - 1]), (int)nsad, 0, P<int>(m.asadcnt),
                                                       nullptr, nullptr, nullptr);
        CHECK_LAUNCH(c);
    }
    TRY(scan(c, P<int>(m.asadcnt), nsad, P<int64_t>(m.asadoff), &m.n_asc, st));
    ENSURE(c, m.astart, sizeof(int) * (size_t)m.n_asc);
    ENSURE(c, m.asad, sizeof(int) * (size_t)m.n_asc);
    ENSURE(c, m.alen, sizeof(int) * (size_t)m.n_asc);
    ENSURE(c, m.aterm, sizeof(int) * (size_t)m.n_asc);
    ENSURE(c, m.aoff, sizeof(int64_t) * (size_t)(m.n_asc + 1));
    ENSURE(c, m.afirst, sizeof(int) * (size_t)m.n_asc);
    if (nsad) {
        k_asc_starts<D><<<nblocks(nsad), TPB, 0, st>>>(dm, P<int>(m.crit[D - 1]), (int)nsad, 1, nullptr,
                                                       P<int64_t>(m.asadoff), P<int>(m.astart), P<int>(m.asad));
        CHECK_LAUNCH(c);
    }
    if (m.n_asc) {
        k_asc_walk<D><<<nblocks(m.n_asc), TPB, 0, st>>>(pl, dm, P<int>(m.astart), (int)m.n_asc, 0, P<int>(m.alen),
                                                        P<int>(m.aterm), nullptr, nullptr, nullptr, werr);
        CHECK_LAUNCH(c);
    }
    TRY(scan(c, P<int>(m.alen), m.n_asc, P<int64_t>(m.aoff), &m.n_asc_cells, st));
    ENSURE(c, m.acell, sizeof(int) * (size_t)m.n_asc_cells);
    ENSURE(c, m.acbr, sizeof(int) * (size_t)m.n_asc_cells);
    if (m.n_asc) {
        k_asc_walk<D><<<nblocks(m.n_asc), TPB, 0, st>>>(pl, dm, P<int>(m.astart), (int)m.n_asc, 1, nullptr, nullptr,
                                                        P<int64_t>(m.aoff), P<int>(m.acell), P<int>(m.acbr), werr);
        CHECK_LAUNCH(c);
    }
    TRY(fill_i32(c, P<int>(m.afirst), m.n_asc, INF32, st));
    HIPCHK(c, hipMemcpyAsync(c->hscratch, werr, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (*reinterpret_cast<unsigned*>(c->hscratch)) return fail(c, DMT_E_HIP, "internal error: a V-path did not end");

    m.n_vlab = m.n_tlab = 0;
    if (labels) {
        m.n_vlab = dm.n;
        m.n_tlab = (int64_t)dm.n * g.ntypes[D];
        ENSURE(c, m.vlab, sizeof(int) * (size_t)m.n_vlab);
        ENSURE(c, m.tlab, sizeof(int) * (size_t)m.n_tlab);
        k_label_init<D><<<nb, TPB, 0, st>>>(pl, dm, P<int>(m.vlab), P<int>(m.tlab));
        CHECK_LAUNCH(c);
        for (int round = 0; round < 64; round++) {
            HIPCHK(c, hipMemsetAsync(c->flags.p, 0, sizeof(unsigned), st));
            k_jump<<<nblocks(m.n_vlab), TPB, 0, st>>>(P<int>(m.vlab), m.n_vlab, P<unsigned>(c->flags));
            k_jump<<<nblocks(m.n_tlab), TPB, 0, st>>>(P<int>(m.tlab), m.n_tlab, P<unsigned>(c->flags));
            CHECK_LAUNCH(c);
            HIPCHK(c, hipMemcpyAsync(c->hscratch, c->flags.p, sizeof(unsigned), hipMemcpyDeviceToHost, st));
            HIPCHK(c, hipStreamSynchronize(st));
            if (*reinterpret_cast<unsigned*>(c->hscratch) == 0) break;
        }
    }
    m.valid = true;
    return DMT_OK;
}

dmt_status read_counters(dmt_context* c, hipStream_t st) {
    HIPCHK(c, hipMemcpyAsync(c->hcnt, c->cnt.p, sizeof(unsigned long long) * CNT_WORDS, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    return DMT_OK;
}

// ---- one correction job --------------------------------------------------------------------

struct Job {
    int D = 2;
    Dims dm{};
    const float* f = nullptr;
    const float* gh = nullptr;
    float xi = 0.0f;
    dmt_options o{};
    float* g_out = nullptr;
    uint8_t* q_out = nullptr;
    JobWs* w = nullptr;
    int slot = 0;           // index of the job's control block in ctl_all (and hctl)
    FrontierBufs B{};
    dmt_stats stats{};
    dmt_status status = DMT_OK;
    // hand-off run length (grid iterations) and the iteration its last run ended at; kept with the
    // job, so that a served job's runs keep growing across the server's rounds
    int krun = 0;
    int64_t resume_it = -2;
};

// a0 (floors, validation flag into *flag) and a1 (gradient of f): launches only.
template <int D>
dmt_status job_setup(dmt_context* c, Job& J, unsigned* flag, hipStream_t st) {
    JobWs& w = *J.w;
    const int n = J.dm.n;
    ENSURE(c, w.lo, sizeof(float) * n);
    ENSURE(c, w.g0, sizeof(float) * n);
    ENSURE(c, w.state, n);
    ENSURE(c, w.fpl, (size_t)plane_stride<D>() * n);
    ENSURE(c, w.gpl, (size_t)plane_stride<D>() * n);
    ENSURE(c, c->req, n);
    {
        ProfScope ps(c, DMT_PROF_SETUP, st, n);
        k_setup<<<nblocks(n), TPB, 0, st>>>(J.f, J.gh, J.xi, n, P<float>(w.lo), P<float>(w.g0), P<uint8_t>(w.state),
                                             P<uint8_t>(c->req), flag);
        CHECK_LAUNCH(c);
    }
    return launch_grad(c, D, J.f, P<uint8_t>(w.fpl), J.dm, st);
}

// Saddle-saddle state of a 3D tier-4 job with DMT_F_SADDLE_SADDLE (f's branches built): the edges
// of f's 2-saddles, the two walk queues (each level holds distinct edges, at most 7 per vertex)
// and zeroed edge stamps.  Returns whether the job walks its connectors.
template <int D>
dmt_status ss_setup(dmt_context* c, Job& J, bool& on, hipStream_t st) {
    on = false;
    if (D != 3 || J.o.tier != 4 || !(J.o.flags & DMT_F_SADDLE_SADDLE)) return DMT_OK;
    JobWs& w = *J.w;
    const int64_t n = J.dm.n;
    const int64_t n2 = w.msc.ncrit[2];
    if (7 * n >= (int64_t)INT32_MAX) return fail(c, DMT_E_INVALID, "grid too large for the saddle-saddle walk");
    ENSURE(c, w.ss_src, sizeof(int) * (size_t)(3 * n2));
    ENSURE(c, w.ss_q0, sizeof(int) * (size_t)(7 * n));
    ENSURE(c, w.ss_q1, sizeof(int) * (size_t)(7 * n));
    ENSURE(c, w.ss_stamp, sizeof(unsigned) * (size_t)(7 * n));
    HIPCHK(c, hipMemsetAsync(w.ss_stamp.p, 0, sizeof(unsigned) * (size_t)(7 * n), st));
    if (n2) {
        k_ss_sources<<<nblocks(n2), TPB, 0, st>>>(P<int>(w.msc.crit[2]), (int)n2, J.dm, P<int>(w.ss_src));
        CHECK_LAUNCH(c);
    }
    on = true;
    return DMT_OK;
}

// a2 (f-branches), frontier buffers and control block of a job whose setup passed; fills J.B.
template <int D>
dmt_status job_frontier(dmt_context* c, Job& J, Ctl* ctl, hipStream_t st) {
    JobWs& w = *J.w;
    const int n = J.dm.n;
    w.msc.valid = false;
    if (J.o.tier >= 3) {
        ProfScope ps(c, DMT_PROF_MSC, st, n);
        TRY(build_msc<D>(c, w.msc, P<uint8_t>(w.fpl), J.dm, false, st));
    }
    ENSURE(c, w.g1, sizeof(float) * n);
    ENSURE(c, w.vmask, sizeof(uint32_t) * n);
    ENSURE(c, w.vl0, sizeof(int) * n);
    ENSURE(c, w.vl1, sizeof(int) * n);
    ENSURE(c, w.dvl0, sizeof(int) * n);
    ENSURE(c, w.dvl1, sizeof(int) * n);
    ENSURE(c, w.dal0, sizeof(int) * n);
    ENSURE(c, w.dal1, sizeof(int) * n);
    ENSURE(c, w.stamps, sizeof(unsigned) * STAMP_STRIDE * n);
    // frozen anchors: targets of up to 4 violations per vertex on average, then none freeze more
    const int64_t ftgt_cap = std::max<int64_t>(4 * (int64_t)n, 1 << 16);
    ENSURE(c, w.fofs, sizeof(int) * n);
    ENSURE(c, w.ftgt, sizeof(int) * (size_t)ftgt_cap);
    ENSURE(c, w.dreq, sizeof(unsigned) * n);
    ENSURE(c, w.frz, sizeof(int) * n);
    HIPCHK(c, hipMemsetAsync(w.dreq.p, 0, sizeof(unsigned) * n, st));
    HIPCHK(c, hipMemcpyAsync(w.g1.p, w.g0.p, sizeof(float) * n, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipMemsetAsync(w.stamps.p, 0, sizeof(unsigned) * STAMP_STRIDE * n, st));
    k_fr_init<<<1, 1, 0, st>>>(ctl);
    CHECK_LAUNCH(c);

    FrontierBufs& B = J.B;
    B = FrontierBufs{};
    B.ctl = ctl;
    B.dm = J.dm;
    B.ndim = D;
    B.f = J.f;
    B.gh = J.gh;
    B.lo = P<float>(w.lo);
    B.gb[0] = P<float>(w.g0);
    B.gb[1] = P<float>(w.g1);
    B.state = P<uint8_t>(w.state);
    B.fpl = P<uint8_t>(w.fpl);
    B.gpl = P<uint8_t>(w.gpl);
    B.vmask = P<uint32_t>(w.vmask);
    B.vl[0] = P<int>(w.vl0);
    B.vl[1] = P<int>(w.vl1);
    B.dvl[0] = P<int>(w.dvl0);
    B.dvl[1] = P<int>(w.dvl1);
    B.dal[0] = P<int>(w.dal0);
    B.dal[1] = P<int>(w.dal1);
    B.vstamp = P<unsigned>(w.stamps);
    B.astamp[0] = P<unsigned>(w.stamps) + 1;
    B.astamp[1] = P<unsigned>(w.stamps) + 2;
    B.rstamp = P<unsigned>(w.stamps) + 3;
    B.fofs = P<int>(w.fofs);
    B.ftgt = P<int>(w.ftgt);
    B.dreq = P<unsigned>(w.dreq);
    B.frz = P<int>(w.frz);
    B.ftgt_cap = (int)ftgt_cap;
    B.log = nullptr;
    if (w.msc.valid) {
        MscBufs& m = w.msc;
        B.dcell = P<int>(m.dcell); B.dcbr = P<int>(m.dcbr); B.dterm = P<int>(m.dterm);
        B.acell = P<int>(m.acell); B.acbr = P<int>(m.acbr); B.aterm = P<int>(m.aterm);
        B.doff = P<int64_t>(m.doff); B.aoff = P<int64_t>(m.aoff);
        B.dfirst = P<int>(m.dfirst); B.afirst = P<int>(m.afirst);
        B.n_dcell = m.n_desc_cells; B.n_acell = m.n_asc_cells;
        B.n_desc = (int)m.n_desc; B.n_asc = (int)m.n_asc;
        // first[] starts at "no difference" (iteration 0 scans every branch); the vertex ->
        // branch lists let later iterations rescan only the branches near their edits
        TRY(fill_i32(c, B.dfirst, B.n_desc, INF32, st));
        TRY(fill_i32(c, B.afirst, B.n_asc, INF32, st));
        const int64_t nbr = m.n_desc + m.n_asc;
        const int64_t ne = m.n_desc_cells + (int64_t)(D + 1) * m.n_asc_cells;
        if (ne >= (int64_t)INT32_MAX) return fail(c, DMT_E_INVALID, "too many separatrix cells");
        const int ntiles = (int)((n + 1023) / 1024);
        ENSURE(c, w.vpos, sizeof(int) * n);
        ENSURE(c, w.vstart, sizeof(int) * (n + 1));
        ENSURE(c, w.tsum, sizeof(int) * ntiles);
        ENSURE(c, w.toff, sizeof(int64_t) * (ntiles + 1));
        ENSURE(c, w.ecell, sizeof(int) * (size_t)ne);
        ENSURE(c, w.tcl, sizeof(int) * (size_t)ne);
        ENSURE(c, w.bstamp, sizeof(unsigned) * (size_t)nbr);
        ENSURE(c, w.dbl, sizeof(int) * (size_t)nbr);
        ENSURE(c, w.newmin, sizeof(unsigned long long) * (size_t)nbr);
        ENSURE(c, w.btgt, sizeof(int) * (size_t)nbr);
        ENSURE(c, w.cand0, sizeof(int) * (size_t)nbr);
        ENSURE(c, w.cand1, sizeof(int) * (size_t)nbr);
        ENSURE(c, w.inlist, (size_t)nbr);
        TRY(fill_i32(c, P<int>(w.newmin), 2 * nbr, -1, st));   // NEWMIN_NONE: all ones
        HIPCHK(c, hipMemsetAsync(w.vpos.p, 0, sizeof(int) * n, st));
        HIPCHK(c, hipMemsetAsync(w.bstamp.p, 0, sizeof(unsigned) * (size_t)nbr, st));
        // counting sort of the entries by vertex: counts, offsets, fill
        if (ne) {
            k_fr_branch_map<D><<<nblocks(ne), TPB, 0, st>>>(B, 0, P<int>(w.vpos), P<int>(w.ecell));
            CHECK_LAUNCH(c);
        }
        k_tile_sum<<<ntiles, TPB, 0, st>>>(P<int>(w.vpos), n, P<int>(w.tsum));
        CHECK_LAUNCH(c);
        TRY(scan(c, P<int>(w.tsum), ntiles, P<int64_t>(w.toff), nullptr, st));
        k_tile_scan<<<ntiles, TPB, 0, st>>>(P<int>(w.vpos), n, P<int64_t>(w.toff), P<int>(w.vstart));
        CHECK_LAUNCH(c);
        if (ne) {
            k_fr_branch_map<D><<<nblocks(ne), TPB, 0, st>>>(B, 1, P<int>(w.vpos), P<int>(w.ecell));
            CHECK_LAUNCH(c);
        }
        B.vstart = P<int>(w.vstart);
        B.ecell = P<int>(w.ecell);
        B.bstamp = P<unsigned>(w.bstamp);
        B.tcl = P<int>(w.tcl);
        B.dbl = P<int>(w.dbl);
        B.newmin = P<unsigned long long>(w.newmin);
        B.btgt = P<int>(w.btgt);
        B.cand[0] = P<int>(w.cand0);
        B.cand[1] = P<int>(w.cand1);
        B.inlist = P<uint8_t>(w.inlist);
    }
    bool ss = false;
    if (w.msc.valid) TRY(ss_setup<D>(c, J, ss, st));
    if (ss) {
        B.ss_src = P<int>(w.ss_src);
        B.n_ss_src = (int)(3 * w.msc.ncrit[2]);
        B.ss_q[0] = P<int>(w.ss_q0);
        B.ss_q[1] = P<int>(w.ss_q1);
        B.ss_stamp = P<unsigned>(w.ss_stamp);
        B.ss_on = 1;
    }
    B.delta = ldexpf(J.xi, -J.o.q_max);
    B.q_max = J.o.q_max;
    B.tier = J.o.tier;
    B.max_iters = J.o.max_iters < 0 ? INT64_MAX : J.o.max_iters;
    return DMT_OK;
}

// Iteration 0's dense gradient of g and violation pass, as full-grid launches.
template <int D>
dmt_status job_iteration0(dmt_context* c, Job& J, hipStream_t st) {
    const int n = J.dm.n;
    const unsigned gfull = nblocks(n) < 2048u ? nblocks(n) : 2048u;
    {
        ProfScope ps(c, DMT_PROF_GRADIENT, st, n);
        k_fr_grad<D><<<gfull, TPB, 0, st>>>(J.B, J.dm);
        CHECK_LAUNCH(c);
    }
    {
        ProfScope ps(c, DMT_PROF_CLASSIFY, st, n);
        k_fr_classify0<D><<<classify_blocks(n), TPB, 0, st>>>(J.B, J.dm);
        CHECK_LAUNCH(c);
    }
    // the requests (and edits) of iteration 0's violations
    ProfScope ps(c, DMT_PROF_APPLY, st, 0);
    k_fr_vr<D><<<gfull, TPB, 0, st>>>(J.B, J.dm);
    const int64_t nbr = (int64_t)J.B.n_desc + J.B.n_asc;
    if (nbr) k_fr_cand_init<D><<<nblocks((nbr + CAND_PER_THREAD - 1) / CAND_PER_THREAD), TPB, 0, st>>>(J.B, J.B.ctl);
    CHECK_LAUNCH(c);
    return DMT_OK;
}

// Grows the single-job log buffer to hold need records, keeping the first keep.
dmt_status grow_log(dmt_context* c, size_t need, int64_t keep, hipStream_t st) {
    const size_t rec = sizeof(long long) * DMT_LOG_WORDS;
    if (c->dlog.cap >= need * rec) return DMT_OK;
    DevBuf nb;
    if (c->arena_on) {
        TRY(arena_take(c, nb, need * 2 * rec));
    } else {
        if (hipMalloc(&nb.p, need * 2 * rec) != hipSuccess) {
            (void)hipGetLastError();
            return fail(c, DMT_E_NOMEM, "log allocation failed");
        }
        nb.cap = need * 2 * rec;
    }
    if (c->dlog.p && keep > 0)
        HIPCHK(c, hipMemcpyAsync(nb.p, c->dlog.p, (size_t)keep * rec, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (c->dlog.p && !c->arena_on) (void)hipFree(c->dlog.p);
    c->dlog = nb;
    return DMT_OK;
}

// K iterations of one job as full-grid launches (one per phase) from the start of iteration
// ctl->it (from its troublemaker pass when from_sstep), then the gradient, violation and branch
// passes of the next one: the state the resident loop starts from.  Launches of a finished job
// return at once.
template <int D>
dmt_status grid_iterations(dmt_context* c, const FrontierBufs& B, const Dims& dm, int K, bool from_sstep,
                           hipStream_t st) {
    const unsigned gfull = nblocks(dm.n) < 2048u ? nblocks(dm.n) : 2048u;
    const unsigned gcls = classify_blocks(dm.n, 2048u);
    if (from_sstep) {
        // paused before the troublemaker pass of iteration ctl->it: finish that iteration first
        k_fr_sapply<D><<<gfull, TPB, 0, st>>>(B, dm);
        if (B.ss_on) k_fr_ss<<<1, 1024, 0, st>>>(B, dm);
        k_fr_finish<<<1, 1, 0, st>>>(B);
    }
    for (int k = 0; k <= K; k++) {
        k_fr_grad<D><<<gfull, TPB, 0, st>>>(B, dm);
        k_fr_classify_dense<D><<<gcls, TPB, 0, st>>>(B, dm);
        k_fr_vr<D><<<gfull, TPB, 0, st>>>(B, dm);
        k_fr_bscan<D><<<gfull, TPB, 0, st>>>(B, dm);
        if (k == K) break;
        if (B.tier >= 3) k_fr_sapply<D><<<gfull, TPB, 0, st>>>(B, dm);
        if (B.ss_on) k_fr_ss<<<1, 1024, 0, st>>>(B, dm);
        k_fr_finish<<<1, 1, 0, st>>>(B);
    }
    CHECK_LAUNCH(c);
    return DMT_OK;
}

// The loops of the jobs in workgroup-resident form: one launch per dimension present, one
// workgroup per job at a time.  A single job may keep a log; its loop pauses when the log is
// full and is launched again after the log has grown.  Every launch ends after a bounded
// number of iterations.
dmt_status run_wg(dmt_context* c, std::vector<Job*>& jobs, bool with_log, hipStream_t st, int max_launches = -1,
                  int max_passes = 1 << 18) {
    const int nj = (int)jobs.size();
    int ncu = 0, occ2 = 0, occ3 = 0;
    HIPCHK(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device));
    const int nt2 = c->tune.loop_threads[0], nt3 = c->tune.loop_threads[1];
    const void* loop2 = nt2 == 512 ? reinterpret_cast<const void*>(k_fr_loop_wg<2, 512>)
                                   : reinterpret_cast<const void*>(k_fr_loop_wg<2, 1024>);
    const void* loop3 = nt3 == 256 ? reinterpret_cast<const void*>(k_fr_loop_wg<3, 256>)
                                   : reinterpret_cast<const void*>(k_fr_loop_wg<3, 512>);
    HIPCHK(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ2, loop2, nt2, 0));
    HIPCHK(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ3, loop3, nt3, 0));
    if (occ2 < 1 || occ3 < 1) return fail(c, DMT_E_HIP, "the loop kernel does not fit a compute unit");
    // jobs ordered 2D first, then 3D; hb[k] belongs to jobs[order[k]] and to control block
    // order[k] (control blocks follow the order of jobs)
    std::vector<int> order;
    for (int pass = 2; pass <= 3; pass++)
        for (int j = 0; j < nj; j++)
            if (jobs[j]->D == pass) order.push_back(j);
    const int n2 = (int)std::count_if(jobs.begin(), jobs.end(), [](const Job* J) { return J->D == 2; });
    ENSURE(c, c->jobs_dev, sizeof(FrontierBufs) * nj);
    ENSURE(c, c->queue, sizeof(int) * 2);
    std::vector<FrontierBufs> hb(nj);
    if (with_log) TRY(grow_log(c, 4096, 0, st));
    const int cap0 = with_log ? (int)(c->dlog.cap / (sizeof(long long) * DMT_LOG_WORDS)) : 0;
    // Every iteration that does not end a job edits at least one vertex, and a vertex takes at
    // most q_max + 1 edits (Section 4.5), so no job runs more than n (q_max + 1) + 1 iterations.
    int64_t bound = 0;
    for (int k = 0; k < nj; k++) {
        const Job* J = jobs[order[k]];
        hb[k] = J->B;
        hb[k].log = with_log ? P<long long>(c->dlog) : nullptr;
        hb[k].log_cap = cap0;
        const int64_t b = (int64_t)J->dm.n * (J->o.q_max + 1) + 1;
        bound = b > bound ? b : bound;
    }
    HIPCHK(c, hipMemcpyAsync(c->jobs_dev.p, hb.data(), sizeof(FrontierBufs) * nj, hipMemcpyHostToDevice, st));
    // iterations with more than `big` affected and listed anchors are handed to full-grid
    // launches (a workgroup takes about 1 us per 100 such anchors, the grid far less); the loop
    // kernel ends once every job has finished or paused, then the host runs a few iterations of
    // each paused job on the whole grid and launches the loop again
    // a paused job of a batch waits for every other workgroup to finish or pause before the
    // host can run its grid iterations, so batches hand off less often and hand over more
    // iterations at a time
    const int32_t* big = nj == 1 ? c->tune.handoff_anchors : c->tune.batch_handoff_anchors;
    const int big2 = big[0], big3 = big[1];
    std::vector<int> pos(nj);
    for (int k = 0; k < nj; k++) pos[order[k]] = k;
    const int grid_batch = c->tune.grid_iterations[nj == 1 ? 0 : 1];
    // a job that pauses again at once after a hand-off (its next iteration is large as well) gets
    // twice as many grid iterations at its next hand-off, up to GRID_RUN_MAX; one that ran
    // iterations in the workgroup in between starts again from grid_batch.  This saves the loop
    // relaunches and host round trips of long runs of large iterations.
    const int krun_max = std::max(grid_batch, GRID_RUN_MAX);
    int64_t progress = -1;
    for (int launch = 0; max_launches < 0 || launch < max_launches; launch++) {
        HIPCHK(c, hipMemsetAsync(c->queue.p, 0, sizeof(int) * 2, st));
        {
            ProfScope ps(c, DMT_PROF_LOOP, st, 0);
            const FrontierBufs* jd = P<FrontierBufs>(c->jobs_dev);
            // 3D jobs of a mixed batch run beside the 2D ones, on the context's second stream,
            // forked from st before either launch and joined back into st after both
            const bool mixed = n2 > 0 && nj > n2;
            hipStream_t s3 = st;
            if (mixed) {
                if (!c->side) {
                    HIPCHK(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
                    HIPCHK(c, hipEventCreateWithFlags(&c->fork, hipEventDisableTiming));
                    HIPCHK(c, hipEventCreateWithFlags(&c->join, hipEventDisableTiming));
                }
                HIPCHK(c, hipEventRecord(c->fork, st));
                HIPCHK(c, hipStreamWaitEvent(c->side, c->fork, 0));
                s3 = c->side;
            }
            if (n2) {
                const int blocks = n2 < ncu * occ2 ? n2 : ncu * occ2;
                if (nt2 == 512)
                    k_fr_loop_wg<2, 512><<<blocks, 512, 0, st>>>(jd, n2, P<int>(c->queue), max_passes, big2);
                else
                    k_fr_loop_wg<2, 1024><<<blocks, 1024, 0, st>>>(jd, n2, P<int>(c->queue), max_passes, big2);
                CHECK_LAUNCH(c);
            }
            if (nj > n2) {
                const int blocks = nj - n2 < ncu * occ3 ? nj - n2 : ncu * occ3;
                if (nt3 == 256)
                    k_fr_loop_wg<3, 256><<<blocks, 256, 0, s3>>>(jd + n2, nj - n2, P<int>(c->queue) + 1, max_passes,
                                                                 big3);
                else
                    k_fr_loop_wg<3, 512><<<blocks, 512, 0, s3>>>(jd + n2, nj - n2, P<int>(c->queue) + 1, max_passes,
                                                                 big3);
                CHECK_LAUNCH(c);
            }
            if (mixed) {
                HIPCHK(c, hipEventRecord(c->join, c->side));
                HIPCHK(c, hipStreamWaitEvent(st, c->join, 0));
            }
        }
        HIPCHK(c, hipMemcpyAsync(c->hctl.data(), c->ctl_all.p, sizeof(Ctl) * c->hctl.size(), hipMemcpyDeviceToHost,
                                 st));
        HIPCHK(c, hipStreamSynchronize(st));
        bool running = false, log_full = false;
        int64_t max_it = 0, sum_it = 0;
        for (int j = 0; j < nj; j++) {
            const Ctl& h = c->hctl[jobs[j]->slot];
            sum_it += h.it + (h.done != 0);
            if (h.done) continue;
            running = true;
            max_it = h.it > max_it ? h.it : max_it;
            if (with_log && h.it >= hb[0].log_cap) log_full = true;
        }
        if (!running) break;
        if (max_it > bound || sum_it == progress)
            return fail(c, DMT_E_HIP, "correction loop exceeded the iteration bound or stopped advancing");
        progress = sum_it;
        std::vector<int> paused;
        for (int j = 0; j < nj; j++)
            if (!c->hctl[jobs[j]->slot].done && c->hctl[jobs[j]->slot].paused) paused.push_back(j);
        // the paused jobs' grid iterations are independent (each touches its own workspace and
        // control block): up to HAND_STREAMS of them run at a time
        if (!paused.empty()) {
            ProfScope ps(c, DMT_PROF_LOOP, st, 0);
            const int ns = (int)std::min<size_t>(HAND_STREAMS, paused.size());
            if (ns > 1) {
                if (!c->fork) HIPCHK(c, hipEventCreateWithFlags(&c->fork, hipEventDisableTiming));
                for (int k = 0; k < ns; k++) {
                    if (!c->hand[k]) {
                        HIPCHK(c, hipStreamCreateWithFlags(&c->hand[k], hipStreamNonBlocking));
                        HIPCHK(c, hipEventCreateWithFlags(&c->hand_join[k], hipEventDisableTiming));
                    }
                }
            }
            for (int j : paused) {
                // a large iteration: reset the pause and make room in the log (on st, before the fork)
                Job* J = jobs[j];
                FrontierBufs& hj = hb[pos[j]];
                const Ctl& h = c->hctl[J->slot];
                const int64_t it0 = h.it;
                J->krun = it0 <= J->resume_it + 1 ? std::min(J->krun * 2, krun_max) : grid_batch;
                J->resume_it = it0 + J->krun + (h.paused == 2);
                if (with_log && it0 + J->krun + 2 > hj.log_cap) {
                    TRY(grow_log(c, (size_t)(it0 + J->krun) * 2 + 4096, it0, st));
                    hj.log = P<long long>(c->dlog);
                    hj.log_cap = (int)(c->dlog.cap / (sizeof(long long) * DMT_LOG_WORDS));
                    HIPCHK(c, hipMemcpyAsync(P<FrontierBufs>(c->jobs_dev) + pos[j], &hj, sizeof(FrontierBufs),
                                             hipMemcpyHostToDevice, st));
                }
                HIPCHK(c, hipMemsetAsync(&J->B.ctl->paused, 0, sizeof(int), st));
            }
            if (ns > 1) {
                HIPCHK(c, hipEventRecord(c->fork, st));
                for (int k = 0; k < ns; k++) HIPCHK(c, hipStreamWaitEvent(c->hand[k], c->fork, 0));
            }
            for (size_t i = 0; i < paused.size(); i++) {
                // a few iterations as full-grid launches
                const int j = paused[i];
                const Job* J = jobs[j];
                const bool from_sstep = c->hctl[J->slot].paused == 2;
                hipStream_t hs = ns > 1 ? c->hand[i % ns] : st;
                TRY(J->D == 2 ? grid_iterations<2>(c, hb[pos[j]], J->dm, J->krun, from_sstep, hs)
                              : grid_iterations<3>(c, hb[pos[j]], J->dm, J->krun, from_sstep, hs));
            }
            if (ns > 1) {
                for (int k = 0; k < ns; k++) {
                    HIPCHK(c, hipEventRecord(c->hand_join[k], c->hand[k]));
                    HIPCHK(c, hipStreamWaitEvent(st, c->hand_join[k], 0));
                }
            }
            continue;
        }
        if (!log_full) continue;
        // the log is full (a single job): grow it, point the job at it and resume
        const int64_t host_it = c->hctl[jobs[0]->slot].it;
        TRY(grow_log(c, (size_t)host_it * 2 + 4096, host_it, st));
        hb[0].log = P<long long>(c->dlog);
        hb[0].log_cap = (int)(c->dlog.cap / (sizeof(long long) * DMT_LOG_WORDS));
        HIPCHK(c, hipMemcpyAsync(c->jobs_dev.p, hb.data(), sizeof(FrontierBufs), hipMemcpyHostToDevice, st));
    }
    return DMT_OK;
}

// The frontier loop as one launch per phase (single job), host synchronisation once per batch.
template <int D>
dmt_status run_phases(dmt_context* c, Job& J, hipStream_t st) {
    const int n = J.dm.n;
    const unsigned gfull = nblocks(n) < 2048u ? nblocks(n) : 2048u;
    const unsigned gcls = classify_blocks(n, 2048u);
    int batch = 4;
    Ctl h{};
    // iteration 0 (dense passes), the first troublemaker candidates, and its decision
    TRY(grow_log(c, (size_t)batch + 2, 0, st));
    J.B.log = P<long long>(c->dlog);
    {
        ProfScope ps(c, DMT_PROF_LOOP, st, 0);
        k_fr_grad<D><<<gfull, TPB, 0, st>>>(J.B, J.dm);
        k_fr_classify0<D><<<classify_blocks(n), TPB, 0, st>>>(J.B, J.dm);
        k_fr_vr<D><<<gfull, TPB, 0, st>>>(J.B, J.dm);
        const int64_t nbr = (int64_t)J.B.n_desc + J.B.n_asc;
        if (nbr) k_fr_cand_init<D><<<nblocks((nbr + CAND_PER_THREAD - 1) / CAND_PER_THREAD), TPB, 0, st>>>(J.B, J.B.ctl);
        if (J.o.tier >= 3) k_fr_sapply<D><<<gfull, TPB, 0, st>>>(J.B, J.dm);
        if (J.B.ss_on) k_fr_ss<<<1, 1024, 0, st>>>(J.B, J.dm);
        k_fr_finish<<<1, 1, 0, st>>>(J.B);
        CHECK_LAUNCH(c);
    }
    int64_t host_it = 1;
    for (;;) {
        TRY(grow_log(c, (size_t)host_it + (size_t)batch + 1, host_it, st));
        J.B.log = P<long long>(c->dlog);
        for (int b = 0; b < batch; b++) {
            ProfScope ps(c, DMT_PROF_LOOP, st, 0);
            k_fr_grad<D><<<gfull, TPB, 0, st>>>(J.B, J.dm);
            k_fr_classify_dense<D><<<gcls, TPB, 0, st>>>(J.B, J.dm);
            k_fr_vr<D><<<gfull, TPB, 0, st>>>(J.B, J.dm);
            k_fr_bscan<D><<<gfull, TPB, 0, st>>>(J.B, J.dm);
            if (J.o.tier >= 3) k_fr_sapply<D><<<gfull, TPB, 0, st>>>(J.B, J.dm);
            if (J.B.ss_on) k_fr_ss<<<1, 1024, 0, st>>>(J.B, J.dm);
            k_fr_finish<<<1, 1, 0, st>>>(J.B);
            CHECK_LAUNCH(c);
        }
        HIPCHK(c, hipMemcpyAsync(&h, J.B.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        host_it = h.it;
        if (h.done) break;
        if (host_it > (int64_t)n * (J.o.q_max + 1) + 1)   // the bound of run_wg
            return fail(c, DMT_E_HIP, "phase loop exceeded the iteration bound");
        if (batch < 256) batch *= 2;
    }
    return DMT_OK;
}

// a8: g_out, q_out and statistics of a finished job; the field of the last iteration is in
// gb[it & 1].
dmt_status job_outputs(dmt_context* c, Job& J, const Ctl& ctl, bool lossless_list, hipStream_t st) {
    const int n = J.dm.n;
    const unsigned nb = nblocks(n);
    JobWs& w = *J.w;
    float* gfin = J.B.gb[ctl.it & 1];
    ENSURE(c, c->cnt, sizeof(unsigned long long) * CNT_WORDS);
    ENSURE(c, c->blk, sizeof(int) * (size_t)nb);
    ENSURE(c, c->blkoff, sizeof(int64_t) * (size_t)(nb + 1));
    unsigned long long* cnt = P<unsigned long long>(c->cnt);
    HIPCHK(c, hipMemcpyAsync(J.g_out, gfin, sizeof(float) * n, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipMemsetAsync(cnt, 0, sizeof(unsigned long long) * CNT_WORDS, st));
    k_qout<<<nb, TPB, 0, st>>>(P<uint8_t>(w.state), gfin, J.gh, J.q_out, n, P<int>(c->blk), cnt);
    CHECK_LAUNCH(c);
    if (lossless_list) {
        TRY(scan(c, P<int>(c->blk), nb, P<int64_t>(c->blkoff), &c->n_lossless, st));
        ENSURE(c, c->ll_idx, sizeof(int64_t) * (size_t)c->n_lossless);
        ENSURE(c, c->ll_val, sizeof(float) * (size_t)c->n_lossless);
        k_lossless_write<<<nb, TPB, 0, st>>>(J.q_out, gfin, n, P<int64_t>(c->blkoff), P<int64_t>(c->ll_idx),
                                             P<float>(c->ll_val));
        CHECK_LAUNCH(c);
    }
    TRY(read_counters(c, st));
    dmt_stats& S = J.stats;
    S.iterations = ctl.it;
    S.c_iterations = ctl.c_it;
    S.s_iterations = ctl.s_it;
    S.n_edited = (int64_t)c->hcnt[CNT_EDITED];
    S.n_quantized = (int64_t)c->hcnt[CNT_QUANT];
    S.n_lossless = (int64_t)c->hcnt[CNT_LOSSLESS];
    S.residual_violations = ctl.done == 1 ? 0 : ctl.residual;
    S.converged = ctl.done == 1;
    S.stalled = ctl.done == 3;
    J.status = ctl.done == 1 ? DMT_OK : DMT_W_NOT_CONVERGED;
    return DMT_OK;
}

// ---- dense reference loop (DMT_F_DENSE): whole gradient and every anchor each iteration ------

template <int D>
dmt_status dense_loop(dmt_context* c, Job& J, Ctl& out, hipStream_t st) {
    const Dims& dm = J.dm;
    const int n = dm.n;
    const unsigned nb = nblocks(n);
    JobWs& w = *J.w;
    const float delta = ldexpf(J.xi, -J.o.q_max);
    const int tier = J.o.tier;
    ENSURE(c, c->cnt, sizeof(unsigned long long) * CNT_WORDS);
    unsigned long long* cnt = P<unsigned long long>(c->cnt);
    float* lo = P<float>(w.lo);
    float* g = P<float>(w.g0);
    uint8_t* state = P<uint8_t>(w.state);
    uint8_t* req = P<uint8_t>(c->req);
    uint8_t* fpl = P<uint8_t>(w.fpl);
    uint8_t* gpl = P<uint8_t>(w.gpl);
    MscBufs& m = w.msc;
    m.valid = false;
    if (tier >= 3) TRY(build_msc<D>(c, m, fpl, dm, false, st));
    bool ss = false;
    if (tier >= 3) TRY(ss_setup<D>(c, J, ss, st));
    c->log.clear();
    int64_t it = 0, c_it = 0, s_it = 0, residual = 0;
    int done = 0;
    const int64_t max_iters = J.o.max_iters < 0 ? INT64_MAX : J.o.max_iters;
    for (;;) {
        TRY(launch_grad(c, D, g, gpl, dm, st));
        HIPCHK(c, hipMemsetAsync(cnt, 0, sizeof(unsigned long long) * CNT_WORDS, st));
        k_classify<D><<<nb, TPB, 0, st>>>(fpl, gpl, J.f, g, req, dm, tier, cnt);
        CHECK_LAUNCH(c);
        TRY(read_counters(c, st));
        int64_t viol = 0;
        for (int k = CNT_FP0; k < CNT_FP0 + 8; k++) viol += (int64_t)c->hcnt[k];
        int kind = 1;
        if (viol == 0 && tier >= 3) {
            kind = 2;
            if (m.n_desc_cells) {
                k_scheck_desc<D><<<nblocks(m.n_desc_cells), TPB, 0, st>>>(fpl, gpl, P<int>(m.dcell), P<int>(m.dcbr),
                                                                       m.n_desc_cells, P<int>(m.dfirst));
                k_starget<D><<<nblocks(m.n_desc), TPB, 0, st>>>(fpl, gpl, dm, 0, P<int>(m.dcell), P<int64_t>(m.doff),
                                                                P<int>(m.dterm), (int)m.n_desc, P<int>(m.dfirst), tier,
                                                                req, cnt);
                CHECK_LAUNCH(c);
            }
            if (m.n_asc_cells) {
                k_scheck_asc<D><<<nblocks(m.n_asc_cells), TPB, 0, st>>>(fpl, gpl, dm, P<int>(m.acell), P<int>(m.acbr),
                                                                        m.n_asc_cells, P<int>(m.afirst));
                k_starget<D><<<nblocks(m.n_asc), TPB, 0, st>>>(fpl, gpl, dm, 1, P<int>(m.acell), P<int64_t>(m.aoff),
                                                               P<int>(m.aterm), (int)m.n_asc, P<int>(m.afirst), tier,
                                                               req, cnt);
                CHECK_LAUNCH(c);
            }
            if (ss)
                k_ss_dense<<<1, 1024, 0, st>>>(fpl, gpl, dm, P<int>(w.ss_src), (int)(3 * m.ncrit[2]), P<int>(w.ss_q0),
                                               P<int>(w.ss_q1), P<unsigned>(w.ss_stamp), (unsigned)it + 1u, req, cnt);
            CHECK_LAUNCH(c);
            TRY(read_counters(c, st));
            viol = (int64_t)(c->hcnt[CNT_TM_DESC] + c->hcnt[CNT_TM_ASC] + c->hcnt[CNT_TM_SS]);
        }
        if (viol == 0) { done = 1; break; }
        if (it == max_iters) {
            residual = viol;
            done = 2;
            k_clear_u8<<<nb, TPB, 0, st>>>(req, n);
            CHECK_LAUNCH(c);
            break;
        }
        k_apply<<<nb, TPB, 0, st>>>(req, J.gh, lo, g, state, delta, J.o.q_max, n, cnt);
        CHECK_LAUNCH(c);
        TRY(read_counters(c, st));
        if (c->hcnt[CNT_CHANGED] == 0) { done = 3; residual = viol; break; }
        int64_t rec[DMT_LOG_WORDS] = {0};
        rec[0] = kind;
        for (int k = 1; k <= CNT_CHANGED; k++) rec[k] = (int64_t)c->hcnt[k];
        rec[20] = (int64_t)c->hcnt[CNT_TM_SS];
        c->log.insert(c->log.end(), rec, rec + DMT_LOG_WORDS);
        it++;
        if (kind == 1) c_it++; else s_it++;
    }
    out = Ctl{};
    out.it = (int)it;
    out.done = done;
    out.c_it = (int)c_it;
    out.s_it = (int)s_it;
    out.residual = residual;
    J.B.gb[0] = g;   // the single buffer of this form, whatever the parity of it
    J.B.gb[1] = g;
    return DMT_OK;
}

// ---- driver shared by dmt_correct and dmt_correct_batch -------------------------------------

// Runs validated jobs.  single: one job; keeps the log and the lossless list in the context
// and honours the DENSE / PHASES flags.
dmt_status run_jobs(dmt_context* c, std::vector<Job>& jobs, bool single, hipStream_t st) {
    const int nj = (int)jobs.size();
    if ((int)c->ws.size() < nj) c->ws.resize(nj);
    ENSURE(c, c->flags, sizeof(unsigned) * (nj + 1));
    HIPCHK(c, hipMemsetAsync(c->flags.p, 0, sizeof(unsigned) * (nj + 1), st));
    // a0, a1 for every job, then one look at the validation flags
    for (int j = 0; j < nj; j++) {
        jobs[j].w = &c->ws[j];
        TRY(jobs[j].D == 2 ? job_setup<2>(c, jobs[j], P<unsigned>(c->flags) + 1 + j, st)
                           : job_setup<3>(c, jobs[j], P<unsigned>(c->flags) + 1 + j, st));
    }
    std::vector<unsigned> fl(nj + 1);
    HIPCHK(c, hipMemcpyAsync(fl.data(), c->flags.p, sizeof(unsigned) * (nj + 1), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    std::vector<Job*> live;
    for (int j = 0; j < nj; j++) {
        const unsigned f = fl[1 + j];
        if (f & 1u) { jobs[j].status = DMT_E_NONFINITE; continue; }
        if (f & 2u) { jobs[j].status = DMT_E_BOUND; continue; }
        live.push_back(&jobs[j]);
    }
    if (live.empty()) return DMT_OK;
    c->hctl.assign(live.size(), Ctl{});
    if (single && (jobs[0].o.flags & DMT_F_DENSE)) {
        Job& J = jobs[0];
        TRY(J.D == 2 ? dense_loop<2>(c, J, c->hctl[0], st) : dense_loop<3>(c, J, c->hctl[0], st));
        return job_outputs(c, J, c->hctl[0], true, st);
    }
    // a2 and frontier state for every live job (control blocks side by side), then the loop
    ENSURE(c, c->ctl_all, sizeof(Ctl) * live.size());
    for (size_t k = 0; k < live.size(); k++) {
        live[k]->slot = (int)k;
        Ctl* ctl = P<Ctl>(c->ctl_all) + k;
        TRY(live[k]->D == 2 ? job_frontier<2>(c, *live[k], ctl, st) : job_frontier<3>(c, *live[k], ctl, st));
    }
    if (single && (jobs[0].o.flags & DMT_F_PHASES)) {
        Job& J = jobs[0];
        TRY(J.D == 2 ? run_phases<2>(c, J, st) : run_phases<3>(c, J, st));
    } else {
        for (Job* J : live) TRY(J->D == 2 ? job_iteration0<2>(c, *J, st) : job_iteration0<3>(c, *J, st));
        TRY(run_wg(c, live, single, st));
    }
    HIPCHK(c, hipMemcpyAsync(c->hctl.data(), c->ctl_all.p, sizeof(Ctl) * live.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    for (int k = 0; k < 3; k++) c->ph[k] = 0;
    for (const Ctl& h : c->hctl)
        for (int k = 0; k < 3; k++) c->ph[k] += h.ph[k];
    for (size_t k = 0; k < live.size(); k++) TRY(job_outputs(c, *live[k], c->hctl[k], single, st));
    if (single) {
        const int64_t nrec = c->hctl[0].it;
        c->log.assign((size_t)nrec * DMT_LOG_WORDS, 0);
        if (nrec > 0)
            HIPCHK(c, hipMemcpy(c->log.data(), c->dlog.p, sizeof(long long) * DMT_LOG_WORDS * (size_t)nrec,
                                hipMemcpyDeviceToHost));
    }
    return DMT_OK;
}

}  // namespace

// ==========================================================================================
// C ABI


// ==========================================================================================
// Served form: a worker thread owns a context and a stream; jobs are admitted while their
// estimated workspace fits the HBM budget, set up, and then advance together in rounds of one
// loop launch (at most ROUND_PASSES iterations per job), so jobs submitted later join the next
// round and finished ones leave after it (continuous batching).

namespace {

constexpr int ROUND_PASSES = 512;
constexpr int SERVER_LANES = 4;   // worker lanes of a server (streams whose jobs overlap on the device)

int64_t workspace_estimate(int D, int64_t n, const dmt_options* o = nullptr) {
    // fields, state, f and g planes, frontier lists and stamps, separatrix branches (an upper
    // estimate of what the correction of one field allocates; the branches are data-dependent),
    // and the saddle-saddle walk's two level queues and edge stamps (7 edges per vertex, 4 B each)
    int64_t est = (D == 2 ? 144 : 264) * n + (1 << 20);
    if (o && D == 3 && o->tier == 4 && (o->flags & DMT_F_SADDLE_SADDLE)) est += 84 * n;
    return est;
}

// Device bytes a workspace holds now.
int64_t held_bytes(JobWs& w) {
    int64_t s = 0;
    for (DevBuf* b : w.all()) s += (int64_t)b->cap;
    return s;
}

void release(JobWs& w) {
    for (DevBuf* b : w.all()) {
        if (b->p) (void)hipFree(b->p);
        *b = DevBuf{};
    }
    w.msc.valid = false;
}

struct Ticket {
    dmt_job job{};
    Job J;
    int64_t bytes = 0;
    int lane = -1;
    int state = 0;          // 0 pending, 1 active, 2 done
};

// One lane of the server: a worker thread with its own context (workspaces for its slots) and
// stream.  Lanes run side by side, so a job admitted by an idle lane starts while other lanes'
// jobs are on the device.
struct Lane {
    dmt_context* c = nullptr;
    hipStream_t st = nullptr;
    std::thread worker;
    std::vector<int> free_slots;
    // HBM accounting: charge[slot] = bytes the slot is counted for (an active job: the larger of
    // its estimate and what its workspace holds; an idle slot: what its workspace still holds)
    std::vector<int64_t> charge;
    std::vector<int64_t> held;      // bytes each slot's workspace held when last accounted
    int64_t shared = 0;             // the lane context's shared buffers
    bool busy = false;              // holds admitted or active jobs
};

}  // namespace

struct dmt_server {
    std::vector<Lane> lanes;
    int64_t budget = 0;
    int max_jobs = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    std::unordered_map<int64_t, Ticket> tickets;
    std::deque<int64_t> pending;
    int64_t next_ticket = 1;
    uint64_t epoch = 0;             // bumped when a job is submitted or finishes
    int jobs_in_flight = 0;
    int idle_lanes = 0;
    int64_t inflight = 0;           // sum over lanes of their charges and shared buffers
    int64_t fail_outputs_at = -1;   // fault injection for tests: the k-th finished job's outputs fail
    std::atomic<int64_t> finished{0};
};

namespace {

int64_t shared_bytes(dmt_context* c) {
    int64_t s = 0;
    for (DevBuf* b : {&c->gpl, &c->req, &c->cnt, &c->flags, &c->part, &c->blk, &c->blkoff, &c->ll_idx, &c->ll_val,
                      &c->dlog, &c->jobs_dev, &c->ctl_all, &c->queue, &c->scan_tsum, &c->scan_toff})
        s += (int64_t)b->cap;
    return s;
}

// Recomputes inflight from every lane's charges (caller holds s->mu).
void recount(dmt_server* s) {
    int64_t t = 0;
    for (const Lane& L : s->lanes) {
        t += L.shared;
        for (int64_t b : L.charge) t += b;
    }
    s->inflight = t;
}

// Ends a ticket that is no longer in any worker list.  The slot keeps its workspace for the next
// job; its charge drops to what the workspace holds.
void server_finish(dmt_server* s, Lane& L, Ticket& t, dmt_status status) {
    const int64_t held = held_bytes(L.c->ws[t.J.slot]);
    const int64_t shared = shared_bytes(L.c);
    std::lock_guard<std::mutex> lk(s->mu);
    t.job.status = status;
    t.job.stats = t.J.stats;
    t.state = 2;
    L.charge[t.J.slot] = held;
    L.held[t.J.slot] = held;
    L.shared = shared;
    recount(s);
    L.free_slots.push_back(t.J.slot);
    s->jobs_in_flight--;
    s->epoch++;
    s->cv_done.notify_all();
    s->cv_work.notify_all();
}

// Setup, f's gradient and branches, frontier state and iteration 0 of newly admitted jobs.  Each
// ticket leaves `admit` when it is finished (validation failure) or moved to `active`; on an
// error the tickets still in `admit` have not been finished.
dmt_status server_admit(dmt_server* s, Lane& L, std::vector<Ticket*>& admit, std::vector<Ticket*>& active) {
    dmt_context* c = L.c;
    const hipStream_t st = L.st;
    const int nslots = (int)L.charge.size();
    HIPCHK(c, hipMemsetAsync(c->flags.p, 0, sizeof(unsigned) * (nslots + 1), st));
    for (Ticket* t : admit) {
        Job& J = t->J;
        J.w = &c->ws[J.slot];
        unsigned* flag = P<unsigned>(c->flags) + 1 + J.slot;
        TRY(J.D == 2 ? job_setup<2>(c, J, flag, st) : job_setup<3>(c, J, flag, st));
    }
    std::vector<unsigned> fl(nslots + 1);
    HIPCHK(c, hipMemcpyAsync(fl.data(), c->flags.p, sizeof(unsigned) * fl.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    while (!admit.empty()) {
        Ticket* t = admit.front();
        Job& J = t->J;
        const unsigned f = fl[1 + J.slot];
        if (f & 3u) {
            admit.erase(admit.begin());
            server_finish(s, L, *t, (f & 1u) ? DMT_E_NONFINITE : DMT_E_BOUND);
            continue;
        }
        Ctl* ctl = P<Ctl>(c->ctl_all) + J.slot;
        TRY(J.D == 2 ? job_frontier<2>(c, J, ctl, st) : job_frontier<3>(c, J, ctl, st));
        TRY(J.D == 2 ? job_iteration0<2>(c, J, st) : job_iteration0<3>(c, J, st));
        admit.erase(admit.begin());
        active.push_back(t);
        // the separatrix buffers are data-dependent: charge what the job holds once they exist
        const int64_t held = held_bytes(c->ws[J.slot]);
        const int64_t shared = shared_bytes(c);
        std::lock_guard<std::mutex> lk(s->mu);
        L.charge[J.slot] = std::max(t->bytes, held);
        L.held[J.slot] = held;
        L.shared = shared;
        recount(s);
    }
    return DMT_OK;
}

// One round of the lane's active jobs; finished ones get their outputs and leave `active` before
// they are handed back.
dmt_status server_round(dmt_server* s, Lane& L, std::vector<Ticket*>& active) {
    dmt_context* c = L.c;
    std::vector<Job*> js;
    for (Ticket* t : active) js.push_back(&t->J);
    TRY(run_wg(c, js, false, L.st, 1, ROUND_PASSES));
    for (size_t i = 0; i < active.size();) {
        Ticket* t = active[i];
        const Ctl h = c->hctl[t->J.slot];
        if (!h.done) {
            i++;
            continue;
        }
        active.erase(active.begin() + (long)i);
        dmt_status rc = DMT_OK;
        if (s->fail_outputs_at >= 0 && s->finished.fetch_add(1) == s->fail_outputs_at)
            rc = fail(c, DMT_E_NOMEM, "injected output failure");
        else
            rc = job_outputs(c, t->J, h, false, L.st);
        server_finish(s, L, *t, rc == DMT_OK ? t->J.status : rc);
        if (rc != DMT_OK) return rc;
    }
    return DMT_OK;
}

// Admission by footprint (caller holds s->mu): the job at the head of the queue is admitted to a
// free slot of lane L if the accounted bytes of all lanes stay within the budget, after releasing
// the workspaces of L's idle slots if that is what it takes; a job always fits an idle server.
bool server_try_admit(dmt_server* s, Lane& L, Ticket& t) {
    if (L.free_slots.empty()) return false;
    const bool idle = s->jobs_in_flight == 0;
    // prefer the idle slot holding the most memory already (its buffers are reused)
    int best = -1;
    for (size_t k = 0; k < L.free_slots.size(); k++)
        if (best < 0 || L.charge[L.free_slots[k]] > L.charge[L.free_slots[best]]) best = (int)k;
    const int slot = L.free_slots[best];
    auto need = [&] { return s->inflight - L.charge[slot] + std::max(t.bytes, L.charge[slot]); };
    if (need() > s->budget) {
        // give back what the lane's other idle slots hold (this lane's worker owns them)
        for (int k : L.free_slots) {
            if (k == slot || L.charge[k] == 0) continue;
            release(L.c->ws[k]);
            L.charge[k] = 0;
            L.held[k] = 0;
        }
        recount(s);
    }
    if (need() > s->budget && !idle) return false;
    L.free_slots.erase(L.free_slots.begin() + best);
    t.J.slot = slot;
    L.charge[slot] = std::max(t.bytes, L.charge[slot]);
    recount(s);
    t.state = 1;
    s->jobs_in_flight++;
    return true;
}

void server_main(dmt_server* s, int li) {
    Lane& L = s->lanes[li];
    (void)hipSetDevice(L.c->device);
    std::vector<Ticket*> active;
    uint64_t seen = ~0ull;   // epoch of an idle lane's last admission attempt that took nothing
    for (;;) {
        std::vector<Ticket*> admit;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (active.empty()) {
                s->cv_work.wait(lk, [&] {
                    return (s->stop && s->pending.empty()) || (!s->pending.empty() && s->epoch != seen);
                });
                if (s->pending.empty()) break;   // stopping, nothing left
            }
            // idle lanes take new jobs first; a busy lane admits more only when every lane is busy
            if (active.empty() || s->idle_lanes == 0) {
                while (!s->pending.empty()) {
                    Ticket& t = s->tickets.at(s->pending.front());
                    if (!server_try_admit(s, L, t)) break;
                    t.lane = li;
                    admit.push_back(&t);
                    s->pending.pop_front();
                }
            }
            if (active.empty() && admit.empty()) {
                seen = s->epoch;
                continue;
            }
            if (!L.busy) {
                L.busy = true;
                s->idle_lanes--;
            }
        }
        dmt_status rc = DMT_OK;
        if (!admit.empty()) rc = server_admit(s, L, admit, active);
        if (rc == DMT_OK && !active.empty()) rc = server_round(s, L, active);
        if (rc != DMT_OK) {
            // a failure ends every job still held by this lane with that status
            for (Ticket* t : active) server_finish(s, L, *t, rc);
            for (Ticket* t : admit) server_finish(s, L, *t, rc);
            active.clear();
        }
        if (active.empty()) {
            std::lock_guard<std::mutex> lk(s->mu);
            L.busy = false;
            s->idle_lanes++;
            seen = ~0ull;
        }
    }
}

}  // namespace

extern "C" {

dmt_status dmt_context_create(dmt_context** ctx, int hip_device) {
    if (!ctx) return DMT_E_INVALID;
    *ctx = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) {
        (void)hipGetLastError();
        return DMT_E_INVALID;
    }
    if (hipSetDevice(hip_device) != hipSuccess) return DMT_E_HIP;
    dmt_context* c = new dmt_context();
    c->device = hip_device;
    c->scratch = scratch_address(hip_device, ndev, c->scratch_err);
    if (hipHostMalloc((void**)&c->hcnt, sizeof(unsigned long long) * CNT_WORDS, 0) != hipSuccess ||
        hipHostMalloc((void**)&c->hscratch, sizeof(int64_t) * 64, 0) != hipSuccess) {
        delete c;
        return DMT_E_NOMEM;
    }
    *ctx = c;
    return DMT_OK;
}

dmt_status dmt_context_destroy(dmt_context* c) {
    if (!c) return DMT_OK;
    (void)hipSetDevice(c->device);
    std::vector<DevBuf*> bufs = context_bufs(c);
    for (DevBuf* b : c->msc.all()) bufs.push_back(b);
    for (MscBufs& m : c->cmp)
        for (DevBuf* b : m.all()) bufs.push_back(b);
    bufs.push_back(&c->gpl2);
    bufs.push_back(&c->agree);
    for (JobWs& w : c->ws)
        for (DevBuf* b : w.all()) bufs.push_back(b);
    for (DevBuf* b : bufs)
        if (b->p) (void)hipFree(b->p);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->fork) (void)hipEventDestroy(c->fork);
    if (c->join) (void)hipEventDestroy(c->join);
    if (c->side) (void)hipStreamDestroy(c->side);
    for (int k = 0; k < HAND_STREAMS; k++) {
        if (c->hand_join[k]) (void)hipEventDestroy(c->hand_join[k]);
        if (c->hand[k]) (void)hipStreamDestroy(c->hand[k]);
    }
    if (c->hcnt) (void)hipHostFree(c->hcnt);
    if (c->hscratch) (void)hipHostFree(c->hscratch);
    delete c;
    return DMT_OK;
}

const char* dmt_last_error(const dmt_context* c) { return c ? c->err.c_str() : "no context"; }

dmt_status dmt_cell_id_space(const dmt_grid* gr, int64_t counts[4]) {
    Dims dm;
    int D;
    if (!counts) return DMT_E_INVALID;
    dmt_status s = check_grid(nullptr, gr, dm, D);
    if (s != DMT_OK) return s;
    for (int d = 0; d < 4; d++) counts[d] = d <= D ? (int64_t)dm.n * ntypes(D, d) : 0;
    return DMT_OK;
}

dmt_status dmt_xi_from_relative(dmt_context* c, const dmt_grid* gr, const float* f, double rel, float* xi_host,
                                hipStream_t st) {
    if (!c || !f || !xi_host) return fail(c, DMT_E_INVALID, "null argument");
    Dims dm;
    int D;
    TRY(check_grid(c, gr, dm, D));
    if (!(rel > 0.0) || !std::isfinite(rel)) return fail(c, DMT_E_INVALID, "rel must be finite and > 0");
    HIPCHK(c, hipSetDevice(c->device));
    const int nbk = 512;
    ENSURE(c, c->part, sizeof(float) * 3 * nbk);
    ENSURE(c, c->flags, 16);
    k_minmax<<<nbk, TPB, 0, st>>>(f, dm.n, P<float>(c->part));
    k_minmax_final<<<1, TPB, 0, st>>>(P<float>(c->part), nbk, P<float>(c->flags));
    CHECK_LAUNCH(c);
    HIPCHK(c, hipMemcpyAsync(c->hscratch, c->flags.p, 3 * sizeof(float), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    const float* h = reinterpret_cast<const float*>(c->hscratch);
    const float mn = h[0], mx = h[1];
    if (h[2] != 0.0f) return fail(c, DMT_E_NONFINITE, "non-finite value in f");
    *xi_host = (float)(rel * ((double)mx - (double)mn));
    return DMT_OK;
}

dmt_status dmt_bounds(dmt_context* c, const float* f, int64_t n, float xi, float* lo, float* hi, hipStream_t st) {
    if (!c || !f || !lo || !hi || n < 0) return fail(c, DMT_E_INVALID, "bad argument");
    if (!(xi >= 0.0f) || !std::isfinite(xi)) return fail(c, DMT_E_INVALID, "xi must be finite and >= 0");
    if (n == 0) return DMT_OK;
    HIPCHK(c, hipSetDevice(c->device));
    k_bounds<<<nblocks(n), TPB, 0, st>>>(f, xi, n, lo, hi);
    CHECK_LAUNCH(c);
    return DMT_OK;
}

dmt_status dmt_gradient_pairs(dmt_context* c, const dmt_grid* gr, const float* field, int64_t* up, int64_t* down,
                              hipStream_t st) {
    if (!c || !field || !up || !down) return fail(c, DMT_E_INVALID, "null argument");
    Dims dm;
    int D;
    TRY(check_grid(c, gr, dm, D));
    HIPCHK(c, hipSetDevice(c->device));
    ENSURE(c, c->gpl, (size_t)plane_bytes(D) * dm.n);
    TRY(launch_grad(c, D, field, P<uint8_t>(c->gpl), dm, st));
    const int64_t o1 = dm.n, o2 = o1 + (int64_t)dm.n * ntypes(D, 1), o3 = o2 + (int64_t)dm.n * ntypes(D, 2);
    if (D == 2) k_export<2><<<nblocks(dm.n), TPB, 0, st>>>(P<uint8_t>(c->gpl), dm, o1, o2, o3, up, down);
    else k_export<3><<<nblocks(dm.n), TPB, 0, st>>>(P<uint8_t>(c->gpl), dm, o1, o2, o3, up, down);
    CHECK_LAUNCH(c);
    HIPCHK(c, hipStreamSynchronize(st));
    return DMT_OK;
}

dmt_status dmt_extract_msc(dmt_context* c, const dmt_grid* gr, const float* field, int64_t counts[32],
                           hipStream_t st) {
    if (!c || !field || !counts) return fail(c, DMT_E_INVALID, "null argument");
    Dims dm;
    int D;
    TRY(check_grid(c, gr, dm, D));
    HIPCHK(c, hipSetDevice(c->device));
    ENSURE(c, c->gpl, (size_t)plane_bytes(D) * dm.n);
    TRY(launch_grad(c, D, field, P<uint8_t>(c->gpl), dm, st));
    MscBufs& m = c->msc;
    TRY(D == 2 ? build_msc<2>(c, m, P<uint8_t>(c->gpl), dm, true, st)
               : build_msc<3>(c, m, P<uint8_t>(c->gpl), dm, true, st));
    HIPCHK(c, hipStreamSynchronize(st));
    for (int k = 0; k < 32; k++) counts[k] = 0;
    for (int d = 0; d < 4; d++) counts[DMT_MSC_CRIT0 + d] = m.ncrit[d];
    counts[DMT_MSC_DESC_SADDLE] = m.n_desc;
    counts[DMT_MSC_DESC_OFFSETS] = m.n_desc + 1;
    counts[DMT_MSC_DESC_CELLS] = m.n_desc_cells;
    counts[DMT_MSC_DESC_TERMINAL] = m.n_desc;
    counts[DMT_MSC_ASC_SADDLE] = m.n_asc;
    counts[DMT_MSC_ASC_OFFSETS] = m.n_asc + 1;
    counts[DMT_MSC_ASC_CELLS] = m.n_asc_cells;
    counts[DMT_MSC_ASC_TERMINAL] = m.n_asc;
    counts[DMT_MSC_MIN_LABEL] = m.n_vlab;
    counts[DMT_MSC_MAX_LABEL] = m.n_tlab;
    return DMT_OK;
}

dmt_status dmt_compare_msc(dmt_context* c, const dmt_grid* gr, const float* f, const float* g,
                           dmt_msc_agreement* out, hipStream_t st) {
    if (!c || !f || !g || !out) return fail(c, DMT_E_INVALID, "null argument");
    Dims dm;
    int D;
    TRY(check_grid(c, gr, dm, D));
    HIPCHK(c, hipSetDevice(c->device));
    const size_t planes = (size_t)plane_bytes(D) * dm.n;
    ENSURE(c, c->gpl, planes);
    ENSURE(c, c->gpl2, planes);
    TRY(launch_grad(c, D, f, P<uint8_t>(c->gpl), dm, st));
    TRY(launch_grad(c, D, g, P<uint8_t>(c->gpl2), dm, st));
    MscBufs& mf = c->cmp[0];
    MscBufs& mg = c->cmp[1];
    TRY(D == 2 ? build_msc<2>(c, mf, P<uint8_t>(c->gpl), dm, false, st)
               : build_msc<3>(c, mf, P<uint8_t>(c->gpl), dm, false, st));
    TRY(D == 2 ? build_msc<2>(c, mg, P<uint8_t>(c->gpl2), dm, false, st)
               : build_msc<3>(c, mg, P<uint8_t>(c->gpl2), dm, false, st));
    constexpr int NW = 8;   // counters: common critical cells by dimension, then (ends, cells) per family
    ENSURE(c, c->agree, sizeof(unsigned long long) * NW);
    unsigned long long* cnt = P<unsigned long long>(c->agree);
    HIPCHK(c, hipMemsetAsync(cnt, 0, sizeof(unsigned long long) * NW, st));
    for (int d = 0; d <= D; d++)
        if (mf.ncrit[d] && mg.ncrit[d]) {
            k_count_common<<<nblocks(mf.ncrit[d]), TPB, 0, st>>>(P<int>(mf.crit[d]), mf.ncrit[d], P<int>(mg.crit[d]),
                                                                 mg.ncrit[d], cnt + d);
            CHECK_LAUNCH(c);
        }
    auto desc = [](MscBufs& m) {
        return BranchList{nullptr, P<int>(m.crit[1]), P<int64_t>(m.doff), P<int>(m.dcell), P<int>(m.dterm), m.n_desc};
    };
    auto asc = [](MscBufs& m) {
        return BranchList{P<int>(m.asad), nullptr, P<int64_t>(m.aoff), P<int>(m.acell), P<int>(m.aterm), m.n_asc};
    };
    if (mf.n_desc && mg.n_desc) {
        k_branch_agree<<<nblocks(mf.n_desc * 64), TPB, 0, st>>>(desc(mf), desc(mg), cnt + 4);
        CHECK_LAUNCH(c);
    }
    if (mf.n_asc && mg.n_asc) {
        k_branch_agree<<<nblocks(mf.n_asc * 64), TPB, 0, st>>>(asc(mf), asc(mg), cnt + 6);
        CHECK_LAUNCH(c);
    }
    HIPCHK(c, hipMemcpyAsync(c->hscratch, cnt, sizeof(unsigned long long) * NW, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    const int64_t* h = c->hscratch;
    *out = dmt_msc_agreement{};
    for (int d = 0; d < 4; d++) {
        out->crit_f[d] = mf.ncrit[d];
        out->crit_g[d] = mg.ncrit[d];
        out->crit_common[d] = d <= D ? h[d] : 0;
    }
    out->sep_f[0] = mf.n_desc; out->sep_g[0] = mg.n_desc;
    out->sep_f[1] = mf.n_asc;  out->sep_g[1] = mg.n_asc;
    out->sep_same_ends[0] = h[4]; out->sep_same_cells[0] = h[5];
    out->sep_same_ends[1] = h[6]; out->sep_same_cells[1] = h[7];
    return DMT_OK;
}

dmt_status dmt_msc_copy(dmt_context* c, int item, int64_t* dst, int64_t cap, hipStream_t st) {
    if (!c || !dst) return fail(c, DMT_E_INVALID, "null argument");
    MscBufs& m = c->msc;
    if (!m.valid) return fail(c, DMT_E_INVALID, "no MSC extracted");
    HIPCHK(c, hipSetDevice(c->device));
    const int* src32 = nullptr;
    const int64_t* src64 = nullptr;
    int64_t n = 0;
    switch (item) {
    case DMT_MSC_CRIT0: case DMT_MSC_CRIT1: case DMT_MSC_CRIT2: case DMT_MSC_CRIT3:
        src32 = P<int>(m.crit[item]); n = m.ncrit[item]; break;
    case DMT_MSC_DESC_SADDLE:
        n = m.n_desc;
        if (n > cap) return fail(c, DMT_E_INVALID, "destination too small");
        if (n) {
            k_desc_saddles<<<nblocks(n), TPB, 0, st>>>(P<int>(m.crit[1]), n, dst);
            CHECK_LAUNCH(c);
            HIPCHK(c, hipStreamSynchronize(st));
        }
        return DMT_OK;
    case DMT_MSC_DESC_OFFSETS: src64 = P<int64_t>(m.doff); n = m.n_desc + 1; break;
    case DMT_MSC_DESC_CELLS: src32 = P<int>(m.dcell); n = m.n_desc_cells; break;
    case DMT_MSC_DESC_TERMINAL: src32 = P<int>(m.dterm); n = m.n_desc; break;
    case DMT_MSC_ASC_SADDLE: src32 = P<int>(m.asad); n = m.n_asc; break;
    case DMT_MSC_ASC_OFFSETS: src64 = P<int64_t>(m.aoff); n = m.n_asc + 1; break;
    case DMT_MSC_ASC_CELLS: src32 = P<int>(m.acell); n = m.n_asc_cells; break;
    case DMT_MSC_ASC_TERMINAL: src32 = P<int>(m.aterm); n = m.n_asc; break;
    case DMT_MSC_MIN_LABEL: src32 = P<int>(m.vlab); n = m.n_vlab; break;
    case DMT_MSC_MAX_LABEL: src32 = P<int>(m.tlab); n = m.n_tlab; break;
    default: return fail(c, DMT_E_INVALID, "unknown item");
    }
    if (n > cap) return fail(c, DMT_E_INVALID, "destination too small");
    if (n == 0) return DMT_OK;
    if (src64) {
        HIPCHK(c, hipMemcpyAsync(dst, src64, sizeof(int64_t) * (size_t)n, hipMemcpyDeviceToDevice, st));
    } else {
        k_i32_to_i64<<<nblocks(n), TPB, 0, st>>>(src32, n, dst);
        CHECK_LAUNCH(c);
    }
    HIPCHK(c, hipStreamSynchronize(st));
    return DMT_OK;
}

dmt_status dmt_correct(dmt_context* c, const dmt_grid* gr, const float* f, const float* g_hat, float xi,
                       const dmt_options* o, float* g_out, uint8_t* q_out, dmt_stats* stats, hipStream_t st) {
    if (!c) return DMT_E_INVALID;
    if (!f || !g_hat || !o || !g_out || !q_out) return fail(c, DMT_E_INVALID, "null argument");
    std::vector<Job> jobs(1);
    Job& J = jobs[0];
    TRY(check_grid(c, gr, J.dm, J.D));
    TRY(check_options(c, o, xi));
    HIPCHK(c, hipSetDevice(c->device));
    J.f = f; J.gh = g_hat; J.xi = xi; J.o = *o; J.g_out = g_out; J.q_out = q_out;
    c->n_lossless = 0;
    c->log.clear();
    TRY(run_jobs(c, jobs, true, st));
    if (J.status == DMT_E_NONFINITE) return fail(c, DMT_E_NONFINITE, "non-finite value in f or g_hat");
    if (J.status == DMT_E_BOUND) return fail(c, DMT_E_BOUND, "|g_hat - f| > xi somewhere");
    if (stats) *stats = J.stats;
    return J.status;
}

dmt_status dmt_correct_noalloc(dmt_context* c, const dmt_grid* gr, const float* f, const float* g_hat, float xi,
                               const dmt_options* o, float* g_out, uint8_t* q_out, int64_t* ll_idx, float* ll_val,
                               int64_t ll_cap, int64_t* ll_count, dmt_stats* stats, hipStream_t st) {
    if (!c) return DMT_E_INVALID;
    if (!f || !g_hat || !o || !g_out || !q_out || !ll_count) return fail(c, DMT_E_INVALID, "null argument");
    if (ll_cap < 0 || (ll_cap > 0 && (!ll_idx || !ll_val))) return fail(c, DMT_E_INVALID, "bad lossless destination");
    Dims dm{};
    int D = 2;
    TRY(check_grid(c, gr, dm, D));
    TRY(check_options(c, o, xi));
    if (!c->scratch) return fail(c, DMT_E_HIP, "no scratch on this device: " + c->scratch_err);
    if (workspace_estimate(D, dm.n, o) > (int64_t)DMT_NOALLOC_SCRATCH_BYTES)
        return fail(c, DMT_E_NOMEM, "field of " + std::to_string((long long)dm.n) + " vertices needs about " +
                                        std::to_string((long long)workspace_estimate(D, dm.n, o)) +
                                        " bytes of scratch; the allocation-free path holds " +
                                        std::to_string((long long)DMT_NOALLOC_SCRATCH_BYTES));
    // Every buffer this call uses starts empty, so ensure() carves it from the scratch arena; the
    // context's own buffers are set aside and put back afterwards.  Kernel timing stays off (it
    // would create events).
    std::vector<DevBuf*> cb = context_bufs(c);
    std::vector<DevBuf> saved_cb;
    for (DevBuf* b : cb) { saved_cb.push_back(*b); *b = DevBuf{}; }
    const bool had_ws = !c->ws.empty();
    JobWs saved_ws;
    if (had_ws) { saved_ws = c->ws[0]; c->ws[0] = JobWs{}; }
    const bool prof = c->prof;
    c->prof = false;
    c->arena_on = true;
    c->arena_used = 0;
    dmt_status s = dmt_correct(c, gr, f, g_hat, xi, o, g_out, q_out, stats, st);
    if (s >= 0) {
        *ll_count = c->n_lossless;
        if (c->n_lossless > ll_cap) {
            s = fail(c, DMT_E_INVALID, "destination too small for the lossless list");
        } else if (c->n_lossless > 0) {
            const size_t m = (size_t)c->n_lossless;
            hipError_t e = hipMemcpyAsync(ll_idx, c->ll_idx.p, sizeof(int64_t) * m, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess) e = hipMemcpyAsync(ll_val, c->ll_val.p, sizeof(float) * m, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) s = fail(c, DMT_E_HIP, std::string("lossless list copy: ") + hipGetErrorString(e));
        }
    }
    c->arena_on = false;
    c->prof = prof;
    for (size_t k = 0; k < cb.size(); k++) *cb[k] = saved_cb[k];
    if (had_ws) c->ws[0] = saved_ws;
    else c->ws.clear();
    c->n_lossless = 0;   // the list was handed to the caller; the context keeps none
    return s;
}

dmt_status dmt_set_tuning(dmt_context* c, const dmt_tuning* t) {
    if (!c) return DMT_E_INVALID;
    if (!t) {
        c->tune = default_tuning();
        return DMT_OK;
    }
    if ((t->loop_threads[0] != 512 && t->loop_threads[0] != 1024) ||
        (t->loop_threads[1] != 256 && t->loop_threads[1] != 512))
        return fail(c, DMT_E_INVALID, "loop_threads must be 512 or 1024 (2D) and 256 or 512 (3D)");
    for (int k = 0; k < 2; k++) {
        if (t->handoff_anchors[k] < 0 || t->batch_handoff_anchors[k] < 0)
            return fail(c, DMT_E_INVALID, "handoff_anchors and batch_handoff_anchors must be >= 0");
        if (t->grid_iterations[k] < 1 || t->grid_iterations[k] > 4096)
            return fail(c, DMT_E_INVALID, "grid_iterations must be in 1..4096");
    }
    c->tune = *t;
    return DMT_OK;
}

dmt_status dmt_get_tuning(const dmt_context* c, dmt_tuning* t) {
    if (!c || !t) return DMT_E_INVALID;
    *t = c->tune;
    return DMT_OK;
}

dmt_status dmt_correct_batch(dmt_context* c, int32_t n_jobs, dmt_job* jobs_host, hipStream_t st) {
    if (!c) return DMT_E_INVALID;
    if (n_jobs < 0 || (n_jobs > 0 && !jobs_host)) return fail(c, DMT_E_INVALID, "bad job list");
    if (n_jobs == 0) return DMT_OK;
    HIPCHK(c, hipSetDevice(c->device));
    std::vector<Job> jobs;
    std::vector<int> idx;
    for (int j = 0; j < n_jobs; j++) {
        dmt_job& h = jobs_host[j];
        h.stats = dmt_stats{};
        Job J;
        dmt_status s = check_grid(c, &h.grid, J.dm, J.D);
        if (s == DMT_OK) s = check_options(c, &h.opts, h.xi);
        if (s == DMT_OK && (h.opts.flags & ~(uint32_t)DMT_F_SADDLE_SADDLE))
            s = fail(c, DMT_E_INVALID, "batched jobs take no flags but DMT_F_SADDLE_SADDLE");
        if (s == DMT_OK && (!h.f || !h.g_hat || !h.g_out || !h.q_out)) s = fail(c, DMT_E_INVALID, "null argument");
        h.status = s;
        if (s != DMT_OK) continue;
        J.f = h.f; J.gh = h.g_hat; J.xi = h.xi; J.o = h.opts; J.g_out = h.g_out; J.q_out = h.q_out;
        jobs.push_back(J);
        idx.push_back(j);
    }
    if (!jobs.empty()) TRY(run_jobs(c, jobs, false, st));
    for (size_t k = 0; k < jobs.size(); k++) {
        jobs_host[idx[k]].status = jobs[k].status;
        jobs_host[idx[k]].stats = jobs[k].stats;
    }
    // the call's status: the first error of any job, else not-converged if any, else ok
    dmt_status worst = DMT_OK;
    for (int j = 0; j < n_jobs; j++) {
        const dmt_status s = jobs_host[j].status;
        if (s < 0 && worst >= 0) worst = s;
        else if (s == DMT_W_NOT_CONVERGED && worst == DMT_OK) worst = s;
    }
    return worst;
}

dmt_status dmt_lossless_edits(dmt_context* c, int64_t* idx_out, float* val_out, int64_t cap, int64_t* count,
                              hipStream_t st) {
    if (!c || !count || cap < 0) return fail(c, DMT_E_INVALID, "bad argument");
    *count = c->n_lossless;
    const int64_t m = cap < c->n_lossless ? cap : c->n_lossless;
    if (m == 0) return DMT_OK;
    if (!idx_out || !val_out) return fail(c, DMT_E_INVALID, "null output");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipMemcpyAsync(idx_out, c->ll_idx.p, sizeof(int64_t) * (size_t)m, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipMemcpyAsync(val_out, c->ll_val.p, sizeof(float) * (size_t)m, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipStreamSynchronize(st));
    return DMT_OK;
}

dmt_status dmt_lossless_list(dmt_context* c, const uint8_t* q_out, const float* g_out, int64_t n, int64_t* idx_out,
                             float* val_out, int64_t cap, int64_t* count, hipStream_t st) {
    if (!c || !q_out || !g_out || !count || n < 0 || cap < 0) return fail(c, DMT_E_INVALID, "bad argument");
    if (n > (int64_t)INT32_MAX) return fail(c, DMT_E_INVALID, "too many vertices");
    *count = 0;
    if (n == 0) return DMT_OK;
    HIPCHK(c, hipSetDevice(c->device));
    const unsigned nb = nblocks(n);
    ENSURE(c, c->blk, sizeof(int) * (size_t)nb);
    ENSURE(c, c->blkoff, sizeof(int64_t) * (size_t)(nb + 1));
    k_lossless_count<<<nb, TPB, 0, st>>>(q_out, (int)n, P<int>(c->blk));
    CHECK_LAUNCH(c);
    int64_t total = 0;
    TRY(scan(c, P<int>(c->blk), nb, P<int64_t>(c->blkoff), &total, st));
    *count = total;
    if (total == 0 || cap == 0) return DMT_OK;
    if (!idx_out || !val_out) return fail(c, DMT_E_INVALID, "null output");
    if (cap < total) return fail(c, DMT_E_INVALID, "destination too small for the lossless list");
    k_lossless_write<<<nb, TPB, 0, st>>>(q_out, g_out, (int)n, P<int64_t>(c->blkoff), idx_out, val_out);
    CHECK_LAUNCH(c);
    HIPCHK(c, hipStreamSynchronize(st));
    return DMT_OK;
}

dmt_status dmt_iteration_log(dmt_context* c, int64_t* log_host, int64_t cap, int64_t* count) {
    if (!c || !count || cap < 0) return fail(c, DMT_E_INVALID, "bad argument");
    const int64_t nrec = (int64_t)c->log.size() / DMT_LOG_WORDS;
    *count = nrec;
    const int64_t m = cap < nrec ? cap : nrec;
    if (m && !log_host) return fail(c, DMT_E_INVALID, "null output");
    if (m) std::memcpy(log_host, c->log.data(), sizeof(int64_t) * DMT_LOG_WORDS * (size_t)m);
    return DMT_OK;
}

dmt_status dmt_profile_enable(dmt_context* c, int enable) {
    if (!c) return DMT_E_INVALID;
    c->prof = enable != 0;
    c->ev_used = 0;
    for (int k = 0; k < DMT_PROF_KERNELS; k++) {
        c->prof_ev[k].clear();
        c->prof_units[k] = 0;
    }
    return DMT_OK;
}

dmt_status dmt_profile_read(dmt_context* c, int kernel, int64_t* launches, double* ms_total, int64_t* units) {
    if (!c || !launches || !ms_total || !units || kernel < 0 || kernel >= DMT_PROF_KERNELS)
        return fail(c, DMT_E_INVALID, "bad argument");
    HIPCHK(c, hipSetDevice(c->device));
    double ms = 0.0;
    for (auto& pr : c->prof_ev[kernel]) {
        HIPCHK(c, hipEventSynchronize(pr.second));
        float t = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&t, pr.first, pr.second));
        ms += t;
    }
    *launches = (int64_t)c->prof_ev[kernel].size();
    *ms_total = ms;
    *units = c->prof_units[kernel];
    if (kernel >= DMT_PROF_LOOP_SAPPLY && kernel <= DMT_PROF_LOOP_VR) {
        // phases inside the resident loop (summed over jobs): wall-clock ticks (100 MHz)
        // recorded by the kernel during the last correction call
        *launches = 0;
        *units = 0;
        *ms_total = (double)c->ph[kernel - DMT_PROF_LOOP_SAPPLY] * 1e-5;
    }
    return DMT_OK;
}

dmt_status dmt_apply_edits(dmt_context* c, const float* g_hat, const uint8_t* q, int64_t n, const int64_t* idx,
                           const float* val, int64_t n_lossless, float xi, int32_t q_max, float* g_out,
                           hipStream_t st) {
    if (!c || !g_hat || !q || !g_out || n < 0 || n_lossless < 0) return fail(c, DMT_E_INVALID, "bad argument");
    if (n_lossless && (!idx || !val)) return fail(c, DMT_E_INVALID, "null lossless arrays");
    if (q_max < 0 || q_max > 7) return fail(c, DMT_E_INVALID, "q_max must be 0..7");
    if (!(xi > 0.0f) || !std::isfinite(xi) || !(ldexpf(xi, -q_max) >= FLT_MIN))
        return fail(c, DMT_E_INVALID, "bad xi");
    if (n == 0) return DMT_OK;
    HIPCHK(c, hipSetDevice(c->device));
    ENSURE(c, c->flags, 16);
    HIPCHK(c, hipMemsetAsync(c->flags.p, 0, sizeof(unsigned), st));
    k_decode<<<nblocks(n), TPB, 0, st>>>(g_hat, q, n, ldexpf(xi, -q_max), g_out);
    if (n_lossless) k_scatter<<<nblocks(n_lossless), TPB, 0, st>>>(idx, val, n_lossless, n, g_out, P<unsigned>(c->flags));
    CHECK_LAUNCH(c);
    HIPCHK(c, hipMemcpyAsync(c->hscratch, c->flags.p, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (*reinterpret_cast<unsigned*>(c->hscratch)) return fail(c, DMT_E_INVALID, "lossless index out of range");
    return DMT_OK;
}


int32_t dmt_edit_bits(int32_t q_max) { return q_max < 0 || q_max > 7 ? -1 : edit_bits(q_max); }

dmt_status dmt_pack_edits(dmt_context* c, const uint8_t* q_out, const float* g_out, int64_t n, int32_t q_max,
                          uint32_t* stream, int64_t stream_words, float* lossless_val, int64_t lossless_cap,
                          int64_t* n_lossless, hipStream_t st) {
    if (!c || !q_out || !g_out || !stream || !n_lossless || n < 0 || lossless_cap < 0)
        return fail(c, DMT_E_INVALID, "bad argument");
    if (q_max < 0 || q_max > 7) return fail(c, DMT_E_INVALID, "q_max must be 0..7");
    if (n > (int64_t)INT32_MAX) return fail(c, DMT_E_INVALID, "too many vertices");
    const int b = edit_bits(q_max);
    const int64_t words = (n * b + 31) / 32;
    if (stream_words < words) return fail(c, DMT_E_INVALID, "stream too small: needs " + std::to_string((long long)words) +
                                                               " words");
    *n_lossless = 0;
    if (n == 0) return DMT_OK;
    HIPCHK(c, hipSetDevice(c->device));
    const unsigned nb = nblocks(n);
    ENSURE(c, c->flags, 16);
    ENSURE(c, c->blk, sizeof(int) * (size_t)nb);
    ENSURE(c, c->blkoff, sizeof(int64_t) * (size_t)(nb + 1));
    HIPCHK(c, hipMemsetAsync(c->flags.p, 0, sizeof(unsigned), st));
    k_pack_edits<<<nblocks(words), TPB, 0, st>>>(q_out, n, q_max, b, words, stream, P<unsigned>(c->flags));
    k_lossless_count<<<nb, TPB, 0, st>>>(q_out, (int)n, P<int>(c->blk));
    CHECK_LAUNCH(c);
    int64_t total = 0;
    TRY(scan(c, P<int>(c->blk), nb, P<int64_t>(c->blkoff), &total, st));   // synchronises
    HIPCHK(c, hipMemcpyAsync(c->hscratch, c->flags.p, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (*reinterpret_cast<unsigned*>(c->hscratch)) return fail(c, DMT_E_INVALID, "q_out holds a value above q_max");
    *n_lossless = total;
    if (total == 0 || lossless_cap == 0) return DMT_OK;
    if (!lossless_val) return fail(c, DMT_E_INVALID, "null lossless_val");
    if (lossless_cap < total) return fail(c, DMT_E_INVALID, "lossless_val too small");
    k_lossless_write<<<nb, TPB, 0, st>>>(q_out, g_out, (int)n, P<int64_t>(c->blkoff), nullptr, lossless_val);
    CHECK_LAUNCH(c);
    HIPCHK(c, hipStreamSynchronize(st));
    return DMT_OK;
}

dmt_status dmt_unpack_edits(dmt_context* c, const uint32_t* stream, int64_t stream_words, int64_t n, int32_t q_max,
                            const float* g_hat, const float* lossless_val, int64_t n_lossless, float xi, float* g_out,
                            uint8_t* q_out, hipStream_t st) {
    if (!c || !stream || !g_hat || !g_out || n < 0 || n_lossless < 0) return fail(c, DMT_E_INVALID, "bad argument");
    if (n_lossless && !lossless_val) return fail(c, DMT_E_INVALID, "null lossless_val");
    if (q_max < 0 || q_max > 7) return fail(c, DMT_E_INVALID, "q_max must be 0..7");
    if (!(xi > 0.0f) || !std::isfinite(xi) || !(ldexpf(xi, -q_max) >= FLT_MIN)) return fail(c, DMT_E_INVALID, "bad xi");
    if (n > (int64_t)INT32_MAX) return fail(c, DMT_E_INVALID, "too many vertices");
    const int b = edit_bits(q_max);
    const int64_t words = (n * b + 31) / 32;
    if (stream_words < words) return fail(c, DMT_E_INVALID, "stream too short for n vertices");
    if (n == 0) return DMT_OK;
    HIPCHK(c, hipSetDevice(c->device));
    const unsigned nb = nblocks(n);
    ENSURE(c, c->flags, 16);
    ENSURE(c, c->blk, sizeof(int) * (size_t)nb);
    ENSURE(c, c->blkoff, sizeof(int64_t) * (size_t)(nb + 1));
    HIPCHK(c, hipMemsetAsync(c->flags.p, 0, sizeof(unsigned), st));
    k_unpack_count<<<nb, TPB, 0, st>>>(stream, words, (int)n, q_max, b, P<int>(c->blk), P<unsigned>(c->flags));
    CHECK_LAUNCH(c);
    int64_t total = 0;
    TRY(scan(c, P<int>(c->blk), nb, P<int64_t>(c->blkoff), &total, st));
    HIPCHK(c, hipMemcpyAsync(c->hscratch, c->flags.p, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (*reinterpret_cast<unsigned*>(c->hscratch)) return fail(c, DMT_E_INVALID, "stream holds a code above q_max + 1");
    if (total != n_lossless)
        return fail(c, DMT_E_INVALID, "stream marks " + std::to_string((long long)total) + " lossless vertices, " +
                                          std::to_string((long long)n_lossless) + " values given");
    k_unpack_write<<<nb, TPB, 0, st>>>(stream, words, (int)n, q_max, b, g_hat, lossless_val, P<int64_t>(c->blkoff),
                                       n_lossless, ldexpf(xi, -q_max), g_out, q_out, P<unsigned>(c->flags));
    CHECK_LAUNCH(c);
    HIPCHK(c, hipStreamSynchronize(st));
    return DMT_OK;
}

int64_t dmt_workspace_bytes(const dmt_grid* gr, const dmt_options* o) {
    if (!gr || !o) return -1;
    Dims dm;
    int D;
    if (check_grid(nullptr, gr, dm, D) != DMT_OK) return -1;
    return workspace_estimate(D, dm.n, o);
}

dmt_status dmt_server_create(dmt_server** out, int hip_device, int64_t hbm_budget_bytes, int32_t max_jobs) {
    if (!out || hbm_budget_bytes <= 0 || max_jobs < 1 || max_jobs > 4096) return DMT_E_INVALID;
    *out = nullptr;
    dmt_server* s = new dmt_server();
    s->budget = hbm_budget_bytes;
    s->max_jobs = max_jobs;
    // up to SERVER_LANES lanes; the max_jobs slots are dealt out among them
    const int nl = std::min(max_jobs, SERVER_LANES);
    s->lanes.resize(nl);
    dmt_status rc = DMT_OK;
    for (int li = 0; li < nl && rc == DMT_OK; li++) {
        Lane& L = s->lanes[li];
        const int nslots = max_jobs / nl + (li < max_jobs % nl ? 1 : 0);
        rc = dmt_context_create(&L.c, hip_device);
        if (rc != DMT_OK) break;
        dmt_context* c = L.c;
        c->ws.resize(nslots);
        c->hctl.assign(nslots, Ctl{});
        if (hipStreamCreateWithFlags(&L.st, hipStreamNonBlocking) != hipSuccess ||
            ensure(c, c->ctl_all, sizeof(Ctl) * nslots) != DMT_OK ||
            ensure(c, c->flags, sizeof(unsigned) * (nslots + 1)) != DMT_OK ||
            hipMemsetAsync(c->ctl_all.p, 0, sizeof(Ctl) * nslots, L.st) != hipSuccess) {
            rc = DMT_E_NOMEM;
            break;
        }
        for (int k = nslots - 1; k >= 0; k--) L.free_slots.push_back(k);
        L.charge.assign(nslots, 0);
        L.held.assign(nslots, 0);
        L.shared = shared_bytes(c);
    }
    if (rc != DMT_OK) {
        for (Lane& L : s->lanes) {
            if (L.st) (void)hipStreamDestroy(L.st);
            if (L.c) dmt_context_destroy(L.c);
        }
        delete s;
        return rc;
    }
    recount(s);
    s->idle_lanes = nl;
    if (const char* e = getenv("DMT_FAULT_OUTPUTS")) s->fail_outputs_at = atoll(e);
    for (int li = 0; li < nl; li++) s->lanes[li].worker = std::thread(server_main, s, li);
    *out = s;
    return DMT_OK;
}

dmt_status dmt_server_destroy(dmt_server* s) {
    if (!s) return DMT_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (Lane& L : s->lanes)
        if (L.worker.joinable()) L.worker.join();
    for (Lane& L : s->lanes) {
        (void)hipSetDevice(L.c->device);
        if (L.st) (void)hipStreamDestroy(L.st);
        dmt_context_destroy(L.c);
    }
    delete s;
    return DMT_OK;
}

dmt_status dmt_server_submit(dmt_server* s, const dmt_job* job, int64_t* ticket) {
    if (!s || !job || !ticket) return DMT_E_INVALID;
    Ticket t;
    t.job = *job;
    t.job.stats = dmt_stats{};
    Job& J = t.J;
    dmt_status rc = check_grid(nullptr, &job->grid, J.dm, J.D);
    if (rc == DMT_OK) rc = check_options(nullptr, &job->opts, job->xi);
    if (rc == DMT_OK && (job->opts.flags & ~(uint32_t)DMT_F_SADDLE_SADDLE)) rc = DMT_E_INVALID;
    if (rc == DMT_OK && (!job->f || !job->g_hat || !job->g_out || !job->q_out)) rc = DMT_E_INVALID;
    if (rc != DMT_OK) return rc;
    J.f = job->f; J.gh = job->g_hat; J.xi = job->xi; J.o = job->opts; J.g_out = job->g_out; J.q_out = job->q_out;
    t.bytes = workspace_estimate(J.D, J.dm.n, &job->opts);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return DMT_E_INVALID;
        *ticket = s->next_ticket++;
        s->tickets.emplace(*ticket, std::move(t));
        s->pending.push_back(*ticket);
        s->epoch++;
    }
    s->cv_work.notify_all();
    return DMT_OK;
}

dmt_status dmt_server_info(dmt_server* s, int64_t* inflight_bytes, int64_t* held_bytes_host, int32_t* free_slots,
                           int32_t* pending, int32_t* distinct_free_slots) {
    if (!s) return DMT_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    if (inflight_bytes) *inflight_bytes = s->inflight;
    int64_t h = 0;
    int32_t nfree = 0, ndistinct = 0;
    for (const Lane& L : s->lanes) {
        h += L.shared;
        for (int64_t b : L.held) h += b;
        nfree += (int32_t)L.free_slots.size();
        std::vector<int> v = L.free_slots;
        std::sort(v.begin(), v.end());
        ndistinct += (int32_t)(std::unique(v.begin(), v.end()) - v.begin());
    }
    if (held_bytes_host) *held_bytes_host = h;
    if (free_slots) *free_slots = nfree;
    if (pending) *pending = (int32_t)s->pending.size();
    if (distinct_free_slots) *distinct_free_slots = ndistinct;
    return DMT_OK;
}

dmt_status dmt_server_poll(dmt_server* s, int64_t ticket, int32_t wait, dmt_job* result) {
    if (!s || !result) return DMT_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return DMT_E_INVALID;
    if (it->second.state != 2) {
        if (!wait) return DMT_W_PENDING;
        s->cv_done.wait(lk, [&] { return it->second.state == 2; });
    }
    *result = it->second.job;
    s->tickets.erase(it);
    return DMT_OK;
}

}  // extern "C"
