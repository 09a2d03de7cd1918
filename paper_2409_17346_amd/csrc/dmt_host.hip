// Host side of the C ABI declared in include/dmt.h: validation, workspace, MSC extraction and
// the C-loop / S-loop driver (Sections 4.2-4.6 of the paper).  All arithmetic on field values
// happens in the kernels of dmt_kernels.h; the host only sequences launches and reads counters.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "dmt.h"
#include "dmt_frontier.h"

using namespace dmt;

namespace {

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
};

constexpr int TPB = 256;
inline unsigned nblocks(int64_t n) { return (unsigned)((n + TPB - 1) / TPB); }

}  // namespace

struct dmt_context {
    int device = 0;
    std::string err;
    DevBuf lo, g, state, req, fpl, gpl, cnt, flags, part, blk, blkoff;
    DevBuf crit[4];
    int64_t ncrit[4] = {0, 0, 0, 0};
    // descending / ascending branches (int32 cell ids, int64 offsets)
    DevBuf dsad, doff, dcell, dcbr, dterm, dlen, dfirst;
    DevBuf asad, aoff, acell, acbr, aterm, alen, afirst, astart, asadcnt, asadoff;
    int64_t n_desc = 0, n_desc_cells = 0, n_asc = 0, n_asc_cells = 0;
    DevBuf vlab, tlab;
    int64_t n_vlab = 0, n_tlab = 0;
    // frontier loop state
    DevBuf ctl, vmask, inlist, vl0, vl1, dvl0, dvl1, dal0, dal1, vstamp, astamp, rstamp, reql, dlog;
    Ctl* hctl = nullptr;                  // pinned
    bool have_msc = false;
    DevBuf ll_idx, ll_val;
    int64_t n_lossless = 0;
    std::vector<int64_t> log;
    unsigned long long* hcnt = nullptr;   // pinned
    int64_t* hscratch = nullptr;          // pinned
    // kernel timing: event pairs per kernel family, recorded on the launch stream
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev[DMT_PROF_KERNELS];
    int64_t prof_units[DMT_PROF_KERNELS] = {0};
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

dmt_status ensure(dmt_context* c, DevBuf& b, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (b.cap >= bytes) return DMT_OK;
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

template <typename T>
T* P(DevBuf& b) { return reinterpret_cast<T*>(b.p); }

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
    return DMT_OK;
}

int nplanes(int D) { return D == 2 ? Geom<2>::NB : Geom<3>::NB; }
int ntypes(int D, int d) { return D == 2 ? G<2>::g.ntypes[d] : G<3>::g.ntypes[d]; }

hipEvent_t next_event(dmt_context* c) {
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->ev_pool.push_back(e);
    }
    return c->ev_pool[c->ev_used++];
}

// Brackets one launch of kernel family k with events when timing is on.
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

// exclusive scan of n ints into n+1 int64 (device), total returned on the host
dmt_status scan(dmt_context* c, const int* in, int64_t n, int64_t* out, int64_t* total, hipStream_t st) {
    k_scan_single<<<1, 1024, 0, st>>>(in, n, out);
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

// Critical cells and separatrix branches of the gradient in planes pl (Section 3.1).
template <int D>
dmt_status build_msc(dmt_context* c, const uint8_t* pl, const Dims& dm, bool labels, hipStream_t st) {
    constexpr auto& g = G<D>::g;
    const unsigned nb = nblocks(dm.n);
    ENSURE(c, c->flags, 16);
    HIPCHK(c, hipMemsetAsync(c->flags.p, 0, sizeof(unsigned), st));
    unsigned* werr = P<unsigned>(c->flags);
    ENSURE(c, c->blk, sizeof(int) * (size_t)(D + 1) * nb);
    ENSURE(c, c->blkoff, sizeof(int64_t) * (size_t)(D + 1) * (nb + 1));
    k_crit_count<D><<<nb, TPB, 0, st>>>(pl, dm, P<int>(c->blk));
    CHECK_LAUNCH(c);
    for (int d = 0; d <= D; d++) {
        dmt_status s = scan(c, P<int>(c->blk) + (size_t)d * nb, nb, P<int64_t>(c->blkoff) + (size_t)d * (nb + 1),
                            &c->ncrit[d], st);
        if (s != DMT_OK) return s;
        ENSURE(c, c->crit[d], sizeof(int) * (size_t)c->ncrit[d]);
    }
    for (int d = D + 1; d < 4; d++) c->ncrit[d] = 0;
    k_crit_write<D><<<nb, TPB, 0, st>>>(pl, dm, P<int64_t>(c->blkoff), (int)nb, P<int>(c->crit[0]),
                                        P<int>(c->crit[1]), P<int>(c->crit[2]), D == 3 ? P<int>(c->crit[3]) : nullptr);
    CHECK_LAUNCH(c);

    // descending branches: two per 1-saddle
    c->n_desc = 2 * c->ncrit[1];
    ENSURE(c, c->dlen, sizeof(int) * (size_t)c->n_desc);
    ENSURE(c, c->dterm, sizeof(int) * (size_t)c->n_desc);
    ENSURE(c, c->doff, sizeof(int64_t) * (size_t)(c->n_desc + 1));
    ENSURE(c, c->dfirst, sizeof(int) * (size_t)c->n_desc);
    if (c->n_desc) {
        k_desc_walk<D><<<nblocks(c->n_desc), TPB, 0, st>>>(pl, dm, P<int>(c->crit[1]), (int)c->n_desc, 0,
                                                           P<int>(c->dlen), P<int>(c->dterm), nullptr, nullptr, nullptr, werr);
        CHECK_LAUNCH(c);
    }
    dmt_status s = scan(c, P<int>(c->dlen), c->n_desc, P<int64_t>(c->doff), &c->n_desc_cells, st);
    if (s != DMT_OK) return s;
    ENSURE(c, c->dcell, sizeof(int) * (size_t)c->n_desc_cells);
    ENSURE(c, c->dcbr, sizeof(int) * (size_t)c->n_desc_cells);
    if (c->n_desc) {
        k_desc_walk<D><<<nblocks(c->n_desc), TPB, 0, st>>>(pl, dm, P<int>(c->crit[1]), (int)c->n_desc, 1, nullptr,
                                                           nullptr, P<int64_t>(c->doff), P<int>(c->dcell), P<int>(c->dcbr), werr);
        CHECK_LAUNCH(c);
    }
    s = fill_i32(c, P<int>(c->dfirst), c->n_desc, INF32, st);
    if (s != DMT_OK) return s;

    // ascending branches: one per top cofacet of each (D-1)-saddle
    const int64_t nsad = c->ncrit[D - 1];
    ENSURE(c, c->asadcnt, sizeof(int) * (size_t)nsad);
    ENSURE(c, c->asadoff, sizeof(int64_t) * (size_t)(nsad + 1));
    if (nsad) {
        k_asc_starts<D><<<nblocks(nsad), TPB, 0, st>>>(dm, P<int>(c->crit[D - 1]), (int)nsad, 0, P<int>(c->asadcnt),
                                                       nullptr, nullptr, nullptr);
        CHECK_LAUNCH(c);
    }
    s = scan(c, P<int>(c->asadcnt), nsad, P<int64_t>(c->asadoff), &c->n_asc, st);
    if (s != DMT_OK) return s;
    ENSURE(c, c->astart, sizeof(int) * (size_t)c->n_asc);
    ENSURE(c, c->asad, sizeof(int) * (size_t)c->n_asc);
    ENSURE(c, c->alen, sizeof(int) * (size_t)c->n_asc);
    ENSURE(c, c->aterm, sizeof(int) * (size_t)c->n_asc);
    ENSURE(c, c->aoff, sizeof(int64_t) * (size_t)(c->n_asc + 1));
    ENSURE(c, c->afirst, sizeof(int) * (size_t)c->n_asc);
    if (nsad) {
        k_asc_starts<D><<<nblocks(nsad), TPB, 0, st>>>(dm, P<int>(c->crit[D - 1]), (int)nsad, 1, nullptr,
                                                       P<int64_t>(c->asadoff), P<int>(c->astart), P<int>(c->asad));
        CHECK_LAUNCH(c);
    }
    if (c->n_asc) {
        k_asc_walk<D><<<nblocks(c->n_asc), TPB, 0, st>>>(pl, dm, P<int>(c->astart), (int)c->n_asc, 0, P<int>(c->alen),
                                                         P<int>(c->aterm), nullptr, nullptr, nullptr, werr);
        CHECK_LAUNCH(c);
    }
    s = scan(c, P<int>(c->alen), c->n_asc, P<int64_t>(c->aoff), &c->n_asc_cells, st);
    if (s != DMT_OK) return s;
    ENSURE(c, c->acell, sizeof(int) * (size_t)c->n_asc_cells);
    ENSURE(c, c->acbr, sizeof(int) * (size_t)c->n_asc_cells);
    if (c->n_asc) {
        k_asc_walk<D><<<nblocks(c->n_asc), TPB, 0, st>>>(pl, dm, P<int>(c->astart), (int)c->n_asc, 1, nullptr, nullptr,
                                                         P<int64_t>(c->aoff), P<int>(c->acell), P<int>(c->acbr), werr);
        CHECK_LAUNCH(c);
    }
    s = fill_i32(c, P<int>(c->afirst), c->n_asc, INF32, st);
    if (s != DMT_OK) return s;

    HIPCHK(c, hipMemcpyAsync(c->hscratch, werr, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (*reinterpret_cast<unsigned*>(c->hscratch)) return fail(c, DMT_E_HIP, "internal error: a V-path did not end");
    c->n_vlab = c->n_tlab = 0;
    if (labels) {
        c->n_vlab = dm.n;
        c->n_tlab = (int64_t)dm.n * g.ntypes[D];
        ENSURE(c, c->vlab, sizeof(int) * (size_t)c->n_vlab);
        ENSURE(c, c->tlab, sizeof(int) * (size_t)c->n_tlab);
        ENSURE(c, c->flags, 16);
        k_label_init<D><<<nb, TPB, 0, st>>>(pl, dm, P<int>(c->vlab), P<int>(c->tlab));
        CHECK_LAUNCH(c);
        for (int round = 0; round < 64; round++) {
            HIPCHK(c, hipMemsetAsync(c->flags.p, 0, sizeof(unsigned), st));
            k_jump<<<nblocks(c->n_vlab), TPB, 0, st>>>(P<int>(c->vlab), c->n_vlab, P<unsigned>(c->flags));
            k_jump<<<nblocks(c->n_tlab), TPB, 0, st>>>(P<int>(c->tlab), c->n_tlab, P<unsigned>(c->flags));
            CHECK_LAUNCH(c);
            HIPCHK(c, hipMemcpyAsync(c->hscratch, c->flags.p, sizeof(unsigned), hipMemcpyDeviceToHost, st));
            HIPCHK(c, hipStreamSynchronize(st));
            if (*reinterpret_cast<unsigned*>(c->hscratch) == 0) break;
        }
    }
    c->have_msc = true;
    return DMT_OK;
}

dmt_status read_counters(dmt_context* c, hipStream_t st) {
    HIPCHK(c, hipMemcpyAsync(c->hcnt, c->cnt.p, sizeof(unsigned long long) * CNT_WORDS, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    return DMT_OK;
}

// Frontier loop: the iterations run on the device in batches; the host reads the control block
// once per batch and grows the log buffer ahead of the next batch.
template <int D>
dmt_status frontier_loop(dmt_context* c, const Dims& dm, const float* f, const float* gh, const float* lo, float* g,
                         uint8_t* state, const uint8_t* fpl, uint8_t* gpl, float delta, const dmt_options* o,
                         int64_t& it, int64_t& c_it, int64_t& s_it, int64_t& residual, int& converged,
                         int& stalled, hipStream_t st) {
    const int n = dm.n;
    ENSURE(c, c->ctl, sizeof(Ctl));
    ENSURE(c, c->vmask, sizeof(uint32_t) * n);
    ENSURE(c, c->inlist, n);
    ENSURE(c, c->vl0, sizeof(int) * n);
    ENSURE(c, c->vl1, sizeof(int) * n);
    ENSURE(c, c->dvl0, sizeof(int) * n);
    ENSURE(c, c->dvl1, sizeof(int) * n);
    ENSURE(c, c->dal0, sizeof(int) * n);
    ENSURE(c, c->dal1, sizeof(int) * n);
    ENSURE(c, c->vstamp, sizeof(unsigned) * n);
    ENSURE(c, c->astamp, sizeof(unsigned) * n);
    ENSURE(c, c->rstamp, sizeof(unsigned) * n);
    ENSURE(c, c->reql, sizeof(int) * n);
    HIPCHK(c, hipMemsetAsync(c->inlist.p, 0, n, st));
    HIPCHK(c, hipMemsetAsync(c->vstamp.p, 0, sizeof(unsigned) * n, st));
    HIPCHK(c, hipMemsetAsync(c->astamp.p, 0, sizeof(unsigned) * n, st));
    HIPCHK(c, hipMemsetAsync(c->rstamp.p, 0, sizeof(unsigned) * n, st));
    k_fr_init<<<1, 1, 0, st>>>(P<Ctl>(c->ctl));
    CHECK_LAUNCH(c);

    FrontierBufs B{};
    B.ctl = P<Ctl>(c->ctl);
    B.f = f; B.gh = gh; B.lo = lo; B.g = g; B.state = state; B.fpl = fpl; B.gpl = gpl;
    B.vmask = P<uint32_t>(c->vmask);
    B.inlist = P<uint8_t>(c->inlist);
    B.vl[0] = P<int>(c->vl0); B.vl[1] = P<int>(c->vl1);
    B.dvl[0] = P<int>(c->dvl0); B.dvl[1] = P<int>(c->dvl1);
    B.dal[0] = P<int>(c->dal0); B.dal[1] = P<int>(c->dal1);
    B.vstamp = P<unsigned>(c->vstamp); B.astamp = P<unsigned>(c->astamp); B.rstamp = P<unsigned>(c->rstamp);
    B.reql = P<int>(c->reql);
    if (o->tier >= 3 && c->have_msc) {
        B.dcell = P<int>(c->dcell); B.dcbr = P<int>(c->dcbr); B.dterm = P<int>(c->dterm);
        B.acell = P<int>(c->acell); B.acbr = P<int>(c->acbr); B.aterm = P<int>(c->aterm);
        B.doff = P<int64_t>(c->doff); B.aoff = P<int64_t>(c->aoff);
        B.dfirst = P<int>(c->dfirst); B.afirst = P<int>(c->afirst);
        B.n_dcell = c->n_desc_cells; B.n_acell = c->n_asc_cells;
        B.n_desc = (int)c->n_desc; B.n_asc = (int)c->n_asc;
    }
    B.delta = delta;
    B.q_max = o->q_max;
    B.tier = o->tier;
    B.max_iters = o->max_iters < 0 ? INT64_MAX : o->max_iters;

    // Persistent form: one cooperative launch runs the loop with grid barriers; it pauses when
    // the log buffer is full, and the host grows the buffer and launches it again.
    size_t log_cap = c->dlog.cap / (sizeof(long long) * DMT_LOG_WORDS);
    auto grow_log = [&](size_t need, int64_t keep) -> dmt_status {
        if (need <= log_cap) return DMT_OK;
        const size_t ncap = need * 2;
        DevBuf nb;
        if (hipMalloc(&nb.p, ncap * sizeof(long long) * DMT_LOG_WORDS) != hipSuccess) {
            (void)hipGetLastError();
            return fail(c, DMT_E_NOMEM, "log allocation failed");
        }
        nb.cap = ncap * sizeof(long long) * DMT_LOG_WORDS;
        if (c->dlog.p && keep > 0)
            HIPCHK(c, hipMemcpyAsync(nb.p, c->dlog.p, (size_t)keep * sizeof(long long) * DMT_LOG_WORDS,
                                     hipMemcpyDeviceToDevice, st));
        HIPCHK(c, hipStreamSynchronize(st));
        if (c->dlog.p) (void)hipFree(c->dlog.p);
        c->dlog = nb;
        log_cap = ncap;
        return DMT_OK;
    };
    bool persistent = !(o->flags & DMT_F_PHASES);
    int coop_blocks = 0;
    if (persistent) {
        int ncu = 0, occ = 0, coop = 0;
        HIPCHK(c, hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, c->device));
        HIPCHK(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device));
        HIPCHK(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(k_fr_loop<D>),
                                                               TPB, 0));
        // The persistent grid only has to cover the frontier (iteration 0 runs as full-grid launches),
        // and a grid barrier costs more the more blocks arrive at it, so the grid is small.
        int want = 32;
        if (const char* e = getenv("DMT_COOP_BLOCKS")) want = atoi(e) > 0 ? atoi(e) : want;
        coop_blocks = want < ncu * occ ? want : ncu * occ;
        persistent = coop && coop_blocks > 0;
    }
    int64_t host_it = 0;
    if (persistent) {
        const unsigned long long timeout = 500000000ull;   // 5 s of the 100 MHz wall clock
        {
            // iteration 0: dense gradient of g and violation masks of every anchor
            const unsigned gfull = nblocks(n) < 2048u ? nblocks(n) : 2048u;
            ProfScope ps(c, DMT_PROF_GRADIENT, st, n);
            k_fr_grad<D><<<gfull, TPB, 0, st>>>(B, dm);
            k_fr_vmask<D><<<gfull, TPB, 0, st>>>(B, dm);
            CHECK_LAUNCH(c);
        }
        for (;;) {
            dmt_status gs = grow_log((size_t)host_it + 4096, host_it);
            if (gs != DMT_OK) return gs;
            B.log = P<long long>(c->dlog);
            int cap = (int)(log_cap < (size_t)INT32_MAX ? log_cap : (size_t)INT32_MAX);
            void* args[] = {&B, (void*)&dm, &cap, (void*)&timeout};
            {
                ProfScope ps(c, DMT_PROF_LOOP, st, 0);
                HIPCHK(c, hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_fr_loop<D>), dim3(coop_blocks),
                                                     dim3(TPB), args, 0, st));
            }
            HIPCHK(c, hipMemcpyAsync(c->hctl, c->ctl.p, sizeof(Ctl), hipMemcpyDeviceToHost, st));
            HIPCHK(c, hipStreamSynchronize(st));
            if (c->hctl->err) return fail(c, DMT_E_HIP, "grid barrier timed out in the persistent loop");
            host_it = c->hctl->it;
            if (c->hctl->done != 4) break;
            const int zero = 0;
            HIPCHK(c, hipMemcpyAsync(&P<Ctl>(c->ctl)->done, &zero, sizeof(int), hipMemcpyHostToDevice, st));
        }
    } else {
        // Launch-per-phase form: batches of iterations without host synchronisation.
        const unsigned gfull = nblocks(n) < 2048u ? nblocks(n) : 2048u;
        int batch = 4;
        for (;;) {
            dmt_status gs = grow_log((size_t)host_it + (size_t)batch + 1, host_it);
            if (gs != DMT_OK) return gs;
            B.log = P<long long>(c->dlog);
            for (int b = 0; b < batch; b++) {
                ProfScope ps(c, DMT_PROF_LOOP, st, 0);
                k_fr_grad<D><<<gfull, TPB, 0, st>>>(B, dm);
                k_fr_vmask<D><<<gfull, TPB, 0, st>>>(B, dm);
                k_fr_requests<D><<<gfull, TPB, 0, st>>>(B, dm);
                if (o->tier >= 3) {
                    k_fr_scheck<D><<<gfull, TPB, 0, st>>>(B, dm);
                    k_fr_stargets<D><<<gfull, TPB, 0, st>>>(B, dm);
                }
                k_fr_apply<D><<<gfull, TPB, 0, st>>>(B, dm);
                k_fr_finish<<<1, 1, 0, st>>>(B);
                CHECK_LAUNCH(c);
            }
            HIPCHK(c, hipMemcpyAsync(c->hctl, c->ctl.p, sizeof(Ctl), hipMemcpyDeviceToHost, st));
            HIPCHK(c, hipStreamSynchronize(st));
            host_it = c->hctl->it;
            if (c->hctl->done) break;
            if (batch < 256) batch *= 2;
        }
    }
    it = c->hctl->it;
    c_it = c->hctl->c_it;
    s_it = c->hctl->s_it;
    residual = c->hctl->residual;
    converged = c->hctl->done == 1;
    stalled = c->hctl->done == 3;
    c->log.assign((size_t)it * DMT_LOG_WORDS, 0);
    if (it > 0)
        HIPCHK(c, hipMemcpy(c->log.data(), c->dlog.p, sizeof(long long) * DMT_LOG_WORDS * (size_t)it,
                            hipMemcpyDeviceToHost));
    return DMT_OK;
}

template <int D>
dmt_status correct_impl(dmt_context* c, const Dims& dm, const float* f, const float* gh, float xi,
                        const dmt_options* o, float* g_out, uint8_t* q_out, dmt_stats* stats, hipStream_t st) {
    const int n = dm.n;
    const unsigned nb = nblocks(n);
    const float delta = ldexpf(xi, -o->q_max);
    const int tier = o->tier;
    ENSURE(c, c->lo, sizeof(float) * n);
    ENSURE(c, c->g, sizeof(float) * n);
    ENSURE(c, c->state, n);
    ENSURE(c, c->req, n);
    ENSURE(c, c->fpl, (size_t)Geom<D>::NB * n);
    ENSURE(c, c->gpl, (size_t)Geom<D>::NB * n);
    ENSURE(c, c->cnt, sizeof(unsigned long long) * CNT_WORDS);
    ENSURE(c, c->flags, 16);
    ENSURE(c, c->blk, sizeof(int) * (size_t)(D + 1) * nb);
    ENSURE(c, c->blkoff, sizeof(int64_t) * (size_t)(D + 1) * (nb + 1));
    unsigned long long* cnt = P<unsigned long long>(c->cnt);
    float* lo = P<float>(c->lo);
    float* g = P<float>(c->g);
    uint8_t* state = P<uint8_t>(c->state);
    uint8_t* req = P<uint8_t>(c->req);
    uint8_t* fpl = P<uint8_t>(c->fpl);
    uint8_t* gpl = P<uint8_t>(c->gpl);

    // a0: floors, validation, state
    HIPCHK(c, hipMemsetAsync(c->flags.p, 0, sizeof(unsigned), st));
    {
        ProfScope ps(c, DMT_PROF_SETUP, st, n);
        k_setup<<<nb, TPB, 0, st>>>(f, gh, xi, n, lo, g, state, req, P<unsigned>(c->flags));
        CHECK_LAUNCH(c);
    }
    HIPCHK(c, hipMemcpyAsync(c->hscratch, c->flags.p, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    const unsigned fl = *reinterpret_cast<unsigned*>(c->hscratch);
    if (fl & 1u) return fail(c, DMT_E_NONFINITE, "non-finite value in f or g_hat");
    if (fl & 2u) return fail(c, DMT_E_BOUND, "|g_hat - f| > xi somewhere");

    // a1, a2: gradient of f and its separatrix branches (fixed for the whole run)
    dmt_status s = launch_grad(c, D, f, fpl, dm, st);
    if (s != DMT_OK) return s;
    c->have_msc = false;
    if (tier >= 3) {
        ProfScope ps(c, DMT_PROF_MSC, st, n);
        s = build_msc<D>(c, fpl, dm, false, st);
        if (s != DMT_OK) return s;
    }

    c->log.clear();
    int64_t it = 0, c_it = 0, s_it = 0, residual = 0;
    int converged = 0, stalled = 0;
    const int64_t max_iters = o->max_iters < 0 ? INT64_MAX : o->max_iters;
    if (!(o->flags & DMT_F_DENSE)) {
        s = frontier_loop<D>(c, dm, f, gh, lo, g, state, fpl, gpl, delta, o, it, c_it, s_it, residual, converged,
                             stalled, st);
        if (s != DMT_OK) return s;
    }
    for (; o->flags & DMT_F_DENSE;) {
        s = launch_grad(c, D, g, gpl, dm, st);
        if (s != DMT_OK) return s;
        HIPCHK(c, hipMemsetAsync(cnt, 0, sizeof(unsigned long long) * CNT_WORDS, st));
        {
            ProfScope ps(c, DMT_PROF_CLASSIFY, st, n);
            k_classify<D><<<nb, TPB, 0, st>>>(fpl, gpl, f, g, req, dm, tier, cnt);
            CHECK_LAUNCH(c);
        }
        s = read_counters(c, st);
        if (s != DMT_OK) return s;
        int64_t viol = 0;
        for (int k = CNT_FP0; k < CNT_FP0 + 8; k++) viol += (int64_t)c->hcnt[k];
        int kind = 1;
        if (viol == 0 && tier >= 3) {
            kind = 2;
            ProfScope ps(c, DMT_PROF_SSTEP, st, c->n_desc_cells + c->n_asc_cells);
            if (c->n_desc_cells) {
                k_scheck_desc<<<nblocks(c->n_desc_cells), TPB, 0, st>>>(fpl, gpl, P<int>(c->dcell), P<int>(c->dcbr),
                                                                        c->n_desc_cells, P<int>(c->dfirst));
                k_starget<D><<<nblocks(c->n_desc), TPB, 0, st>>>(fpl, gpl, dm, 0, P<int>(c->dcell), P<int64_t>(c->doff),
                                                                 P<int>(c->dterm), (int)c->n_desc, P<int>(c->dfirst),
                                                                 tier, req, cnt);
                CHECK_LAUNCH(c);
            }
            if (c->n_asc_cells) {
                k_scheck_asc<D><<<nblocks(c->n_asc_cells), TPB, 0, st>>>(fpl, gpl, dm, P<int>(c->acell), P<int>(c->acbr),
                                                                         c->n_asc_cells, P<int>(c->afirst));
                k_starget<D><<<nblocks(c->n_asc), TPB, 0, st>>>(fpl, gpl, dm, 1, P<int>(c->acell), P<int64_t>(c->aoff),
                                                                P<int>(c->aterm), (int)c->n_asc, P<int>(c->afirst),
                                                                tier, req, cnt);
                CHECK_LAUNCH(c);
            }
            s = read_counters(c, st);
            if (s != DMT_OK) return s;
            viol = (int64_t)(c->hcnt[CNT_TM_DESC] + c->hcnt[CNT_TM_ASC]);
        }
        if (viol == 0) { converged = 1; break; }
        if (it == max_iters) {
            residual = viol;
            k_clear_u8<<<nb, TPB, 0, st>>>(req, n);
            CHECK_LAUNCH(c);
            break;
        }
        {
            ProfScope ps(c, DMT_PROF_APPLY, st, n);
            k_apply<<<nb, TPB, 0, st>>>(req, gh, lo, g, state, delta, o->q_max, n, cnt);
            CHECK_LAUNCH(c);
        }
        s = read_counters(c, st);
        if (s != DMT_OK) return s;
        if (c->hcnt[CNT_CHANGED] == 0) { stalled = 1; residual = viol; break; }
        int64_t rec[DMT_LOG_WORDS] = {0};
        rec[0] = kind;
        for (int k = 1; k <= CNT_CHANGED; k++) rec[k] = (int64_t)c->hcnt[k];
        c->log.insert(c->log.end(), rec, rec + DMT_LOG_WORDS);
        it++;
        if (kind == 1) c_it++; else s_it++;
    }

    // a8: outputs
    HIPCHK(c, hipMemcpyAsync(g_out, g, sizeof(float) * n, hipMemcpyDeviceToDevice, st));
    HIPCHK(c, hipMemsetAsync(cnt, 0, sizeof(unsigned long long) * CNT_WORDS, st));
    k_qout<<<nb, TPB, 0, st>>>(state, g, gh, q_out, n, P<int>(c->blk), cnt);
    CHECK_LAUNCH(c);
    s = scan(c, P<int>(c->blk), nb, P<int64_t>(c->blkoff), &c->n_lossless, st);
    if (s != DMT_OK) return s;
    ENSURE(c, c->ll_idx, sizeof(int64_t) * (size_t)c->n_lossless);
    ENSURE(c, c->ll_val, sizeof(float) * (size_t)c->n_lossless);
    k_lossless_write<<<nb, TPB, 0, st>>>(q_out, g, n, P<int64_t>(c->blkoff), P<int64_t>(c->ll_idx), P<float>(c->ll_val));
    CHECK_LAUNCH(c);
    s = read_counters(c, st);
    if (s != DMT_OK) return s;
    if (stats) {
        stats->iterations = it;
        stats->c_iterations = c_it;
        stats->s_iterations = s_it;
        stats->n_edited = (int64_t)c->hcnt[CNT_EDITED];
        stats->n_quantized = (int64_t)c->hcnt[CNT_QUANT];
        stats->n_lossless = (int64_t)c->hcnt[CNT_LOSSLESS];
        stats->residual_violations = residual;
        stats->converged = converged;
        stats->stalled = stalled;
    }
    return converged ? DMT_OK : DMT_W_NOT_CONVERGED;
}

}  // namespace

// ==========================================================================================
// C ABI

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
    if (hipHostMalloc((void**)&c->hcnt, sizeof(unsigned long long) * CNT_WORDS, 0) != hipSuccess ||
        hipHostMalloc((void**)&c->hctl, sizeof(Ctl), 0) != hipSuccess ||
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
    DevBuf* bufs[] = {&c->lo, &c->g, &c->state, &c->req, &c->fpl, &c->gpl, &c->cnt, &c->flags, &c->part, &c->blk,
                      &c->blkoff, &c->crit[0], &c->crit[1], &c->crit[2], &c->crit[3], &c->dsad, &c->doff, &c->dcell,
                      &c->dcbr, &c->dterm, &c->dlen, &c->dfirst, &c->asad, &c->aoff, &c->acell, &c->acbr, &c->aterm,
                      &c->alen, &c->afirst, &c->astart, &c->asadcnt, &c->asadoff, &c->vlab, &c->tlab, &c->ll_idx,
                      &c->ll_val, &c->ctl, &c->vmask, &c->inlist, &c->vl0, &c->vl1, &c->dvl0, &c->dvl1, &c->dal0,
                      &c->dal1, &c->vstamp, &c->astamp, &c->rstamp, &c->reql, &c->dlog};
    for (DevBuf* b : bufs)
        if (b->p) (void)hipFree(b->p);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->hcnt) (void)hipHostFree(c->hcnt);
    if (c->hctl) (void)hipHostFree(c->hctl);
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
    dmt_status s = check_grid(c, gr, dm, D);
    if (s != DMT_OK) return s;
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
    const bool nonfinite = h[2] != 0.0f;
    if (nonfinite) return fail(c, DMT_E_NONFINITE, "non-finite value in f");
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
    dmt_status s = check_grid(c, gr, dm, D);
    if (s != DMT_OK) return s;
    HIPCHK(c, hipSetDevice(c->device));
    ENSURE(c, c->gpl, (size_t)nplanes(D) * dm.n);
    s = launch_grad(c, D, field, P<uint8_t>(c->gpl), dm, st);
    if (s != DMT_OK) return s;
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
    dmt_status s = check_grid(c, gr, dm, D);
    if (s != DMT_OK) return s;
    HIPCHK(c, hipSetDevice(c->device));
    ENSURE(c, c->gpl, (size_t)nplanes(D) * dm.n);
    s = launch_grad(c, D, field, P<uint8_t>(c->gpl), dm, st);
    if (s != DMT_OK) return s;
    s = D == 2 ? build_msc<2>(c, P<uint8_t>(c->gpl), dm, true, st) : build_msc<3>(c, P<uint8_t>(c->gpl), dm, true, st);
    if (s != DMT_OK) return s;
    HIPCHK(c, hipStreamSynchronize(st));
    for (int k = 0; k < 32; k++) counts[k] = 0;
    for (int d = 0; d < 4; d++) counts[DMT_MSC_CRIT0 + d] = c->ncrit[d];
    counts[DMT_MSC_DESC_SADDLE] = c->n_desc;
    counts[DMT_MSC_DESC_OFFSETS] = c->n_desc + 1;
    counts[DMT_MSC_DESC_CELLS] = c->n_desc_cells;
    counts[DMT_MSC_DESC_TERMINAL] = c->n_desc;
    counts[DMT_MSC_ASC_SADDLE] = c->n_asc;
    counts[DMT_MSC_ASC_OFFSETS] = c->n_asc + 1;
    counts[DMT_MSC_ASC_CELLS] = c->n_asc_cells;
    counts[DMT_MSC_ASC_TERMINAL] = c->n_asc;
    counts[DMT_MSC_MIN_LABEL] = c->n_vlab;
    counts[DMT_MSC_MAX_LABEL] = c->n_tlab;
    return DMT_OK;
}

dmt_status dmt_msc_copy(dmt_context* c, int item, int64_t* dst, int64_t cap, hipStream_t st) {
    if (!c || !dst) return fail(c, DMT_E_INVALID, "null argument");
    if (!c->have_msc) return fail(c, DMT_E_INVALID, "no MSC extracted");
    HIPCHK(c, hipSetDevice(c->device));
    const int* src32 = nullptr;
    const int64_t* src64 = nullptr;
    int64_t n = 0;
    switch (item) {
    case DMT_MSC_CRIT0: case DMT_MSC_CRIT1: case DMT_MSC_CRIT2: case DMT_MSC_CRIT3:
        src32 = P<int>(c->crit[item]); n = c->ncrit[item]; break;
    case DMT_MSC_DESC_SADDLE:
        n = c->n_desc;
        if (n > cap) return fail(c, DMT_E_INVALID, "destination too small");
        if (n) {
            k_desc_saddles<<<nblocks(n), TPB, 0, st>>>(P<int>(c->crit[1]), n, dst);
            CHECK_LAUNCH(c);
            HIPCHK(c, hipStreamSynchronize(st));
        }
        return DMT_OK;
    case DMT_MSC_DESC_OFFSETS: src64 = P<int64_t>(c->doff); n = c->n_desc + 1; break;
    case DMT_MSC_DESC_CELLS: src32 = P<int>(c->dcell); n = c->n_desc_cells; break;
    case DMT_MSC_DESC_TERMINAL: src32 = P<int>(c->dterm); n = c->n_desc; break;
    case DMT_MSC_ASC_SADDLE: src32 = P<int>(c->asad); n = c->n_asc; break;
    case DMT_MSC_ASC_OFFSETS: src64 = P<int64_t>(c->aoff); n = c->n_asc + 1; break;
    case DMT_MSC_ASC_CELLS: src32 = P<int>(c->acell); n = c->n_asc_cells; break;
    case DMT_MSC_ASC_TERMINAL: src32 = P<int>(c->aterm); n = c->n_asc; break;
    case DMT_MSC_MIN_LABEL: src32 = P<int>(c->vlab); n = c->n_vlab; break;
    case DMT_MSC_MAX_LABEL: src32 = P<int>(c->tlab); n = c->n_tlab; break;
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
    Dims dm;
    int D;
    dmt_status s = check_grid(c, gr, dm, D);
    if (s != DMT_OK) return s;
    if (o->tier < 1 || o->tier > 4) return fail(c, DMT_E_INVALID, "tier must be 1..4");
    if (o->q_max < 0 || o->q_max > 7) return fail(c, DMT_E_INVALID, "q_max must be 0..7");
    if (o->flags & ~(uint32_t)(DMT_F_DENSE | DMT_F_PHASES)) return fail(c, DMT_E_INVALID, "unknown flags");
    if (!(xi > 0.0f) || !std::isfinite(xi)) return fail(c, DMT_E_INVALID, "xi must be finite and > 0");
    if (!(ldexpf(xi, -o->q_max) >= FLT_MIN)) return fail(c, DMT_E_INVALID, "xi / 2^q_max is not a normal float");
    HIPCHK(c, hipSetDevice(c->device));
    c->n_lossless = 0;
    return D == 2 ? correct_impl<2>(c, dm, f, g_hat, xi, o, g_out, q_out, stats, st)
                  : correct_impl<3>(c, dm, f, g_hat, xi, o, g_out, q_out, stats, st);
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
    if (kernel >= DMT_PROF_LOOP_GRAD && kernel <= DMT_PROF_LOOP_APPLY) {
        // phases inside the persistent loop: wall-clock ticks (100 MHz) recorded by the kernel
        *launches = 0;
        *units = 0;
        *ms_total = c->ctl.p ? (double)c->hctl->ph[kernel - DMT_PROF_LOOP_GRAD] * 1e-5 : 0.0;
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

}  // extern "C"
