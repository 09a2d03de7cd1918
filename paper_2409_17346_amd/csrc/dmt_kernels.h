// Device kernels of the MSC-preserving correction (gfx950, wave64).
//
// Data layout in HBM (N = nx*ny*nz vertices, x fastest):
//   f, g_hat, g, lo        fp32[N]
//   state                  u8[N]   bits 0-2 quantized edit count q, bit 7 set once floored
//   req                    u8[N]   1 = vertex requested for an edit this iteration
//   gradient codes         u8[N][PS], anchor-major (byte p of vertex a's group is the code of
//                          the cell of plane p anchored at a, see dmt_geom.h; PS = 8 in 2D, 32
//                          in 3D), one array for f (built once) and one for g
// Every kernel is data parallel with no cross-thread ordering: requests are idempotent
// byte stores and are only consumed by a later kernel (Jacobi semantics), counters are
// reduced in LDS and added to global 64-bit counters.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "dmt_geom.h"

namespace dmt {

constexpr uint8_t CODE_CRIT = 0x00;
constexpr uint8_t CODE_UP = 0x40;
constexpr uint8_t CODE_DOWN = 0x80;
constexpr uint8_t CODE_NONE = 0xFF;
constexpr int INF32 = 0x7fffffff;

// Code planes are stored anchor-major: the codes of the cells anchored at vertex a (one per
// plane, i.e. per cell type) are bytes [a * PS, a * PS + NB) of the array, PS = 8 in 2D (NB = 6)
// and 32 in 3D (NB = 26); the other bytes are unused.  All codes of one anchor share one cache
// line (and one page), which the scattered accesses of the correction loop rely on, and a dense
// pass reads or writes one contiguous run per anchor.
template <int D>
constexpr int plane_stride() { return D == 2 ? 8 : 32; }

template <int D>
__host__ __device__ __forceinline__ size_t pidx(int p, int a) {
    return (size_t)a * plane_stride<D>() + p;
}

struct Dims {
    int nx, ny, nz, nxy, n;
    // division by nx and by nxy as a multiply-high, add and shift (set_divisors):
    // floor(v / d) = (mulhi(v, m) + v) >> l for 0 <= v < 2^31
    uint32_t mx, mxy;
    int lx, lxy;
};

// Multiplier and shift of the exact unsigned division by d >= 1 (the round-up method for
// division by invariant integers, Granlund and Montgomery 1994): l = ceil(log2 d),
// m = floor(2^32 (2^l - d) / d) + 1.  mulhi(v, m) + v stays below 2^32 for v < 2^31.
inline void div_magic(uint32_t d, uint32_t& m, int& l) {
    l = 0;
    while ((1ull << l) < d) l++;
    m = (uint32_t)((((1ull << l) - d) << 32) / d + 1);
}

inline void set_divisors(Dims& d) {
    div_magic((uint32_t)d.nx, d.mx, d.lx);
    div_magic((uint32_t)d.nxy, d.mxy, d.lxy);
}

__device__ __forceinline__ int div_by(int v, uint32_t m, int l) {
    return (int)((__umulhi((uint32_t)v, m) + (uint32_t)v) >> l);
}

// Counter block layout (one iteration): matches the public per-iteration log record.
enum {
    CNT_KIND = 0, CNT_FP0 = 1,  // FP_d = 1 + 2d, FN_d = 2 + 2d
    CNT_TM_DESC = 9, CNT_TM_ASC = 10, CNT_NREQ = 11, CNT_CHANGED = 12,
    CNT_EDITED = 13, CNT_QUANT = 14, CNT_LOSSLESS = 15,
    CNT_TM_SS = 16,   // saddle-saddle troublemakers (log word 20)
    CNT_WORDS = 17
};

__device__ __forceinline__ int c27_lin(const Dims& d, int c) {
    int dz = c / 9 - 1;
    int r = c - (dz + 1) * 9;
    int dy = r / 3 - 1;
    int dx = r - (dy + 1) * 3 - 1;
    return dx + d.nx * dy + d.nxy * dz;
}

__device__ __forceinline__ void coords(const Dims& d, int v, int& x, int& y, int& z) {
    z = div_by(v, d.mxy, d.lxy);
    int r = v - z * d.nxy;
    y = div_by(r, d.mx, d.lx);
    x = r - y * d.nx;
}

// Does the cell of plane p anchored at (x, y, z) lie inside the grid?
template <int D, int P>
__device__ __forceinline__ bool cell_exists(const Dims& d, int x, int y, int z) {
    constexpr auto& g = G<D>::g;
    return x + g.bmax[P][0] < d.nx && y + g.bmax[P][1] < d.ny && z + g.bmax[P][2] < d.nz;
}

__device__ __forceinline__ uint32_t fbits(float x) { return __float_as_uint(x); }

// a precedes b in the simulation-of-simplicity order (ties: smaller vertex id first)
__device__ __forceinline__ bool prec(float ha, int a, float hb, int b) {
    return ha < hb || (ha == hb && a < b);
}

// ----------------------------------------------------------------------------------------
// Block-level helpers

template <int NC>
__device__ __forceinline__ void block_add_counters(unsigned long long* __restrict__ gcnt, const int* cnt) {
    __shared__ unsigned long long sc[NC];
    if (threadIdx.x < NC) sc[threadIdx.x] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NC; k++)
        if (cnt[k]) atomicAdd(&sc[k], (unsigned long long)cnt[k]);
    __syncthreads();
    if (threadIdx.x < NC && sc[threadIdx.x]) atomicAdd(&gcnt[threadIdx.x], sc[threadIdx.x]);
}

// Exclusive scan of one int per thread across a block of 256 threads; returns the block total.
__device__ __forceinline__ int block_exclusive_scan(int v, int& total) {
    __shared__ int wsum[8];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    int woff = 0, tot = 0;
    const int nw = blockDim.x >> 6;
    for (int w = 0; w < nw; w++) {
        int s = wsum[w];
        if (w < wid) woff += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return woff + incl - v;
}

// ----------------------------------------------------------------------------------------
// a0: setup.  Floors lo = smallest fp32 >= f - xi, via an exact TwoSum error term; bound and
// finiteness checks; g = g_hat; state = 0.

__device__ __forceinline__ float next_up(float s) {
    uint32_t u = fbits(s);
    if (s == 0.0f) return __uint_as_float(1u);
    return __uint_as_float(s > 0.0f ? u + 1 : u - 1);
}
__device__ __forceinline__ float next_down(float s) {
    uint32_t u = fbits(s);
    if (s == 0.0f) return __uint_as_float(0x80000001u);
    return __uint_as_float(s > 0.0f ? u - 1 : u + 1);
}
// err = exact(a + b) - fl(a + b), Knuth's TwoSum (needs round-to-nearest, no contraction)
__device__ __forceinline__ float two_sum_err(float a, float b, float s) {
    float bb = s - a;
    float ab = s - bb;
    return (a - ab) + (b - bb);
}
__device__ __forceinline__ float floor_bound(float f, float xi) {
    float s = f - xi;
    float e = two_sum_err(f, -xi, s);
    return e > 0.0f ? next_up(s) : s;
}
__device__ __forceinline__ float ceil_bound(float f, float xi) {
    float s = f + xi;
    float e = two_sum_err(f, xi, s);
    return e < 0.0f ? next_down(s) : s;
}

__global__ void __launch_bounds__(256) k_setup(const float* __restrict__ f, const float* __restrict__ gh,
                                               float xi, int n, float* __restrict__ lo, float* __restrict__ g,
                                               uint8_t* __restrict__ state, uint8_t* __restrict__ req,
                                               unsigned int* __restrict__ flags) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float fi = f[i], gi = gh[i];
    unsigned int fl = 0;
    if (!isfinite(fi) || !isfinite(gi)) fl |= 1u;
    float l = floor_bound(fi, xi), h = ceil_bound(fi, xi);
    if (!(l <= gi && gi <= h)) fl |= 2u;
    if (fl) atomicOr(flags, fl);
    lo[i] = l;
    g[i] = gi;
    state[i] = 0;
    req[i] = 0;
}

__global__ void __launch_bounds__(256) k_bounds(const float* __restrict__ f, float xi, int64_t n,
                                                float* __restrict__ lo, float* __restrict__ hi) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float fi = f[i];
    lo[i] = floor_bound(fi, xi);
    hi[i] = ceil_bound(fi, xi);
}

// min / max / finiteness partials for the relative error bound
__global__ void __launch_bounds__(256) k_minmax(const float* __restrict__ f, int n, float* __restrict__ part) {
    __shared__ float smin[256], smax[256];
    __shared__ int snf[256];
    float mn = INFINITY, mx = -INFINITY;
    int nf = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        float v = f[i];
        if (!isfinite(v)) nf = 1;
        mn = fminf(mn, v);
        mx = fmaxf(mx, v);
    }
    smin[threadIdx.x] = mn; smax[threadIdx.x] = mx; snf[threadIdx.x] = nf;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            smin[threadIdx.x] = fminf(smin[threadIdx.x], smin[threadIdx.x + s]);
            smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + s]);
            snf[threadIdx.x] |= snf[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = smin[0];
        part[3 * blockIdx.x + 1] = smax[0];
        part[3 * blockIdx.x + 2] = snf[0] ? 1.0f : 0.0f;
    }
}

// ----------------------------------------------------------------------------------------
// a1 / a3: discrete gradient, one thread per vertex v, computing the pairing of every cell
// whose highest vertex is v (its lower star).  Every pair (sigma, sigma + {x}) adds a vertex x
// below all of sigma, so both cells have the same highest vertex: the lower star of v decides
// them completely from the values on v's closed 1-ring.  Rules (Section 4.2):
//   vertex v pairs with the edge to its lowest lower neighbour (else a minimum);
//   edge (v, a), a lower, not claimed by v: pairs with the triangle (v, a, b) of lowest b below a;
//   triangle (v, a, b), v > a > b: claimed by edge (v, a) if that edge chose b, else pairs with
//   the tetrahedron of lowest apex below b;  tetrahedron (v, a, b, c): claimed by its top
//   triangle (v, a, b) if that triangle chose c, else a maximum.
// Codes are scattered into the planes at the cells' anchors.

// Compile-time loop: f(std::integral_constant<int, i>) for i = B .. E-1, so table lookups
// indexed by i fold to constants (the loop bodies below index constexpr geometry tables).
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(static_cast<F&&>(f));
    }
}

// c27 code of neighbour slot SLOT relative to the anchor at slot AS (-1: v itself), as a
// compile-time constant (a static member, so uses never read the table at run time).
template <int D, int SLOT, int AS>
struct C27Rel {
    static constexpr int ax = AS < 0 ? 0 : G<D>::g.slot_d[AS < 0 ? 0 : AS][0];
    static constexpr int ay = AS < 0 ? 0 : G<D>::g.slot_d[AS < 0 ? 0 : AS][1];
    static constexpr int az = AS < 0 ? 0 : G<D>::g.slot_d[AS < 0 ? 0 : AS][2];
    static constexpr uint8_t value = (uint8_t)c27_of(G<D>::g.slot_d[SLOT][0] - ax, G<D>::g.slot_d[SLOT][1] - ay,
                                                     G<D>::g.slot_d[SLOT][2] - az);
};

// Linear id of the anchor at neighbour slot AS of v (-1: v itself).
template <int D, int AS>
__device__ __forceinline__ int anchor_at(int v, const Dims& dm) {
    if constexpr (AS < 0) {
        return v;
    } else {
        constexpr auto& g = G<D>::g;
        return v + g.slot_d[AS][0] + dm.nx * g.slot_d[AS][1] + dm.nxy * g.slot_d[AS][2];
    }
}

// With TRACK, returns whether the code of v or of a top cell of v's lower star changed (the
// cells a discrete gradient path can run through); otherwise false.
template <int D, bool TRACK = false>
__device__ __forceinline__ bool grad_vertex(const int v, const float* __restrict__ h, uint8_t* __restrict__ planes,
                                            const Dims& dm) {
    constexpr int NS = Geom<D>::NS;
    constexpr int FULL = Geom<D>::FULL;
    constexpr int NTRI = Geom<D>::NTRI;
    int x, y, z;
    coords(dm, v, x, y, z);
    const float hv = h[v];
    float hn[NS];
    uint32_t L = 0, inside = 0;
    static_for<0, NS>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        constexpr int dx = G<D>::g.slot_d[s][0], dy = G<D>::g.slot_d[s][1], dz = G<D>::g.slot_d[s][2];
        const bool ok = (unsigned)(x + dx) < (unsigned)dm.nx && (unsigned)(y + dy) < (unsigned)dm.ny &&
                        (unsigned)(z + dz) < (unsigned)dm.nz;
        inside |= (uint32_t)ok << s;
        // unconditional load (a neighbour outside the grid reads v itself) so that all loads are
        // issued together; its value is then replaced by 0 and never used (L excludes it)
        const float hs = h[ok ? v + dx + dm.nx * dy + dm.nxy * dz : v];
        hn[s] = ok ? hs : 0.0f;
        // neighbour ids below v's are in slots < FULL: they win ties
        const bool lw = s < FULL ? (hn[s] <= hv) : (hn[s] < hv);
        L |= (uint32_t)(ok && lw) << s;
    });
    // 2D with TRACK: the old codes of v and of its triangles are loaded here, beside the
    // neighbour values, rather than just before each store (where every load would wait for the
    // stores before it); a triangle outside the grid reads v's own entry, never used
    uint8_t old_v = 0;
    uint8_t old_t[NTRI];
    if constexpr (TRACK && D == 2) {
        old_v = planes[pidx<D>(0, v)];
        static_for<0, NTRI>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int s = G<D>::g.tri_s[i], t = G<D>::g.tri_t[i];
            constexpr int as = G<D>::g.tri_anchor_slot[i];
            const bool ex = ((inside >> s) & 1) && ((inside >> t) & 1);
            old_t[i] = planes[ex ? pidx<D>(G<D>::g.tri_plane[i], anchor_at<D, as>(v, dm)) : pidx<D>(0, v)];
        });
    }
    // below[s] = lower neighbours that precede neighbour s (slot order = id order)
    uint32_t below[NS];
    static_for<0, NS>([&](auto sc) { below[decltype(sc)::value] = 0; });
    static_for<0, NS>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        static_for<s + 1, NS>([&](auto tc) {
            constexpr int t = decltype(tc)::value;
            const bool tb = hn[t] < hn[s];
            below[s] |= (uint32_t)tb << t;
            below[t] |= (uint32_t)(!tb) << s;
        });
    });
    static_for<0, NS>([&](auto sc) { below[decltype(sc)::value] &= L; });

    // vertex
    int m = -1;
    uint8_t vcode = CODE_CRIT;
    static_for<0, NS>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        if (((L >> s) & 1) && below[s] == 0) { m = s; vcode = CODE_UP | C27Rel<D, s, -1>::value; }
    });
    bool changed = false;
    if constexpr (TRACK) changed = (D == 2 ? old_v : planes[pidx<D>(0, v)]) != vcode;
    planes[pidx<D>(0, v)] = vcode;

    // edges (v, s)
    int emin[NS];
    static_for<0, NS>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        emin[s] = -1;
        if (!((L >> s) & 1)) return;
        constexpr int as = G<D>::g.edge_anchor_slot[s];
        constexpr uint32_t trimask = G<D>::g.edge_trimask[s];
        uint8_t code;
        if (m == s) {
            code = CODE_DOWN | C27Rel<D, s, as>::value;
        } else {
            const uint32_t cand = trimask & below[s];
            code = CODE_CRIT;
            static_for<0, NS>([&](auto tc) {
                constexpr int t = decltype(tc)::value;
                if constexpr (((trimask >> t) & 1u) != 0u) {
                    if (((cand >> t) & 1) && (below[t] & cand) == 0) { emin[s] = t; code = CODE_UP | C27Rel<D, t, as>::value; }
                }
            });
        }
        planes[pidx<D>(G<D>::g.edge_plane[s], anchor_at<D, as>(v, dm))] = code;
    });

    // triangles (v, s, t)
    int tmin[NTRI];
    static_for<0, NTRI>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int s = G<D>::g.tri_s[i], t = G<D>::g.tri_t[i];
        tmin[i] = -1;
        if (!((L >> s) & 1) || !((L >> t) & 1)) return;
        constexpr int as = G<D>::g.tri_anchor_slot[i];
        const bool t_below_s = (below[s] >> t) & 1;   // then s is the middle vertex, t the lowest
        const bool claimed = t_below_s ? (emin[s] == t) : (emin[t] == s);
        uint8_t code;
        if (claimed) {
            code = CODE_DOWN | (t_below_s ? C27Rel<D, t, as>::value : C27Rel<D, s, as>::value);
        } else {
            code = CODE_CRIT;
            if constexpr (D == 3) {
                constexpr uint32_t tetmask = G<D>::g.tri_tetmask[i];
                const uint32_t cand = tetmask & (t_below_s ? below[t] : below[s]);
                static_for<0, NS>([&](auto uc) {
                    constexpr int u = decltype(uc)::value;
                    if constexpr (((tetmask >> u) & 1u) != 0u) {
                        if (((cand >> u) & 1) && (below[u] & cand) == 0) { tmin[i] = u; code = CODE_UP | C27Rel<D, u, as>::value; }
                    }
                });
            }
        }
        uint8_t* const dst = &planes[pidx<D>(G<D>::g.tri_plane[i], anchor_at<D, as>(v, dm))];
        if constexpr (TRACK && D == 2) changed |= old_t[i] != code;
        *dst = code;
    });

    // tetrahedra (v, s, t, u)
    if constexpr (D == 3) {
        static_for<0, Geom<D>::NTET>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int s = G<D>::g.tet_s[i], t = G<D>::g.tet_t[i], u = G<D>::g.tet_u[i];
            if (!((L >> s) & 1) || !((L >> t) & 1) || !((L >> u) & 1)) return;
            constexpr int as = G<D>::g.tet_anchor_slot[i];
            const bool t_s = (below[s] >> t) & 1, u_s = (below[s] >> u) & 1, u_t = (below[t] >> u) & 1;
            // lowest of the three, and the top triangle made of v and the other two
            int low, tm;
            uint8_t downc;
            if (u_s && u_t) { low = u; tm = tmin[G<D>::g.tri_index[s][t]]; downc = CODE_DOWN | C27Rel<D, u, as>::value; }
            else if (t_s && !u_t) { low = t; tm = tmin[G<D>::g.tri_index[s][u]]; downc = CODE_DOWN | C27Rel<D, t, as>::value; }
            else { low = s; tm = tmin[G<D>::g.tri_index[t][u]]; downc = CODE_DOWN | C27Rel<D, s, as>::value; }
            const uint8_t code = (tm == low) ? downc : CODE_CRIT;
            uint8_t* const dst = &planes[pidx<D>(G<D>::g.tet_plane[i], anchor_at<D, as>(v, dm))];
            if constexpr (TRACK) changed |= *dst != code;
            *dst = code;
        });
    }
    return changed;
}

template <int D>
__global__ void __launch_bounds__(256) k_grad(const float* __restrict__ h, uint8_t* __restrict__ planes, Dims dm) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < dm.n) grad_vertex<D>(v, h, planes, dm);
}

// ----------------------------------------------------------------------------------------
// a4: critical-cell violations (Section 4.3), one thread per anchor, every plane.
// False positive (paired in f, critical in g): request the apex of the f-pair.
// False negative (critical in f, paired in g as (sigma, sigma + {x})): request the vertex of
// sigma lowest in g among those preceding x in f; if none precedes x, request the apex of
// sigma's f-pair.  tier 1 looks at vertices and top cells only.

template <int D, int P>
__device__ __forceinline__ void classify_plane(const Dims& dm, int a, int x, int y, int z,
                                               const uint8_t* __restrict__ fpl, const uint8_t* __restrict__ gpl,
                                               const float* __restrict__ f, const float* __restrict__ gv,
                                               uint8_t* __restrict__ req, int tier, int* cnt) {
    constexpr auto& g = G<D>::g;
    constexpr int dim = g.bdim[P];
    if (tier == 1 && dim != 0 && dim != D) return;
    if (!cell_exists<D, P>(dm, x, y, z)) return;
    const uint8_t fc = fpl[pidx<D>(P, a)];
    const uint8_t gc = gpl[pidx<D>(P, a)];
    const bool fcrit = fc == CODE_CRIT, gcrit = gc == CODE_CRIT;
    if (fcrit == gcrit) return;
    int target;
    if (!fcrit) {
        target = a + c27_lin(dm, fc & 63);
        cnt[2 * dim]++;
    } else {
        const int gx = gc & 63;
        const int xv = a + c27_lin(dm, gx);
        const float fx = f[xv];
        // vertices of sigma: the whole cell (g pairs it upward) or the cell minus x
        const bool up = (gc & CODE_UP) != 0;
        int best = -1;
        float gbest = 0.0f;
        int kx = 0;
#pragma unroll
        for (int k = 0; k < g.bnv[P]; k++) {
            const int ck = c27_of(g.bvert[P][k][0], g.bvert[P][k][1], g.bvert[P][k][2]);
            if (!up && ck == gx) { kx = k; continue; }
            const int w = a + g.bvert[P][k][0] + dm.nx * g.bvert[P][k][1] + dm.nxy * g.bvert[P][k][2];
            if (!prec(f[w], w, fx, xv)) continue;
            const float gw = gv[w];
            if (best < 0 || prec(gw, w, gbest, best)) { best = w; gbest = gw; }
        }
        if (best < 0) {
            // sigma = cell minus vertex kx is paired in f: lower the apex of its f-pair
            int fa = a, fp = 0;
#pragma unroll
            for (int k = 0; k < g.bnv[P]; k++) {
                if (k == kx) {
                    fa = a + g.facet_anchor[P][k][0] + dm.nx * g.facet_anchor[P][k][1] + dm.nxy * g.facet_anchor[P][k][2];
                    fp = g.facet_plane[P][k];
                }
            }
            const uint8_t sc = fpl[pidx<D>(fp, fa)];
            best = fa + c27_lin(dm, sc & 63);
        }
        target = best;
        cnt[2 * dim + 1]++;
    }
    req[target] = 1;
}

template <int D, int P>
__device__ __forceinline__ void classify_all(const Dims& dm, int a, int x, int y, int z, const uint8_t* fpl,
                                             const uint8_t* gpl, const float* f, const float* gv, uint8_t* req,
                                             int tier, int* cnt) {
    classify_plane<D, P>(dm, a, x, y, z, fpl, gpl, f, gv, req, tier, cnt);
    if constexpr (P + 1 < Geom<D>::NB) classify_all<D, P + 1>(dm, a, x, y, z, fpl, gpl, f, gv, req, tier, cnt);
}

template <int D>
__global__ void __launch_bounds__(256) k_classify(const uint8_t* __restrict__ fpl, const uint8_t* __restrict__ gpl,
                                                  const float* __restrict__ f, const float* __restrict__ gv,
                                                  uint8_t* __restrict__ req, Dims dm, int tier,
                                                  unsigned long long* __restrict__ cnt_out) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    int cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (a < dm.n) {
        int x, y, z;
        coords(dm, a, x, y, z);
        classify_all<D, 0>(dm, a, x, y, z, fpl, gpl, f, gv, req, tier, cnt);
    }
    block_add_counters<8>(cnt_out + CNT_FP0, cnt);
}

// ----------------------------------------------------------------------------------------
// a5: Equation 2 for every requested vertex (one step per iteration).  The edited value is
// g_hat - (q+1)*Delta rounded once (fma), taken while q < q_max and it stays >= lo; otherwise
// the vertex drops to lo and is final.

__global__ void __launch_bounds__(256) k_apply(uint8_t* __restrict__ req, const float* __restrict__ gh,
                                               const float* __restrict__ lo, float* __restrict__ g,
                                               uint8_t* __restrict__ state, float delta, int q_max, int n,
                                               unsigned long long* __restrict__ cnt_out) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    int cnt[2] = {0, 0};
    if (v < n && req[v]) {
        req[v] = 0;
        cnt[0] = 1;
        const uint8_t st = state[v];
        if (!(st & 0x80)) {
            const int q = st & 7;
            const float t = fmaf(-(float)(q + 1), delta, gh[v]);
            if (q < q_max && t >= lo[v]) {
                state[v] = (uint8_t)(q + 1);
                g[v] = t;
            } else {
                state[v] = (uint8_t)(0x80 | q);
                g[v] = lo[v];
            }
            cnt[1] = 1;
        }
    }
    block_add_counters<2>(cnt_out + CNT_NREQ, cnt);
}

__global__ void __launch_bounds__(256) k_clear_u8(uint8_t* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ----------------------------------------------------------------------------------------
// a8: outputs.  q_out = q, or 0xFF for a floored vertex whose bits differ from g_hat.

__global__ void __launch_bounds__(256) k_qout(const uint8_t* __restrict__ state, const float* __restrict__ g,
                                              const float* __restrict__ gh, uint8_t* __restrict__ q_out, int n,
                                              int* __restrict__ lossless_blk, unsigned long long* __restrict__ cnt_out) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    int c[3] = {0, 0, 0};
    int ll = 0;
    if (v < n) {
        const uint8_t st = state[v];
        uint8_t q = st & 7;
        if (st & 0x80) q = fbits(g[v]) != fbits(gh[v]) ? 0xFF : 0;
        q_out[v] = q;
        if (q) c[0] = 1;
        if (q == 0xFF) { c[2] = 1; ll = 1; }
        else if (q) c[1] = 1;
    }
    block_add_counters<3>(cnt_out + CNT_EDITED, c);
    int tot;
    block_exclusive_scan(ll, tot);
    if (threadIdx.x == 0) lossless_blk[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(256) k_lossless_write(const uint8_t* __restrict__ q_out, const float* __restrict__ g,
                                                        int n, const int64_t* __restrict__ blk_off,
                                                        int64_t* __restrict__ idx, float* __restrict__ val) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    const int ll = (v < n && q_out[v] == 0xFF) ? 1 : 0;
    int tot;
    const int off = block_exclusive_scan(ll, tot);
    if (ll) {
        const int64_t k = blk_off[blockIdx.x] + off;
        if (idx) idx[k] = v;
        val[k] = g[v];
    }
}

// Per-block count of lossless entries (q_out == 0xFF) of a finished job's outputs.
__global__ void __launch_bounds__(256) k_lossless_count(const uint8_t* __restrict__ q_out, int n,
                                                        int* __restrict__ lossless_blk) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    const int ll = (v < n && q_out[v] == 0xFF) ? 1 : 0;
    int tot;
    block_exclusive_scan(ll, tot);
    if (threadIdx.x == 0) lossless_blk[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(256) k_decode(const float* __restrict__ gh, const uint8_t* __restrict__ q,
                                                int64_t n, float delta, float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint8_t qi = q[i];
    out[i] = qi == 0xFF ? gh[i] : fmaf(-(float)qi, delta, gh[i]);
}

__global__ void __launch_bounds__(256) k_scatter(const int64_t* __restrict__ idx, const float* __restrict__ val,
                                                 int64_t m, int64_t n, float* __restrict__ out,
                                                 unsigned int* __restrict__ bad) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const int64_t i = idx[k];
    if (i < 0 || i >= n) { atomicOr(bad, 1u); return; }
    out[i] = val[k];
}

// ----------------------------------------------------------------------------------------
// Exclusive scan of int -> int64 (single block, any length): out[i] = sum in[0..i), out[n] = total.

__global__ void __launch_bounds__(1024) k_scan_single(const int* __restrict__ in, int64_t n, int64_t* __restrict__ out) {
    __shared__ long long part[1024];
    const int64_t per = (n + blockDim.x - 1) / blockDim.x;
    const int64_t b = threadIdx.x * per, e = b + per < n ? b + per : n;
    long long s = 0;
    for (int64_t i = b; i < e; i++) s += in[i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long acc = 0;
        for (int i = 0; i < (int)blockDim.x; i++) { long long t = part[i]; part[i] = acc; acc += t; }
        out[n] = acc;
    }
    __syncthreads();
    long long acc = part[threadIdx.x];
    for (int64_t i = b; i < e; i++) { out[i] = acc; acc += in[i]; }
}

// Exclusive scan of int counts in tiles of 1024 (256 threads x 4 consecutive elements).
// k_tile_sum: tsum[t] = sum of tile t.  k_tile_scan, given toff = exclusive scan of tsum
// (toff[ntiles] = total): out[i] = exclusive prefix of in at i, out[n] = total; in is
// overwritten with the same offsets (fill positions for a counting sort).
__global__ void __launch_bounds__(256) k_tile_sum(const int* __restrict__ in, int n, int* __restrict__ tsum) {
    const int i0 = blockIdx.x * 1024 + threadIdx.x * 4;
    int s = 0;
#pragma unroll
    for (int k = 0; k < 4; k++)
        if (i0 + k < n) s += in[i0 + k];
    int total = 0;
    (void)block_exclusive_scan(s, total);
    if (threadIdx.x == 0) tsum[blockIdx.x] = total;
}

__global__ void __launch_bounds__(256) k_tile_scan(int* __restrict__ in, int n, const int64_t* __restrict__ toff,
                                                   int* __restrict__ out) {
    const int i0 = blockIdx.x * 1024 + threadIdx.x * 4;
    int v[4];
    int s = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        v[k] = i0 + k < n ? in[i0 + k] : 0;
        s += v[k];
    }
    int total = 0;
    int acc = (int)toff[blockIdx.x] + block_exclusive_scan(s, total);
#pragma unroll
    for (int k = 0; k < 4; k++) {
        if (i0 + k < n) {
            out[i0 + k] = acc;
            in[i0 + k] = acc;
        }
        acc += v[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = (int)toff[gridDim.x];
}

// The same with int64 offsets, leaving in untouched: out[i] = prefix of in at i, out[n] = total.
__global__ void __launch_bounds__(256) k_tile_scan64(const int* __restrict__ in, int n,
                                                     const int64_t* __restrict__ toff, int64_t* __restrict__ out) {
    const int i0 = blockIdx.x * 1024 + threadIdx.x * 4;
    int v[4];
    int s = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        v[k] = i0 + k < n ? in[i0 + k] : 0;
        s += v[k];
    }
    int total = 0;
    int64_t acc = toff[blockIdx.x] + block_exclusive_scan(s, total);
#pragma unroll
    for (int k = 0; k < 4; k++) {
        if (i0 + k < n) out[i0 + k] = acc;
        acc += v[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = toff[gridDim.x];
}

// ----------------------------------------------------------------------------------------
// MSC: critical cells (ascending ids per dimension), compacted with block scans.

template <int D, int P>
__device__ __forceinline__ void crit_count_plane(const Dims& dm, const uint8_t* __restrict__ pl, int a, int x,
                                                 int y, int z, int* c) {
    constexpr auto& g = G<D>::g;
    if (cell_exists<D, P>(dm, x, y, z) && pl[pidx<D>(P, a)] == CODE_CRIT) c[g.bdim[P]]++;
    if constexpr (P + 1 < Geom<D>::NB) crit_count_plane<D, P + 1>(dm, pl, a, x, y, z, c);
}

template <int D, int P>
__device__ __forceinline__ void crit_write_plane(const Dims& dm, const uint8_t* __restrict__ pl, int a, int x,
                                                 int y, int z, int* pos, int* const* out) {
    constexpr auto& g = G<D>::g;
    if (cell_exists<D, P>(dm, x, y, z) && pl[pidx<D>(P, a)] == CODE_CRIT) {
        constexpr int d = g.bdim[P];
        out[d][pos[d]++] = a * g.ntypes[d] + (P - g.base[d]);
    }
    if constexpr (P + 1 < Geom<D>::NB) crit_write_plane<D, P + 1>(dm, pl, a, x, y, z, pos, out);
}

template <int D>
__global__ void __launch_bounds__(256) k_crit_count(const uint8_t* __restrict__ pl, Dims dm, int* __restrict__ blk) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    int c[4] = {0, 0, 0, 0};
    if (a < dm.n) {
        int x, y, z;
        coords(dm, a, x, y, z);
        crit_count_plane<D, 0>(dm, pl, a, x, y, z, c);
    }
#pragma unroll
    for (int d = 0; d <= D; d++) {
        int tot;
        block_exclusive_scan(c[d], tot);
        if (threadIdx.x == 0) blk[(size_t)d * gridDim.x + blockIdx.x] = tot;
    }
}

template <int D>
__global__ void __launch_bounds__(256) k_crit_write(const uint8_t* __restrict__ pl, Dims dm,
                                                    const int64_t* __restrict__ blk_off, int nblk,
                                                    int* __restrict__ o0, int* __restrict__ o1,
                                                    int* __restrict__ o2, int* __restrict__ o3) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    int c[4] = {0, 0, 0, 0};
    int x = 0, y = 0, z = 0;
    if (a < dm.n) {
        coords(dm, a, x, y, z);
        crit_count_plane<D, 0>(dm, pl, a, x, y, z, c);
    }
    int pos[4] = {0, 0, 0, 0};
#pragma unroll
    for (int d = 0; d <= D; d++) {
        int tot;
        pos[d] = (int)(blk_off[(size_t)d * (nblk + 1) + blockIdx.x]) + block_exclusive_scan(c[d], tot);
    }
    int* outs[4] = {o0, o1, o2, o3};
    if (a < dm.n) crit_write_plane<D, 0>(dm, pl, a, x, y, z, pos, outs);
}

// ----------------------------------------------------------------------------------------
// MSC: V-paths.  Descending step: a vertex paired with an edge moves to that edge's other
// vertex.  Ascending step: a top cell paired with a facet moves to the facet's other top
// cofacet, or to BOUNDARY (-1) if the facet lies on the domain boundary.

template <int D>
__device__ __forceinline__ int top_id(int a, int tp) {
    constexpr auto& g = G<D>::g;
    return a * g.ntypes[D] + (tp - g.base[D]);
}

// Next top cell after top cell (a, tp) in gradient planes pl; returns false at a critical cell.
// On a boundary exit sets a = -1.
template <int D>
__device__ __forceinline__ bool asc_step(const Dims& dm, const uint8_t* __restrict__ pl, int& a, int& tp) {
    const uint8_t code = pl[pidx<D>(tp, a)];
    if (code == CODE_CRIT) return false;
    const int c = code & 63;
    int x, y, z;
    coords(dm, a, x, y, z);
    int na = -1, np = -1;
    constexpr int B0 = G<D>::g.base[D], NT = G<D>::g.ntypes[D];
    static_for<B0, B0 + NT>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        if (q != tp) return;
        static_for<0, D + 1>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            constexpr auto& g = G<D>::g;
            if (c != c27_of(g.bvert[q][k][0], g.bvert[q][k][1], g.bvert[q][k][2])) return;
            const int ax = x + g.nbr_anchor[q][k][0], ay = y + g.nbr_anchor[q][k][1], az = z + g.nbr_anchor[q][k][2];
            constexpr int p2 = g.nbr_plane[q][k];
            bool ok = ax >= 0 && ay >= 0 && az >= 0;
            if constexpr (p2 >= B0 && p2 < B0 + NT)
                ok = ok && ax + g.bmax[p2][0] < dm.nx && ay + g.bmax[p2][1] < dm.ny && az + g.bmax[p2][2] < dm.nz;
            if (ok) { na = ax + dm.nx * ay + dm.nxy * az; np = p2; }
        });
    });
    a = na;
    tp = np;
    return true;
}

// Labels: initial successor of every vertex / top cell id (self when critical).
template <int D>
__global__ void __launch_bounds__(256) k_label_init(const uint8_t* __restrict__ pl, Dims dm,
                                                    int* __restrict__ vlab, int* __restrict__ tlab) {
    constexpr auto& g = G<D>::g;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= dm.n) return;
    const uint8_t vc = pl[pidx<D>(0, a)];
    vlab[a] = vc == CODE_CRIT ? a : a + c27_lin(dm, vc & 63);
    int x, y, z;
    coords(dm, a, x, y, z);
#pragma unroll
    for (int q = g.base[D]; q < g.base[D] + g.ntypes[D]; q++) {
        const int id = top_id<D>(a, q);
        const bool ex = x + g.bmax[q][0] < dm.nx && y + g.bmax[q][1] < dm.ny && z + g.bmax[q][2] < dm.nz;
        if (!ex) { tlab[id] = -2; continue; }
        int na = a, np = q;
        if (!asc_step<D>(dm, pl, na, np)) tlab[id] = id;
        else tlab[id] = na < 0 ? -1 : top_id<D>(na, np);
    }
}

// Pointer jumping in place: lab[i] <- lab[lab[i]] (negative labels are terminal).
__global__ void __launch_bounds__(256) k_jump(int* __restrict__ lab, int64_t n, unsigned int* __restrict__ changed) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int l = lab[i];
    if (l < 0) return;
    const int l2 = lab[l];
    if (l2 != l) {
        lab[i] = l2;
        *changed = 1u;
    }
}

// second pass over the (min, max, nonfinite) triples of k_minmax
__global__ void __launch_bounds__(256) k_minmax_final(const float* __restrict__ part, int nb, float* __restrict__ out) {
    __shared__ float smin[256], smax[256], snf[256];
    float mn = INFINITY, mx = -INFINITY, nf = 0.0f;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        mn = fminf(mn, part[3 * b]);
        mx = fmaxf(mx, part[3 * b + 1]);
        nf = fmaxf(nf, part[3 * b + 2]);
    }
    smin[threadIdx.x] = mn; smax[threadIdx.x] = mx; snf[threadIdx.x] = nf;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            smin[threadIdx.x] = fminf(smin[threadIdx.x], smin[threadIdx.x + s]);
            smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + s]);
            snf[threadIdx.x] = fmaxf(snf[threadIdx.x], snf[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out[0] = smin[0]; out[1] = smax[0]; out[2] = snf[0]; }
}

// saddle of descending branch b is the critical edge b / 2
__global__ void __launch_bounds__(256) k_desc_saddles(const int* __restrict__ crit1, int64_t nbr, int64_t* __restrict__ out) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nbr) out[b] = crit1[b >> 1];
}

__global__ void __launch_bounds__(256) k_i32_to_i64(const int* __restrict__ in, int64_t n, int64_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i];
}

// Descending branches: for each critical edge (sorted), endpoints in id order.
// mode 0: length (vertices incl. both ends) and terminal; mode 1: write the sequence.
template <int D>
__global__ void __launch_bounds__(256) k_desc_walk(const uint8_t* __restrict__ pl, Dims dm, const int* __restrict__ sad,
                                                   int nbr, int mode, int* __restrict__ len, int* __restrict__ term,
                                                   const int64_t* __restrict__ off, int* __restrict__ cells,
                                                   int* __restrict__ cell_branch, unsigned int* __restrict__ err) {
    constexpr auto& g = G<D>::g;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbr) return;
    const int e = sad[b >> 1];
    const int a = e / g.ntypes[1];
    const int t = e - a * g.ntypes[1];
    int v = a;
    if (b & 1) {
#pragma unroll
        for (int q = 0; q < g.ntypes[1]; q++)
            if (q == t) {
                        v = a + g.bvert[g.base[1] + q][1][0] + dm.nx * g.bvert[g.base[1] + q][1][1] +
                    dm.nxy * g.bvert[g.base[1] + q][1][2];
            }
    }
    int64_t k = mode ? off[b] : 0;
    int n = 0;
    // a V-path visits every vertex at most once; the cap only guards against corrupt codes
    for (;;) {
        if (mode) { cells[k] = v; cell_branch[k] = b; k++; }
        n++;
        const uint8_t c = pl[pidx<D>(0, v)];
        if (c == CODE_CRIT) break;
        if (n >= dm.n) { atomicOr(err, 4u); break; }
        v += c27_lin(dm, c & 63);
    }
    if (!mode) { len[b] = n; term[b] = v; }
}

// Ascending branch starts: for each critical (D-1)-cell (sorted), its existing top cofacets
// in id order.  mode 0: count per saddle; mode 1: write branch start ids and saddles.
template <int D>
__global__ void __launch_bounds__(256) k_asc_starts(Dims dm, const int* __restrict__ sad, int nsad, int mode,
                                                    int* __restrict__ cnt, const int64_t* __restrict__ off,
                                                    int* __restrict__ start, int* __restrict__ bsad) {
    constexpr auto& g = G<D>::g;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsad) return;
    const int s = sad[i];
    const int T1 = g.ntypes[D - 1];
    const int a = s / T1;
    const int t = s - a * T1;
    int x, y, z;
    coords(dm, a, x, y, z);
    int ids[2] = {0, 0};
    int n = 0;
#pragma unroll
    for (int q = g.base[D - 1]; q < g.base[D - 1] + g.ntypes[D - 1]; q++) {
        if (q - g.base[D - 1] != t) continue;
#pragma unroll
        for (int j = 0; j < 2; j++) {
            const int ax = x + g.cof_anchor[q][j][0], ay = y + g.cof_anchor[q][j][1], az = z + g.cof_anchor[q][j][2];
            const int p2 = g.cof_plane[q][j];
            bool ok = ax >= 0 && ay >= 0 && az >= 0;
#pragma unroll
            for (int r = g.base[D]; r < g.base[D] + g.ntypes[D]; r++)
                if (r == p2) ok = ok && ax + g.bmax[r][0] < dm.nx && ay + g.bmax[r][1] < dm.ny && az + g.bmax[r][2] < dm.nz;
            if (ok) ids[n++] = top_id<D>(ax + dm.nx * ay + dm.nxy * az, p2);
        }
    }
    if (n == 2 && ids[1] < ids[0]) { int tmp = ids[0]; ids[0] = ids[1]; ids[1] = tmp; }
    if (!mode) { cnt[i] = n; return; }
    for (int j = 0; j < n; j++) { start[off[i] + j] = ids[j]; bsad[off[i] + j] = s; }
}

template <int D>
__global__ void __launch_bounds__(256) k_asc_walk(const uint8_t* __restrict__ pl, Dims dm, const int* __restrict__ start,
                                                  int nbr, int mode, int* __restrict__ len, int* __restrict__ term,
                                                  const int64_t* __restrict__ off, int* __restrict__ cells,
                                                  int* __restrict__ cell_branch, unsigned int* __restrict__ err) {
    constexpr auto& g = G<D>::g;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbr) return;
    const int T0 = start[b];
    int a = T0 / g.ntypes[D];
    int tp = T0 - a * g.ntypes[D] + g.base[D];
    int64_t k = mode ? off[b] : 0;
    int n = 0;
    int terminal;
    const int cap = dm.n * g.ntypes[D];
    for (;;) {
        const int id = top_id<D>(a, tp);
        if (mode) { cells[k] = id; cell_branch[k] = b; k++; }
        n++;
        if (!asc_step<D>(dm, pl, a, tp)) { terminal = id; break; }
        if (a < 0) { terminal = -1; break; }
        if (n >= cap) { atomicOr(err, 4u); terminal = -1; break; }
    }
    if (!mode) { len[b] = n; term[b] = terminal; }
}

// ----------------------------------------------------------------------------------------
// a6: S-step (Section 4.4).  Along every f-branch, the first cell whose g pairing differs from
// its f pairing is the troublemaker; the apex of its f-pair is requested.  Tier 3 keeps only
// branches whose g-path ends elsewhere than the f-path.

template <int D>
__global__ void __launch_bounds__(256) k_scheck_desc(const uint8_t* __restrict__ fpl, const uint8_t* __restrict__ gpl,
                                                     const int* __restrict__ cells, const int* __restrict__ cbr,
                                                     int64_t ncell, int* __restrict__ first) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ncell) return;
    const int v = cells[k];
    if (fpl[pidx<D>(0, v)] != gpl[pidx<D>(0, v)]) atomicMin(&first[cbr[k]], (int)k);
}

template <int D>
__global__ void __launch_bounds__(256) k_scheck_asc(const uint8_t* __restrict__ fpl, const uint8_t* __restrict__ gpl,
                                                    Dims dm, const int* __restrict__ cells, const int* __restrict__ cbr,
                                                    int64_t ncell, int* __restrict__ first) {
    constexpr auto& g = G<D>::g;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ncell) return;
    const int T = cells[k];
    const int a = T / g.ntypes[D];
    const int tp = T - a * g.ntypes[D] + g.base[D];
    const size_t o = pidx<D>(tp, a);
    if (fpl[o] != gpl[o]) atomicMin(&first[cbr[k]], (int)k);
}

template <int D>
__global__ void __launch_bounds__(256) k_starget(const uint8_t* __restrict__ fpl, const uint8_t* __restrict__ gpl,
                                                 Dims dm, int asc, const int* __restrict__ cells,
                                                 const int64_t* __restrict__ off, const int* __restrict__ term,
                                                 int nbr, int* __restrict__ first, int tier, uint8_t* __restrict__ req,
                                                 unsigned long long* __restrict__ cnt_out) {
    constexpr auto& g = G<D>::g;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    int c = 0;
    if (b < nbr && first[b] != INF32) {
        const int k = first[b];
        first[b] = INF32;
        bool ok = true;
        if (tier == 3) {
            // terminal of the g-path from the branch start
            int gt;
            if (!asc) {
                int v = cells[off[b]];
                for (int step = 0; step < dm.n; step++) {
                    const uint8_t cc = gpl[pidx<D>(0, v)];
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
                    if (!asc_step<D>(dm, gpl, a, tp)) { gt = id; break; }
                    if (a < 0) { gt = -1; break; }
                }
            }
            ok = gt != term[b];
        }
        if (ok) {
            int target;
            if (!asc) {
                const int v = cells[k];
                target = v + c27_lin(dm, fpl[pidx<D>(0, v)] & 63);
            } else {
                const int T = cells[k];
                const int a = T / g.ntypes[D];
                const int tp = T - a * g.ntypes[D] + g.base[D];
                target = a + c27_lin(dm, fpl[pidx<D>(tp, a)] & 63);
            }
            req[target] = 1;
            c = 1;
        }
    }
    block_add_counters<1>(cnt_out + (asc ? CNT_TM_ASC : CNT_TM_DESC), &c);
}

// ----------------------------------------------------------------------------------------
// Export of the gradient as cell-id pairs (test and inspection aid).

template <int D, int P>
__device__ __forceinline__ void export_plane(const Dims& dm, const uint8_t* __restrict__ pl, int a, int x, int y,
                                             int z, const int64_t* offs, int64_t* __restrict__ up,
                                             int64_t* __restrict__ down) {
    constexpr auto& g = G<D>::g;
    constexpr int d = g.bdim[P];
    const int64_t id = (int64_t)a * g.ntypes[d] + (P - g.base[d]);
    int64_t u = -1, w = -1;
    if (cell_exists<D, P>(dm, x, y, z)) {
        const uint8_t c = pl[pidx<D>(P, a)];
        const int cc = c & 63;
        if (c != CODE_CRIT && (c & CODE_UP)) {
#pragma unroll
            for (int j = 0; j < g.ncofall[P]; j++) {
                if (g.cofall_apex[P][j] != cc) continue;
                const int na = a + g.cofall_anchor[P][j][0] + dm.nx * g.cofall_anchor[P][j][1] +
                               dm.nxy * g.cofall_anchor[P][j][2];
                constexpr int d1 = d + 1 <= D ? d + 1 : D;
                u = (int64_t)na * g.ntypes[d1] + (g.cofall_plane[P][j] - g.base[d1]);
            }
        } else if (c != CODE_CRIT) {
#pragma unroll
            for (int k = 0; k < g.bnv[P]; k++) {
                if (c27_of(g.bvert[P][k][0], g.bvert[P][k][1], g.bvert[P][k][2]) != cc) continue;
                const int na = a + g.facet_anchor[P][k][0] + dm.nx * g.facet_anchor[P][k][1] +
                               dm.nxy * g.facet_anchor[P][k][2];
                constexpr int d0 = d > 0 ? d - 1 : 0;
                w = (int64_t)na * g.ntypes[d0] + (g.facet_plane[P][k] - g.base[d0]);
            }
        }
    }
    up[offs[d] + id] = u;
    down[offs[d] + id] = w;
    if constexpr (P + 1 < Geom<D>::NB) export_plane<D, P + 1>(dm, pl, a, x, y, z, offs, up, down);
}

template <int D>
__global__ void __launch_bounds__(256) k_export(const uint8_t* __restrict__ pl, Dims dm, int64_t o1, int64_t o2,
                                                int64_t o3, int64_t* __restrict__ up, int64_t* __restrict__ down) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= dm.n) return;
    int x, y, z;
    coords(dm, a, x, y, z);
    const int64_t offs[4] = {0, o1, o2, o3};
    export_plane<D, 0>(dm, pl, a, x, y, z, offs, up, down);
}

}  // namespace dmt
