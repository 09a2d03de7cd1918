// Agreement of two Morse-Smale complexes (Section 5.1, "Evaluation Metrics"): how many critical
// cells and separatrices of the original field f are present in another field g, from which the
// critical / separatrix recall (common / f's) and precision (common / g's) follow.
//
// Critical cells are compared by (dimension, id).  A separatrix is identified by its saddle and
// its first cell (the endpoint vertex of a descending branch, the cofacet top cell of an
// ascending one), which the geometry fixes; two separatrices with the same identity agree in
// connectivity when they end at the same extremum (or both leave through the boundary) and in
// geometry when their cell sequences are equal.  Branch lists are ordered by saddle id, then by
// first cell id, so the counterpart of a branch of f is found by binary search in g's list.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dmt {

// Entries of the ascending array a[0, na) that also occur in the ascending array b[0, nb):
// one thread per entry of a, binary search in b, one atomic per wave.
__global__ void __launch_bounds__(256) k_count_common(const int* __restrict__ a, int64_t na,
                                                      const int* __restrict__ b, int64_t nb,
                                                      unsigned long long* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool hit = false;
    if (i < na) {
        const int x = a[i];
        int64_t lo = 0, hi = nb;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (b[mid] < x) lo = mid + 1;
            else hi = mid;
        }
        hit = lo < nb && b[lo] == x;
    }
    const unsigned long long m = __ballot(hit);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(out, (unsigned long long)__popcll(m));
}

// One branch list of a complex: per-branch saddle id (nullptr: the descending form, where branch
// b belongs to saddle crit1[b / 2]), CSR offsets, cells and terminals.
struct BranchList {
    const int* sad;
    const int* crit1;
    const int64_t* off;
    const int* cell;
    const int* term;
    int64_t n;
};

__device__ __forceinline__ int branch_saddle(const BranchList& L, int64_t b) {
    return L.sad ? L.sad[b] : L.crit1[b >> 1];
}

__device__ __forceinline__ int branch_first(const BranchList& L, int64_t b) {
    return L.off[b + 1] > L.off[b] ? L.cell[L.off[b]] : -1;
}

// For every branch of F, its counterpart in G (same saddle, same first cell) if any: out[0]
// counts branches whose counterpart has the same terminal, out[1] those whose whole cell sequence
// is equal.  One wave per branch of F; the sequences are compared 64 cells at a time.
__global__ void __launch_bounds__(256) k_branch_agree(BranchList F, BranchList G, unsigned long long* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t b = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (b >= F.n) return;   // whole waves leave together: b is uniform across a wave
    const int s = branch_saddle(F, b), x = branch_first(F, b);
    int64_t lo = 0, hi = G.n;
    while (lo < hi) {   // first g-branch with key >= (s, x)
        const int64_t mid = (lo + hi) >> 1;
        const int ms = branch_saddle(G, mid);
        if (ms < s || (ms == s && branch_first(G, mid) < x)) lo = mid + 1;
        else hi = mid;
    }
    if (lo >= G.n || branch_saddle(G, lo) != s || branch_first(G, lo) != x) return;
    const int64_t gb = lo;
    const bool ends = F.term[b] == G.term[gb];
    const int64_t f0 = F.off[b], len = F.off[b + 1] - f0;
    const int64_t g0 = G.off[gb];
    bool same = ends && G.off[gb + 1] - g0 == len;
    for (int64_t k = 0; same && k < len; k += 64) {
        const bool bad = k + lane < len && F.cell[f0 + k + lane] != G.cell[g0 + k + lane];
        same = __ballot(bad) == 0;
    }
    if (lane == 0) {
        if (ends) atomicAdd(&out[0], 1ull);
        if (same) atomicAdd(&out[1], 1ull);
    }
}

}  // namespace dmt
