// Quantized edit stream (Section 4.7, "Quantized Representation of Edits"): every vertex's edit
// count q in 0..q_max, or the lossless marker, stored in a fixed number of bits, so the stream is
// a dense bitmap of the field; the values of the lossless vertices follow in vertex order (their
// positions are the marked codes, so no index is stored).
//
// Code of a vertex: q (0..q_max), or q_max + 1 for a lossless vertex (q_out == 0xFF).  Bits per
// code: the least b with 2^b >= q_max + 2 (q_max 6 -> 3 bits).  Code k occupies bits
// [k*b, (k+1)*b) of the stream, little-endian within 32-bit words; a code may straddle two words.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dmt {

__host__ __device__ constexpr int edit_bits(int q_max) {
    int b = 1;
    while ((1 << b) < q_max + 2) b++;
    return b;
}

// One thread per output word: gathers the (at most 32) codes whose bits overlap word w.
__global__ void __launch_bounds__(256) k_pack_edits(const uint8_t* __restrict__ q, int64_t n, int q_max, int b,
                                                    int64_t n_words, uint32_t* __restrict__ out,
                                                    unsigned* __restrict__ bad) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= n_words) return;
    const int64_t bit0 = w * 32;
    const int64_t k0 = bit0 / b;
    const int64_t k1 = (bit0 + 31) / b;   // last code touching the word
    uint32_t word = 0;
    for (int64_t k = k0; k <= k1 && k < n; k++) {
        const uint8_t qk = q[k];
        if (qk > q_max && qk != 0xFF) atomicOr(bad, 1u);
        const uint32_t code = qk == 0xFF ? (uint32_t)(q_max + 1) : (uint32_t)qk;
        const int64_t sh = k * b - bit0;   // position of the code's lowest bit in this word
        if (sh >= 0) word |= code << sh;
        else word |= code >> (-sh);
    }
    out[w] = word;
}

// Code of vertex v from the stream (a 64-bit window over the one or two words it touches).
__device__ __forceinline__ uint32_t edit_code(const uint32_t* __restrict__ s, int64_t n_words, int64_t v, int b) {
    const int64_t bit = v * b;
    const int64_t w = bit >> 5;
    const uint64_t lo = s[w];
    const uint64_t hi = w + 1 < n_words ? s[w + 1] : 0;
    return (uint32_t)(((hi << 32 | lo) >> (bit & 31)) & ((1u << b) - 1));
}

// Per-block count of lossless codes (blocks of 256 vertices), for their positions in the value list.
__global__ void __launch_bounds__(256) k_unpack_count(const uint32_t* __restrict__ s, int64_t n_words, int n, int q_max,
                                                      int b, int* __restrict__ blk, unsigned* __restrict__ bad) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    int ll = 0;
    if (v < n) {
        const uint32_t c = edit_code(s, n_words, v, b);
        ll = c == (uint32_t)(q_max + 1);
        if (c > (uint32_t)(q_max + 1)) atomicOr(bad, 1u);
    }
    int tot;
    block_exclusive_scan(ll, tot);
    if (threadIdx.x == 0) blk[blockIdx.x] = tot;
}

// Decoder: g = g_hat - q * xi / 2^q_max rounded once (Equation 2), or the next lossless value;
// q_out (optional) gets the edit counts as dmt_correct writes them.
__global__ void __launch_bounds__(256) k_unpack_write(const uint32_t* __restrict__ s, int64_t n_words, int n,
                                                      int q_max, int b, const float* __restrict__ gh,
                                                      const float* __restrict__ val, const int64_t* __restrict__ blkoff,
                                                      int64_t n_val, float delta, float* __restrict__ g,
                                                      uint8_t* __restrict__ q_out, unsigned* __restrict__ bad) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t c = 0;
    if (v < n) c = edit_code(s, n_words, v, b);
    const int ll = v < n && c == (uint32_t)(q_max + 1);
    int tot;
    const int off = block_exclusive_scan(ll, tot);
    if (v >= n) return;
    if (ll) {
        const int64_t k = blkoff[blockIdx.x] + off;
        if (k >= n_val) {
            atomicOr(bad, 2u);
            g[v] = gh[v];
        } else {
            g[v] = val[k];
        }
    } else {
        g[v] = fmaf(-(float)c, delta, gh[v]);
    }
    if (q_out) q_out[v] = ll ? (uint8_t)0xFF : (uint8_t)c;
}

}  // namespace dmt
