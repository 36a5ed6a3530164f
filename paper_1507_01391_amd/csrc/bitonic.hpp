// Register-resident bitonic building blocks for one wavefront holding 64 x 64 items
// (lane L, register c), and conflict-free LDS layout moves between such layouts.
// Used by the tile sort (sort.hip) and the run merge (merge.hip).
#pragma once

#include "common.hpp"

namespace ts {
namespace bt {

constexpr int R = 64;  // registers (columns) per lane

// Keep the instruction scheduler from interleaving consecutive network stages: each
// stage rewrites all 64 registers in place, and interleaving keeps old and new copies
// alive at once (register pressure above 256 and a single wave per SIMD).
TS_DEV void stage_fence() {}

// Composites are 64-bit integers below 2^62.  Read as IEEE doubles such bit patterns are
// non-negative and finite (subnormal below 2^52) and order exactly like the integers, so
// the smaller and larger of two composites are one v_min_f64 and one v_max_f64 each:
// two instructions per compare-exchange where a 64-bit integer compare and four 32-bit
// selects take five.  No rounding is involved (min and max return one operand's bits)
// and the kernels keep fp64 subnormals (the default float mode), so the bits come back
// unchanged.  Written as assembly: the compiler's own min and max first quiet possible
// signalling NaNs, one more instruction per operand.
constexpr uint64_t COMP_MASK = (uint64_t(1) << 62) - 1;  // x ^ COMP_MASK reverses the order

TS_DEV uint64_t comp_min(uint64_t a, uint64_t b) {
    uint64_t r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
TS_DEV uint64_t comp_max(uint64_t a, uint64_t b) {
    uint64_t r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

TS_DEV void cas(uint64_t& a, uint64_t& b) {  // afterwards a <= b
    const uint64_t lo = comp_min(a, b), hi = comp_max(a, b);
    a = lo;
    b = hi;
}

// One stage of a bitonic network on the register index: pairs (i, i ^ J); ascending
// where bit K of i is clear (K = 0: everywhere ascending).  The networks below are
// spelled out by template recursion so that every register index is a compile-time
// constant (a partially unrolled loop would index the register array at run time and
// put it in scratch memory).
template <int K, int J>
TS_DEV void net_stage(uint64_t (&v)[R]) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int l = i ^ J;
        if (l > i) {
            if (K == 0 || (i & K) == 0) cas(v[i], v[l]);
            else cas(v[l], v[i]);
        }
    }
}

// Stages J, J/2, .. 1 with direction bit K.
template <int K, int J>
TS_DEV void net_stages(uint64_t (&v)[R]) {
    net_stage<K, J>(v);
    stage_fence();
    if constexpr (J > 1) net_stages<K, J / 2>(v);
}

// Levels K, 2K, .. R of a bitonic sort on the register index.
template <int K>
TS_DEV void net_levels(uint64_t (&v)[R]) {
    net_stages<(K < R ? K : 0), K / 2>(v);
    if constexpr (K < R) net_levels<2 * K>(v);
}

// Ascending bitonic sort of the 64 registers of every lane (672 compare-exchanges).
TS_DEV void row_sort(uint64_t (&v)[R]) { net_levels<2>(v); }

// Ascending bitonic merge of the 64 registers of every lane (stages 32 .. 1).
TS_DEV void row_merge(uint64_t (&v)[R]) { net_stages<0, R / 2>(v); }

// Stages j = 2^(KB-1) .. 1 of bitonic level 2^KB on the register index, direction
// given by bit KB of the register index (ascending when clear).
template <int KB>
TS_DEV void reg_level_stages(uint64_t (&v)[R]) {
    net_stages<(KB < 6 ? (1 << KB) : 0), (1 << (KB - 1))>(v);
}

TS_DEV void xor_all(uint64_t (&v)[R], uint64_t m) {
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] ^= m;
}

enum Move : int { MOVE_NONE = 0, MOVE_T = 1, MOVE_RM2CM = 2, MOVE_CM2RM = 3 };

// Destination (lane, register) of register c of lane L, and the slot skew h(c').
TS_DEV void move_dst(int move, int L, int c, int& Ld, int& cd) {
    if (move == MOVE_T) {
        Ld = c;
        cd = L;
    } else if (move == MOVE_RM2CM) {  // super-row of 8 rows: row-major p = 64 i + c
        Ld = (L & ~7) + (c & 7);
        cd = 8 * (L & 7) + (c >> 3);
    } else {  // MOVE_CM2RM: column-major p = 8 c + i
        Ld = (L & ~7) + (c >> 3);
        cd = 8 * (c & 7) + (L & 7);
    }
}
TS_DEV int move_skew(int move, int cd) {
    return move == MOVE_T ? cd : (move == MOVE_RM2CM ? (cd >> 3) : (cd & 7));
}

// Words of the LDS array a layout move needs (16.25 KiB).
constexpr int MOVE_WORDS = 64 * 65;

// Apply a layout move through the LDS array A (MOVE_WORDS words).  One wave.
// The 64-bit composites travel as two 32-bit planes (high words, then low words)
// through the same array, which halves the LDS a wavefront needs.  In every 32-lane
// phase of every 32-bit write and read the word addresses are distinct modulo 32, so
// no instruction has a bank conflict:
//  * the transpose stores (L', c') at word 65 c' + L' (a row pitch of 65 words skews
//    row c' by c' banks); a lane's 64 writes and 64 reads are then one base address
//    plus immediate offsets;
//  * the super-row moves store (L', c') at word 64 c' + ((L' + h(c')) mod 64) with the
//    per-move skew h of move_skew.
TS_DEV void layout_move(uint32_t* A, uint64_t (&v)[R], int move, int lane_in) {
#pragma unroll
    for (int half = 1; half >= 0; --half) {
        wave_lds_fence();  // earlier reads of A (other lanes' slots) stay before these writes
        // a fresh opaque copy per plane: addresses are recomputed next to their use
        // instead of being kept live across both planes
        const int lane = (int)opaque((uint32_t)lane_in);
        if (move == MOVE_T) {
#pragma unroll
            for (int c = 0; c < R; ++c)
                lds_store(A, (uint32_t)(65 * lane + c) * 4u, half ? hi32(v[c]) : lo32(v[c]));
        } else {
#pragma unroll
            for (int c = 0; c < R; ++c) {
                int Ld, cd;
                move_dst(move, lane, c, Ld, cd);
                const uint32_t slot = (uint32_t)(cd * 64 + ((Ld + move_skew(move, cd)) & 63));
                lds_store(A, slot * 4u, half ? hi32(v[c]) : lo32(v[c]));
            }
        }
        wave_lds_fence();  // the reads below see every lane's writes
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const uint32_t slot = (move == MOVE_T)
                                      ? (uint32_t)(65 * c + lane)
                                      : (uint32_t)(c * 64 + ((lane + move_skew(move, c)) & 63));
            const uint32_t w = lds_load(A, slot * 4u);
            v[c] = half ? pack(w, lo32(v[c])) : pack(hi32(v[c]), w);
        }
    }
    wave_lds_fence();  // later writes of A stay after these reads
}

// Lanes whose bit `b` is set get an all-ones mask (complemented composites sort in
// the reverse order).
TS_DEV uint64_t lane_bit_mask(int lane, int b) { return ((lane >> b) & 1) ? COMP_MASK : 0ull; }

// Level 2^(6+KB) of the bitonic sort below (KB = 1 .. 6).
template <int KB>
TS_DEV void bitonic_level(uint32_t* A, uint64_t (&v)[R], int lane) {
    layout_move(A, v, MOVE_T, lane);  // lane bits become register bits
    reg_level_stages<KB>(v);
    layout_move(A, v, MOVE_T, lane);  // back: register bits
    const uint64_t m = (KB < 6) ? lane_bit_mask(lane, KB) : 0ull;
    xor_all(v, m);
    row_merge(v);
    xor_all(v, m);
    if constexpr (KB < 6) bitonic_level<KB + 1>(A, v, lane);
}

// Batcher's bitonic sort of the 4096 composites of one wavefront.  On entry register c
// of lane L holds any item; on exit register c of lane L holds rank 64 c + L.  Stages
// on register bits run in registers; stages on lane bits run in registers after a
// conflict-free transpose through A.
TS_DEV void bitonic_sort4096(uint32_t* A, uint64_t (&v)[R], int lane) {
    // levels 2 .. 64: rows (lanes) sorted, odd rows descending
    xor_all(v, lane_bit_mask(lane, 0));
    row_sort(v);
    xor_all(v, lane_bit_mask(lane, 0));
    bitonic_level<1>(A, v, lane);     // levels 128 .. 4096
    layout_move(A, v, MOVE_T, lane);  // to store order
}

// Bitonic merge of one wavefront's 4096 composites.  On entry register c of lane L
// holds element 64 c + L of a bitonic sequence; on exit it holds rank 64 c + L.
// Stages 2048 .. 64 compare registers; stages 32 .. 1 compare registers after a
// transpose.
TS_DEV void bitonic_merge4096(uint32_t* A, uint64_t (&v)[R], int lane) {
    row_merge(v);
    layout_move(A, v, MOVE_T, lane);
    row_merge(v);
    layout_move(A, v, MOVE_T, lane);
}

// ---------------------------------------------------------------------------------
// Tiles spread over H wavefronts of one workgroup (H = 2, 4, 8): every wavefront holds
// 4096 items in its 64 registers x 64 lanes.

// Registers per exchange round of cross_wave_stage.
constexpr int XCH = 32;

// Compare-exchange of every register with the same register of wavefront hp (same
// lane): the wavefront with the lower index keeps the smaller composite when `asc`.
// XCH registers at a time go through LDS as 64-bit words, lane L of wavefront h at
// slot (XCH h + j) 64 + L of X (XCH H x 64 slots): 16 (writes) or 32 (reads)
// consecutive 8-byte slots per phase, no bank conflicts; two rounds of two barriers
// each.  All H wavefronts take part.
TS_DEV void cross_wave_stage(uint64_t* X, uint64_t (&v)[R], int h, int hp, bool asc, int lane) {
    const bool keep_min = (h < hp) == asc;
#pragma unroll
    for (int g = 0; g < R; g += XCH) {
        __syncthreads();  // earlier readers of X are done
#pragma unroll
        for (int j = 0; j < XCH; ++j) X[(XCH * h + j) * 64 + lane] = v[g + j];
        __syncthreads();
#pragma unroll
        for (int j0 = 0; j0 < XCH; j0 += 16) {  // 16 partner registers in flight at a time
            uint64_t y[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) y[j] = X[(XCH * hp + j0 + j) * 64 + lane];
            if (keep_min) {  // wave-uniform
#pragma unroll
                for (int j = 0; j < 16; ++j) v[g + j0 + j] = comp_min(v[g + j0 + j], y[j]);
            } else {
#pragma unroll
                for (int j = 0; j < 16; ++j) v[g + j0 + j] = comp_max(v[g + j0 + j], y[j]);
            }
        }
    }
}

// Words of LDS the wide bitonic sort needs: one transpose array per wavefront (the
// exchange buffer of cross_wave_stage, XCH H x 64 x 2 words, fits in it).
template <int H>
constexpr int wide_bitonic_words() {
    static_assert(XCH * H * 64 * 2 <= H * MOVE_WORDS, "the exchange buffer fits the transpose arrays");
    return H * MOVE_WORDS;
}

// Batcher's bitonic sort of 4096 H composites held by H wavefronts (wavefront h = the
// item indices 4096 h .. 4096 h + 4095).  Every wavefront sorts its own 4096 items
// (descending in odd wavefronts); each further level compares across wavefronts on the
// wavefront bits and finishes inside each wavefront with the 12 merge stages of
// bitonic_merge4096.  On exit register c of lane L in wavefront h holds rank
// 4096 h + 64 c + L.  A: wide_bitonic_words<H>() words, wavefront h uses its own
// MOVE_WORDS part for the transposes.
template <int H>
TS_DEV void bitonic_sort_wide(uint32_t* A, uint64_t (&v)[R], int h, int lane) {
    uint64_t* X = (uint64_t*)A;
    uint32_t* Aw = A + h * MOVE_WORDS;
    const uint64_t m0 = (h & 1) ? COMP_MASK : 0ull;
    xor_all(v, m0);
    bitonic_sort4096(Aw, v, lane);
    xor_all(v, m0);
#pragma unroll
    for (int k = 1; (1 << k) <= H; ++k) {
        // level 4096 * 2^k: blocks of 2^k wavefronts, ascending where bit k of h is clear
        const bool asc = ((h >> k) & 1) == 0;
#pragma unroll
        for (int b = k - 1; b >= 0; --b) cross_wave_stage(X, v, h, h ^ (1 << b), asc, lane);
        __syncthreads();  // the exchange buffer overlaps the transpose arrays
        const uint64_t m = asc ? 0ull : COMP_MASK;
        xor_all(v, m);
        bitonic_merge4096(Aw, v, lane);
        xor_all(v, m);
    }
}

}  // namespace bt
}  // namespace ts
