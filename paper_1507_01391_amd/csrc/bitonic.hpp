// Register-resident bitonic building blocks for one wavefront holding 64 x 64 items
// (lane L, register c), and conflict-free LDS layout moves between such layouts.
// Used by the tile sort (sort.hip) and the run merge (merge.hip).
#pragma once

#include "common.hpp"

namespace ts {
namespace bt {

constexpr int R = 64;  // registers (columns) per lane

// A 32-bit LDS read that the compiler does not pair with its neighbour into one
// two-word read: such a pair lands in two adjacent registers, and moving the words into
// the halves of the 64-bit composites they belong to cost about one extra move and one
// address add per word (19 % of the sorting kernels' VALU instructions); a volatile
// access to the LDS address space is issued as it stands.
TS_DEV uint32_t lds_load_single(const uint32_t* base, uint32_t byte_off) {
    typedef __attribute__((address_space(3))) volatile const uint32_t lds_word;
    return *(lds_word*)((__attribute__((address_space(3))) const char*)base + byte_off);
}

// Composites are 64-bit integers below 2^62.  Read as IEEE doubles such bit patterns are
// non-negative and finite (subnormal below 2^52) and order exactly like the integers, so
// the smaller and larger of two composites are one v_min_f64 and one v_max_f64 each:
// two instructions per compare-exchange where a 64-bit integer compare and four 32-bit
// selects take five.  No rounding is involved (min and max return one operand's bits)
// and the kernels keep fp64 subnormals (the default float mode), so the bits come back
// unchanged.  Written as assembly: the compiler's own min and max first quiet possible
// signalling NaNs, one more instruction per operand.
constexpr uint64_t COMP_MASK = (uint64_t(1) << 62) - 1;  // x ^ COMP_MASK reverses the order
#if defined(__FAST_MATH__)
#error "the fp64 min/max compare-exchange needs fp64 subnormals kept: build without fast math"
#endif

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
            const uint32_t w = lds_load_single(A, slot * 4u);
            v[c] = half ? pack(w, lo32(v[c])) : pack(hi32(v[c]), w);
        }
    }
    wave_lds_fence();  // later writes of A stay after these reads
}

// The transposes of the bitonic sort below, with lane reversal: in the transposed
// layout register r (a row) keeps column c at lane c, or at lane 63 - c when bit KB-1
// of r is set (the upper half of every block of 2^KB rows).  TO_ROWS = false: from the
// row layout (lane = row, register = column) to that layout; true: back.  The reversal
// only changes which lane-dependent base an access adds its immediate offset to
// (lane or 63 - lane), and a 32-lane phase still touches 32 consecutive words of one
// row (reads) or words 65 apart (writes): no bank conflicts, no extra instructions.
template <int KB, bool TO_ROWS>
TS_DEV void transpose_rev(uint32_t* A, uint64_t (&v)[R], int lane_in) {
#pragma unroll
    for (int half = 1; half >= 0; --half) {
        wave_lds_fence();  // earlier reads of A (other lanes' slots) stay before these writes
        const int lane = (int)opaque((uint32_t)lane_in);
        const int rlane = 63 - lane;
#pragma unroll
        for (int c = 0; c < R; ++c) {
            // writer: row layout (lane = row, register c = column) or the reversed layout
            // (register c = row c, this lane = column lane or 63 - lane)
            const int base = (TO_ROWS && ((c >> (KB - 1)) & 1)) ? rlane : lane;
            lds_store(A, (uint32_t)(65 * base + c) * 4u, half ? hi32(v[c]) : lo32(v[c]));
        }
        wave_lds_fence();  // the reads below see every lane's writes
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const int base = (!TO_ROWS && ((c >> (KB - 1)) & 1)) ? rlane : lane;
            const uint32_t w = lds_load_single(A, (uint32_t)(65 * c + base) * 4u);
            v[c] = half ? pack(w, lo32(v[c])) : pack(hi32(v[c]), w);
        }
    }
    wave_lds_fence();  // later writes of A stay after these reads
}

// Level 2^(6+KB) of the bitonic sort below (KB = 1 .. 6) in the form whose first stage
// compares every item with its mirror image in the block (item i of a block of B
// against item B-1-i) and whose later stages all sort ascending, so that no row is
// sorted descending and no composite is complemented.  Item index 64 r + c (row r =
// lane, column c = register).  In the lane-reversed transposed layout the mirror of
// (row r, column c), (row r ^ (2^KB - 1), column 63 - c), sits at the same lane.
template <int KB>
TS_DEV void bitonic_level(uint32_t* A, uint64_t (&v)[R], int lane) {
    transpose_rev<KB, false>(A, v, lane);            // rows become registers
    net_stage<0, (1 << KB) - 1>(v);                  // mirror stage on the row bits
    if constexpr (KB >= 2) net_stages<0, (1 << (KB - 2))>(v);  // the other row-bit stages
    transpose_rev<KB, true>(A, v, lane);             // back: columns are registers
    row_merge(v);                                    // column-bit stages 32 .. 1
    if constexpr (KB < 6) bitonic_level<KB + 1>(A, v, lane);
}

// Batcher's bitonic sort of the 4096 composites of one wavefront.  On entry register c
// of lane L holds any item; on exit register c of lane L holds rank 64 c + L.  Stages
// on register bits run in registers; stages on lane bits run in registers after a
// conflict-free transpose through A.
TS_DEV void bitonic_sort4096(uint32_t* A, uint64_t (&v)[R], int lane) {
    row_sort(v);                      // levels 2 .. 64: every row ascending
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

// First stage of a level of the wide sort in mirror form: item i of wavefront h
// (i = 64 c + L) against item 4095 - i of wavefront hp (register 63 - c, lane 63 - L);
// the wavefront with the lower index keeps the smaller composite.  Registers go through
// X in two exchange rounds of 32 registers closed under c -> 63 - c (the first takes
// c < 16 and c >= 48, the second 16 <= c < 48), register c of lane L at slot
// (32 h + s(c)) 64 + L with s(63 - c) = 31 - s(c), so both partners read slot 31 - s at
// lane 63 - L: the same register indices in every wavefront, consecutive slots per
// phase (reads descending), no bank conflicts.  All H wavefronts take part.
TS_DEV void cross_wave_mirror(uint64_t* X, uint64_t (&v)[R], int h, int hp, int lane_in) {
    static_assert(XCH == 32, "two rounds of 32 registers");
    const bool keep_min = h < hp;  // wave-uniform
    const int lane = (int)opaque((uint32_t)lane_in);
    const int rl = 63 - lane;
#pragma unroll
    for (int round = 0; round < 2; ++round) {
        __syncthreads();  // earlier readers of X are done
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            const int c = round == 0 ? (j < 16 ? j : j + 32) : j + 16;
            X[(32 * h + j) * 64 + lane] = v[c];
        }
        __syncthreads();
#pragma unroll
        for (int j0 = 0; j0 < 32; j0 += 16) {  // 16 partner registers in flight at a time
            uint64_t y[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) y[j] = X[(32 * hp + 31 - (j0 + j)) * 64 + rl];
            if (keep_min) {
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int jj = j0 + j, c = round == 0 ? (jj < 16 ? jj : jj + 32) : jj + 16;
                    v[c] = comp_min(v[c], y[j]);
                }
            } else {
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int jj = j0 + j, c = round == 0 ? (jj < 16 ? jj : jj + 32) : jj + 16;
                    v[c] = comp_max(v[c], y[j]);
                }
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
// ascending; each further level (blocks of 2^k wavefronts) starts with the mirror
// stage against wavefront h ^ (2^k - 1), compares across wavefronts on the lower
// wavefront bits, and finishes inside each wavefront with the 12 merge stages of
// bitonic_merge4096, all ascending.  On exit register c of lane L in wavefront h holds
// rank 4096 h + 64 c + L.  A: wide_bitonic_words<H>() words, wavefront h uses its own
// MOVE_WORDS part for the transposes.
template <int H>
TS_DEV void bitonic_sort_wide(uint32_t* A, uint64_t (&v)[R], int h, int lane) {
    uint64_t* X = (uint64_t*)A;
    uint32_t* Aw = A + h * MOVE_WORDS;
    bitonic_sort4096(Aw, v, lane);
#pragma unroll
    for (int k = 1; (1 << k) <= H; ++k) {
        cross_wave_mirror(X, v, h, h ^ ((1 << k) - 1), lane);
#pragma unroll
        for (int b = k - 2; b >= 0; --b) cross_wave_stage(X, v, h, h ^ (1 << b), true, lane);
        __syncthreads();  // the exchange buffer overlaps the transpose arrays
        bitonic_merge4096(Aw, v, lane);
    }
}

}  // namespace bt
}  // namespace ts
