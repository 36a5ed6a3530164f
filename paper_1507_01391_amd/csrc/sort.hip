// Sorting tiles of up to 4096 uint32 keys in one wavefront without LDS bank conflicts.
//
// Problem: Afshani & Sitchinava, Sec. 1 ("Problems of interest", sorting).  The
// tile is the paper's w x m matrix with w = m = 64: lane L holds "row" L in 64
// registers.  Items are 64-bit composites (ordered key << 32 | tile position), all
// distinct, so any correct sort is the unique stable order.
//
// Two schedules share the same building blocks:
//  * a row sort: every lane sorts its 64 registers with a bitonic network
//    (register-only, no memory traffic: the paper's row sort, Sec. 2);
//  * direction masks: a row (or super-row) sorted descending is sorted ascending
//    on complemented composites, which reverses their order;
//  * layout moves through LDS: each lane writes register c to the slot of its
//    destination (lane L', register c') and then reads its new registers.  The
//    slot of (L', c') is c' * 64 + ((L' + h(c')) mod 64) with a per-move skew h
//    chosen so that every read instruction (32-lane phases of 8-byte slots) and
//    every write instruction (16-lane phases) touches distinct banks.
//
// THM2 follows Sec. 2, Theorem 2 for w = m = 64 with super-rows of 8 rows:
// Lemma 1 on every super-row (two rounds of {rows in alternating order,
// row-major -> column-major, rows ascending, column-major -> row-major}, then a
// final row sort), a column sort (transpose, row sort, transpose), Lemma 1 again
// with super-rows in alternating directions, a column sort and a final row sort:
// 13 row sorts.
//
// BITONIC is Batcher's bitonic network on the 4096 items, with the stages on
// register bits done in registers and the stages on lane bits done in registers
// after a conflict-free transpose (the same transpose the column sort uses).
#include "common.hpp"
#include "kernels.hpp"

namespace ts {

namespace {

constexpr int R = 64;  // registers (columns) per lane

TS_DEV void cas(uint64_t& a, uint64_t& b) {  // afterwards a <= b
    const bool s = b < a;
    const uint64_t lo = s ? b : a;
    const uint64_t hi = s ? a : b;
    a = lo;
    b = hi;
}

// Ascending bitonic sort of the 64 registers of every lane (672 compare-exchanges).
TS_DEV void row_sort(uint64_t (&v)[R]) {
#pragma unroll
    for (int k = 2; k <= R; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    if ((i & k) == 0) cas(v[i], v[l]);
                    else cas(v[l], v[i]);
                }
            }
        }
    }
}

// Ascending bitonic merge of the 64 registers of every lane (stages 32 .. 1).
TS_DEV void row_merge(uint64_t (&v)[R]) {
#pragma unroll
    for (int j = R >> 1; j > 0; j >>= 1) {
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int l = i ^ j;
            if (l > i) cas(v[i], v[l]);
        }
    }
}

// Stages j = 2^(KB-1) .. 1 of bitonic level 2^KB on the register index, direction
// given by bit KB of the register index (ascending when clear).
template <int KB>
TS_DEV void reg_level_stages(uint64_t (&v)[R]) {
#pragma unroll
    for (int j = 1 << (KB - 1); j > 0; j >>= 1) {
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int l = i ^ j;
            if (l > i) {
                if (((i >> KB) & 1) == 0) cas(v[i], v[l]);
                else cas(v[l], v[i]);
            }
        }
    }
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

// Apply a layout move through the LDS array A (4096 slots of 8 bytes).  One wave.
TS_DEV void layout_move(uint64_t* A, uint64_t (&v)[R], int move, int lane_in) {
    const int lane = (int)opaque((uint32_t)lane_in);  // keep addresses out of outer loops
#pragma unroll
    for (int c = 0; c < R; ++c) {
        int Ld, cd;
        move_dst(move, lane, c, Ld, cd);
        const uint32_t slot = (uint32_t)(cd * 64 + ((Ld + move_skew(move, cd)) & 63));
        lds_store(A, slot * 8u, v[c]);
    }
    // (LDS operations of one wave complete in order: the reads see the writes)
#pragma unroll
    for (int c = 0; c < R; ++c) {
        const uint32_t slot = (uint32_t)(c * 64 + ((lane + move_skew(move, c)) & 63));
        v[c] = lds_load(A, slot * 8u);
    }
}

// One phase of a schedule: xor with `pre`, row sort, xor with `post`, then a layout
// move.
struct Phase {
    uint8_t pre, post;   // mask kinds, see mask_of
    uint8_t move;        // Move
};

// Mask kinds: 0 none; 1 odd lanes (alternating rows); 2 odd super-rows (lanes 8..15,
// 24..31, ...); 3 both; 8 + kb: lanes with bit kb set (bitonic direction).
TS_DEV uint64_t mask_of(int kind, int lane) {
    bool on = false;
    if (kind == 0) on = false;
    else if (kind == 1) on = lane & 1;
    else if (kind == 2) on = (lane >> 3) & 1;
    else if (kind == 3) on = ((lane & 1) ^ ((lane >> 3) & 1)) != 0;
    else on = (lane >> (kind - 8)) & 1;
    return on ? ~0ull : 0ull;
}

// Theorem 2 (w = m = 64, super-rows of 8 rows): 13 row sorts.
__constant__ Phase kThm2[13] = {
    // Lemma 1 on every super-row, ascending
    {1, 1, MOVE_RM2CM}, {0, 0, MOVE_CM2RM},   // round 1
    {1, 1, MOVE_RM2CM}, {0, 0, MOVE_CM2RM},   // round 2
    {0, 0, MOVE_T},                              // final row sort; column sort starts
    {0, 0, MOVE_T},                              // column sort: sort, transpose back
    // Lemma 1 again, odd super-rows descending: their values stay complemented from
    // the first pre-mask (3 = super-row ^ alternation) to the last post-mask (2)
    {3, 1, MOVE_RM2CM}, {0, 0, MOVE_CM2RM},   // round 1
    {1, 1, MOVE_RM2CM}, {0, 0, MOVE_CM2RM},   // round 2
    {0, 2, MOVE_T},                              // final row sort; column sort starts
    {0, 0, MOVE_T},                              // column sort: sort, transpose back
    {0, 0, MOVE_T},                              // final row sort; to store order
};

template <int SCHED>  // 2 = THM2, 3 = BITONIC
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3)))
void sort4096_kernel(SortArgs a, const int64_t* __restrict__ offs) {
    __shared__ uint64_t A[4096];
    const int lane = lane_id();
    for (int64_t t = blockIdx.x; t < a.num_tiles; t += gridDim.x) {
        const int64_t o = offs[t];
        const int64_t len = offs[t + 1] - o;
        if (len > 4096) {
            if (lane == 0) atomicOr(a.err, ERR_TILE_TOO_LONG);
            continue;
        }
        const int n = (int)len;
        // ---- load: register c, lane L = item 64c + L (coalesced); padding sorts last
        uint64_t v[R];
        {
            uint32_t kk[R];
            load_columns<R>(a.keys_in, 1, o, n, 0, lane, kk, offs);
#pragma unroll
            for (int c = 0; c < R; ++c) {
                const uint32_t i = (uint32_t)(64 * c + lane);
                const uint32_t key = (i < (uint32_t)n) ? (a.f32 ? f32_to_ordered(kk[c]) : kk[c]) : 0xFFFFFFFFu;
                v[c] = pack(key, i);
            }
        }

        if (SCHED == 2) {
#pragma unroll 1
            for (int p = 0; p < 13; ++p) {
                const Phase ph = kThm2[p];
                xor_all(v, mask_of(ph.pre, lane));
                row_sort(v);
                xor_all(v, mask_of(ph.post, lane));
                layout_move(A, v, ph.move, lane);
            }
        } else {
            // levels 2 .. 64: rows sorted, odd rows descending
            xor_all(v, mask_of(1, lane));
            row_sort(v);
            xor_all(v, mask_of(1, lane));
#pragma unroll 1
            for (int kb = 1; kb <= 6; ++kb) {
                layout_move(A, v, MOVE_T, lane);  // lane bits become register bits
                switch (kb) {
                    case 1: reg_level_stages<1>(v); break;
                    case 2: reg_level_stages<2>(v); break;
                    case 3: reg_level_stages<3>(v); break;
                    case 4: reg_level_stages<4>(v); break;
                    case 5: reg_level_stages<5>(v); break;
                    default: reg_level_stages<6>(v); break;
                }
                layout_move(A, v, MOVE_T, lane);  // back: register bits
                const uint64_t m = (kb < 6) ? mask_of(8 + kb, lane) : 0ull;
                xor_all(v, m);
                row_merge(v);
                xor_all(v, m);
            }
            layout_move(A, v, MOVE_T, lane);  // to store order
        }

        // ---- store: register c, lane L holds rank 64 c + L
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const int r = 64 * c + lane;
            if (r < n) {
                const uint32_t key = hi32(v[c]);
                if (a.keys_out) store_item(a.keys_out, 1, o, r, a.f32 ? ordered_to_f32(key) : key);
                if (a.perm_out) store_item(a.perm_out, 1, o, r, (int32_t)lo32(v[c]));
            }
        }
    }
}

template <int SCHED>
hipError_t launch_s4096(const SortArgs& a, hipStream_t s) {
    auto kern = sort4096_kernel<SCHED>;
    const int grid = persistent_grid((const void*)kern, 64, 0, a.num_tiles);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64), 0, s, a, a.offsets);
    return hipGetLastError();
}

}  // namespace

int64_t sort_capacity(int sched) { return (sched == 2 || sched == 3) ? 4096 : 16384; }

hipError_t launch_sort(const SortArgs& a, int64_t max_len, int sched, hipStream_t s) {
    if (a.num_tiles == 0) return hipSuccess;
    if (sched == 2) return launch_s4096<2>(a, s);
    if (sched == 3) return launch_s4096<3>(a, s);
    return launch_sort_split(a, max_len, s);
}

}  // namespace ts
