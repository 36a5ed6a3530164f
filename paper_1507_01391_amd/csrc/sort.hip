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
//    destination (lane L', register c') and then reads its new registers, one 32-bit
//    plane of the composites at a time, with slots skewed so that every 32-lane
//    phase of every read and write instruction touches distinct banks.
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
#include "bitonic.hpp"
#include "common.hpp"
#include "kernels.hpp"

namespace ts {

namespace {

using namespace bt;

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
    {1, 1, MOVE_RM2CM}, {0, 0, MOVE_CM2RM},   // steps 1-4, first time
    {1, 1, MOVE_RM2CM}, {0, 0, MOVE_CM2RM},   // steps 1-4, second time
    {0, 0, MOVE_T},                              // final row sort; column sort starts
    {0, 0, MOVE_T},                              // column sort: sort, transpose back
    // Lemma 1 again, odd super-rows descending: their values stay complemented from
    // the first pre-mask (3 = super-row ^ alternation) to the last post-mask (2)
    {3, 1, MOVE_RM2CM}, {0, 0, MOVE_CM2RM},   // steps 1-4, first time
    {1, 1, MOVE_RM2CM}, {0, 0, MOVE_CM2RM},   // steps 1-4, second time
    {0, 2, MOVE_T},                              // final row sort; column sort starts
    {0, 0, MOVE_T},                              // column sort: sort, transpose back
    {0, 0, MOVE_T},                              // final row sort; to store order
};

template <int SCHED>  // 2 = THM2, 3 = BITONIC
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
void sort4096_kernel(SortArgs a, const int64_t* __restrict__ offs) {
    __shared__ uint32_t A[MOVE_WORDS];
    for (int64_t t = blockIdx.x; t < a.num_tiles; t += gridDim.x) {
        // lane-derived values are recomputed per tile rather than kept live (and
        // spilled) across the whole loop
        const int lane = (int)opaque((uint32_t)lane_id());
        const int64_t o = offs[t];
        const int64_t len = offs[t + 1] - o;
        if (len > 4096) {
            if (lane == 0) atomicOr(a.err, ERR_TILE_TOO_LONG);
            continue;
        }
        const int n = (int)len;
        // ---- load: 16 coalesced columns at a time, staged through LDS (word 64 c + L);
        // register c of lane L then holds item 64 c + L; padding sorts last
#pragma unroll 1
        for (int g = 0; g < R; g += 16) {
            uint32_t kk[16];
            load_columns<16>(a.keys_in, 1, o, n, g, lane, kk, offs);
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const uint32_t i = (uint32_t)(64 * (g + j) + lane);
                lds_store(A, i * 4u, (i < (uint32_t)n) ? (a.f32 ? f32_to_ordered(kk[j]) : kk[j]) : 0xFFFFFFFFu);
            }
        }
        uint64_t v[R];
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const uint32_t i = (uint32_t)(64 * c + lane);
            v[c] = pack(lds_load(A, i * 4u), i);
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
            bitonic_sort4096(A, v, lane);
        }

        // ---- store: register c, lane L holds rank 64 c + L (addresses computed here,
        // not hoisted above the network)
        const int sl = (int)opaque((uint32_t)lane);
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const int r = 64 * c + sl;
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
