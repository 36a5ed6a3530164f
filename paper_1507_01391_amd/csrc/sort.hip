// Sorting tiles of up to 4096 uint32 keys in one wavefront, and of up to 16384 keys in
// one workgroup of 2 or 4 wavefronts, without LDS bank conflicts.
//
// Problem: Afshani & Sitchinava, Sec. 1 ("Problems of interest", sorting).  The
// tile is the paper's w x m matrix with w = 64 rows (banks): for m = 64 lane L holds
// "row" L in 64 registers; for m = 128 and 256 the row is spread over H = m / 64
// wavefronts, wavefront h holding columns 64h .. 64h + 63 of every row.  Items are
// 64-bit composites (ordered key << 30 | tile position, below 2^62 as the networks of
// bitonic.hpp require), all distinct, so any correct sort is the unique stable order.
//
// The schedules share these building blocks:
//  * a row sort: every lane sorts its 64 registers with a bitonic network
//    (register-only, no memory traffic: the paper's row sort, Sec. 2); a row spread
//    over H wavefronts is finished by compare-exchanges between wavefronts (each
//    writes its registers to LDS and reads its partner's) and in-register merges;
//  * direction masks (Theorem 2): a row (or super-row) sorted descending is sorted
//    ascending on complemented composites, which reverses their order;
//  * layout moves through LDS: each lane writes register c to the slot of its
//    destination (lane L', register c') and then reads its new registers, one 32-bit
//    plane of the composites at a time, with slots skewed so that every 32-lane
//    phase of every read and write instruction touches distinct banks.
//
// THM2 follows Sec. 2, Theorem 2 with super-rows of 8 rows: Lemma 1 on every
// super-row (two rounds of {rows sorted in alternating directions, move from
// row-major to column-major order, rows sorted ascending, move back}, then an
// ascending row sort), a column sort (transpose, sort, transpose), Lemma 1 again with
// super-rows in alternating directions, a column sort and a final row sort: 13 row
// sorts.  For m = 128 and 256 this is the schedule with super-rows of sqrt(w) = 8
// rows, which satisfy Lemma 1's condition (8 <= sqrt(m)) for every m >= 64; a column
// (64 items, one per row) lies inside one wavefront's columns, so the column sorts
// need no exchange between wavefronts.
//
// BITONIC is Batcher's bitonic network on the 4096 items in its mirror form (no
// descending blocks, no masks), with the stages on register bits done in registers and
// the stages on lane bits done in registers after a conflict-free transpose (the one the
// column sort uses, with the lanes of half the rows reversed); tiles of 8192 and 16384
// keys spread the network over 2 and 4 wavefronts, whose stages on the wavefront bits
// compare through LDS.
#include "bitonic.hpp"
#include "common.hpp"
#include "kernels.hpp"

namespace ts {

namespace {

using namespace bt;

// Composite of an ordered key and its tile position (< 2^30).
constexpr int SORT_POS_BITS = 30;
TS_DEV uint64_t comp(uint32_t key, uint32_t pos) { return ((uint64_t)key << SORT_POS_BITS) | pos; }
TS_DEV uint32_t comp_key(uint64_t c) { return (uint32_t)(c >> SORT_POS_BITS); }
TS_DEV uint32_t comp_pos(uint64_t c) { return (uint32_t)c & ((1u << SORT_POS_BITS) - 1u); }

// One phase of a schedule: xor with `pre`, row sort, xor with `post`, then a layout
// move.  `runs` (see row_sort_from): 1 when every row enters the phase as runs sorted
// in alternating directions (rows sorted in alternating directions, then moved from
// row-major to column-major order inside their super-row), 2 when every column does
// (the column sort after the second such Lemma 1); 0 otherwise.
struct Phase {
    uint8_t pre, post;   // mask kinds, see mask_of
    uint8_t move;        // Move
    uint8_t runs;
};

// The register row sort from bitonic level `start` on (2 = the whole network).  Where a
// phase's rows arrive as runs of r items sorted in alternating directions, every block
// of 2r registers is already bitonic and levels 2 .. r are skipped: r = 8 for the
// 64 x 64 tile and for the column sorts, r = 8H for a row of a 64 x 64H tile (each
// wavefront's part holds runs of 8H items of 8 source rows).  `start` is wave-uniform,
// so each level is one scalar branch and the network's code appears once.
template <int K>
TS_DEV void sort_level(uint64_t (&v)[R]) { net_stages<(K < R ? K : 0), K / 2>(v); }
TS_DEV void row_sort_from(uint64_t (&v)[R], int start) {
    if (start <= 2) sort_level<2>(v);
    __builtin_amdgcn_sched_barrier(0);
    if (start <= 4) sort_level<4>(v);
    __builtin_amdgcn_sched_barrier(0);
    if (start <= 8) sort_level<8>(v);
    __builtin_amdgcn_sched_barrier(0);
    if (start <= 16) sort_level<16>(v);
    __builtin_amdgcn_sched_barrier(0);
    if (start <= 32) sort_level<32>(v);
    __builtin_amdgcn_sched_barrier(0);
    sort_level<64>(v);
}
TS_DEV int runs_start(int runs, int H) {
    const int r = runs == 1 ? 8 * H : 8;
    return runs == 0 ? 2 : (2 * r < 64 ? 2 * r : 64);
}

// Mask kinds: 0 none; 1 odd lanes (alternating rows); 2 odd super-rows (lanes 8..15,
// 24..31, ...); 3 both; 8 + kb: lanes with bit kb set (bitonic direction).
TS_DEV uint64_t mask_of(int kind, int lane) {
    bool on = false;
    if (kind == 0) on = false;
    else if (kind == 1) on = lane & 1;
    else if (kind == 2) on = (lane >> 3) & 1;
    else if (kind == 3) on = ((lane & 1) ^ ((lane >> 3) & 1)) != 0;
    else on = (lane >> (kind - 8)) & 1;
    return on ? COMP_MASK : 0ull;
}

// Theorem 2 (w = m = 64, super-rows of 8 rows): 13 row sorts.
__constant__ Phase kThm2[13] = {
    // Lemma 1 on every super-row, ascending: alternate-direction row sort + RM->CM,
    // ascending row sort + CM->RM, twice
    {1, 1, MOVE_RM2CM, 0}, {0, 0, MOVE_CM2RM, 1},
    {1, 1, MOVE_RM2CM, 0}, {0, 0, MOVE_CM2RM, 1},
    {0, 0, MOVE_T, 0},                           // ascending row sort; column sort starts
    {0, 0, MOVE_T, 0},                           // column sort: sort, transpose back
    // Lemma 1 again, odd super-rows descending: their values stay complemented from
    // the first pre-mask (3 = super-row ^ alternation) to the last post-mask (2)
    {3, 1, MOVE_RM2CM, 0}, {0, 0, MOVE_CM2RM, 1},
    {1, 1, MOVE_RM2CM, 0}, {0, 0, MOVE_CM2RM, 1},
    {0, 2, MOVE_T, 0},                           // ascending row sort; column sort starts
    {0, 0, MOVE_T, 2},                           // column sort: sort, transpose back
    {0, 0, MOVE_T, 0},                           // final row sort; to store order
};

// Stores of keys and positions: register c of lane L holds rank rb + 64 c + L, valid
// below n.  Buffer resources over the ranks rb ..: a column is the lane offset plus an
// immediate, and stores of ranks >= n are dropped by the hardware range check, so
// there is no per-register branch or 64-bit address.
TS_DEV void store_sorted(const SortArgs& a, int64_t o, int rb, int n, const uint64_t (&v)[R], int lane_in) {
    const int ln = (int)opaque((uint32_t)lane_in);
    const uint32_t nv = n > rb ? (uint32_t)(n - rb) : 0u;
    const uint32_t off = (uint32_t)ln * 4u;
    if (a.keys_out) {
        const rsrc_t r = buffer_rsrc(a.keys_out + o + rb, nv * 4u);
        if (a.f32) {
#pragma unroll
            for (int c = 0; c < R; ++c) buffer_store(r, off + 256u * c, ordered_to_f32(comp_key(v[c])));
        } else {
#pragma unroll
            for (int c = 0; c < R; ++c) buffer_store(r, off + 256u * c, comp_key(v[c]));
        }
    }
    if (a.perm_out) {
        const rsrc_t r = buffer_rsrc(a.perm_out + o + rb, nv * 4u);
#pragma unroll
        for (int c = 0; c < R; ++c) buffer_store(r, off + 256u * c, comp_pos(v[c]));
    }
}

// Payload of the ranks a lane holds, gathered from the input at each rank's source
// position (a global gather inside the tile, no LDS): register c of lane L holds rank
// rank_of(c), whose source position is pos[c].  Used where no permutation is kept for a
// second, routed launch (partition through a sort schedule).  Addresses are rebuilt per
// channel from an opaque lane index, so none stay live across the channel loop.
template <int NREG, typename RankFn>
TS_DEV void gather_payload(const SortArgs& a, int64_t o, int n, const uint32_t (&pos)[NREG], int lane,
                           RankFn rank_of) {
    const PayloadRef& p = a.pay;
#pragma unroll 1
    for (uint32_t ch = 0; ch < p.channels; ++ch) {
        const int ln = (int)opaque((uint32_t)lane);
        const uint32_t* src = p.in + (int64_t)ch * p.cs + o * p.es;
        uint32_t* dst = p.out + (int64_t)ch * p.cs + o * p.es;
#pragma unroll
        for (int g = 0; g < NREG; g += 16) {
            uint32_t w[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int r = rank_of(g + j, ln);
                w[j] = (r < n) ? src[(int64_t)pos[g + j] * p.es] : 0u;
            }
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int r = rank_of(g + j, ln);
                if (r < n) dst[(int64_t)r * p.es] = w[j];
            }
            __builtin_amdgcn_sched_barrier(0);  // one group of addresses live at a time
        }
    }
}

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
        const rsrc_t rk = buffer_rsrc(a.keys_in + o, (uint32_t)(n > 0 ? n : 0) * 4u);  // 0 past the end
#pragma unroll 1
        for (int g = 0; g < R; g += 16) {
            uint32_t kk[16];
            buffer_load_columns<16>(rk, (uint32_t)lane * 4u + 256u * (uint32_t)g, kk);
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
            v[c] = comp(lds_load(A, i * 4u), i);
        }

        if (SCHED == 2) {
#pragma unroll 1
            for (int p = 0; p < 13; ++p) {
                const Phase ph = kThm2[p];
                xor_all(v, mask_of(ph.pre, lane));
                row_sort_from(v, runs_start(ph.runs, 1));
                xor_all(v, mask_of(ph.post, lane));
                layout_move(A, v, ph.move, lane);
            }
        } else {
            bitonic_sort4096(A, v, lane);
        }

        // ---- store: register c, lane L holds rank 64 c + L
        store_sorted(a, o, 0, n, v, lane);
        if (a.fuse_pay) {
            uint32_t pos[R];
#pragma unroll
            for (int c = 0; c < R; ++c) pos[c] = comp_pos(v[c]);
            gather_payload<R>(a, o, n, pos, lane, [](int c, int ln) { return 64 * c + ln; });
        }
    }
}

// ---------------------------------------------------------------------------------
// Theorem 2 on a 64 x m tile, m = 64 H (H = 2, 4 wavefronts): wavefront h holds columns
// 64h .. 64h + 63 of every row (lane L = row L, register c = column 64h + c).

// Phase kinds of the wide schedule: the sort a phase runs, and the move after it.
enum WideSort : uint8_t { SORT_ROW = 0, SORT_COL = 1 };
enum WideMove : uint8_t { WM_RM2CM = 0, WM_CM2RM = 1, WM_T = 2, WM_FINAL = 3 };
struct WidePhase {
    uint8_t pre, post, sort, move, runs;
};

// The 13 row sorts of the Theorem 2 schedule, as in kThm2; the two column sorts sort
// 64-item columns after an in-wavefront transpose, and the last move puts the tile in
// store order.
__constant__ WidePhase kThm2Wide[13] = {
    {1, 1, SORT_ROW, WM_RM2CM, 0}, {0, 0, SORT_ROW, WM_CM2RM, 1},
    {1, 1, SORT_ROW, WM_RM2CM, 0}, {0, 0, SORT_ROW, WM_CM2RM, 1},
    {0, 0, SORT_ROW, WM_T, 0},     {0, 0, SORT_COL, WM_T, 0},
    {3, 1, SORT_ROW, WM_RM2CM, 0}, {0, 0, SORT_ROW, WM_CM2RM, 1},
    {1, 1, SORT_ROW, WM_RM2CM, 0}, {0, 0, SORT_ROW, WM_CM2RM, 1},
    {0, 2, SORT_ROW, WM_T, 0},     {0, 0, SORT_COL, WM_T, 2},
    {0, 0, SORT_ROW, WM_FINAL, 0},
};

// LDS words of the wide kernel: the largest of the cross-wavefront moves (one 32-bit
// plane of 64 x m items; the final move pitches rows at m + 1 words), the per-wavefront
// transpose arrays, and the exchange buffers (XCH registers of 64 bits per lane and
// wavefront).
template <int H>
constexpr int wide_words() {
    constexpr int a = 64 * (64 * H + 1), b = H * MOVE_WORDS, c = H * XCH * 64 * 2;
    return a > b ? (a > c ? a : c) : (b > c ? b : c);
}

// Ascending sort of every row of m = 64 H items spread over the H wavefronts: a bitonic
// sort whose stages on register bits run in registers and whose stages on wavefront
// bits compare across wavefronts.  The caller has sorted each wavefront's 64 registers,
// ascending in even and descending in odd wavefronts (level 64); this finishes levels
// 128 and 256.
template <int H>
TS_DEV void wide_row_merge(uint64_t* X, uint64_t (&v)[R], int h, int lane) {
    // level 128: pairs of wavefronts; with H = 4 the second pair merges descending
    const bool asc128 = (H == 2) || ((h >> 1) & 1) == 0;
    cross_wave_stage(X, v, h, h ^ 1, asc128, lane);
    const uint64_t m2 = asc128 ? 0ull : COMP_MASK;
    xor_all(v, m2);
    row_merge(v);
    xor_all(v, m2);
    if constexpr (H == 4) {  // level 256
        cross_wave_stage(X, v, h, h ^ 2, true, lane);
        cross_wave_stage(X, v, h, h ^ 1, true, lane);
        row_merge(v);
    }
}

// Super-row moves of a 64 x m tile (super-rows of 8 rows): source (row L, column c)
// -> destination (row Ld, column cd), and the slot skew of destination column cd.
// RM->CM: row-major position p = 8-row index i * m + c goes to (p mod 8, p / 8);
// CM->RM: column-major position p = 8 c + i goes to (p / m, p mod m).
template <int M>
TS_DEV void wide_move_dst(int move, int L, int c, int& Ld, int& cd) {
    const int i = L & 7;
    if (move == WM_RM2CM) {
        const int p = i * M + c;
        Ld = (L & ~7) + (p & 7);
        cd = p >> 3;
    } else {
        const int p = 8 * c + i;
        Ld = (L & ~7) + p / M;
        cd = p % M;
    }
}
template <int M>
TS_DEV int wide_skew(int move, int cd) { return move == WM_RM2CM ? cd / (M / 8) : (cd & 7); }

// A layout move through LDS, one 32-bit plane at a time; the transpose (T) stays inside
// each wavefront's own array (the 64 x 64 pitch-65 transpose of bitonic.hpp), the other
// moves cross wavefronts.  Super-row moves
// store (Ld, cd) at word 64 cd + ((Ld + skew(cd)) mod 64): in every write instruction
// the 32 lanes of a phase reach 8 rows Ld = 8g + const and 8 columns cd whose skews are
// the 8 values i, so the words are distinct modulo 32; reads are 64 consecutive words
// rotated.  The final move stores rank q = L m + 64 h + c at word q + q / m: writes are
// m + 1 words apart per lane (distinct modulo 32), reads 64 consecutive words.
template <int H>
TS_DEV void wide_move(uint32_t* A, uint64_t (&v)[R], int move, int h, int lane_in) {
    constexpr int M = 64 * H;
#pragma unroll
    for (int half = 1; half >= 0; --half) {
        __syncthreads();  // earlier readers of A are done
        const int lane = (int)opaque((uint32_t)lane_in);
        if (move == WM_FINAL || move == WM_T) {
            // FINAL: rows pitched at m + 1 words; T: this wavefront's own 64 x 65 array
            const uint32_t base = (move == WM_FINAL) ? (uint32_t)(lane * (M + 1) + 64 * h)
                                                     : (uint32_t)(h * MOVE_WORDS + 65 * lane);
#pragma unroll
            for (int c = 0; c < R; ++c) lds_store(A, (base + (uint32_t)c) * 4u, half ? hi32(v[c]) : lo32(v[c]));
        } else {
#pragma unroll
            for (int c = 0; c < R; ++c) {
                int Ld, cd;
                wide_move_dst<M>(move, lane, 64 * h + c, Ld, cd);
                const uint32_t slot = (uint32_t)(cd * 64 + ((Ld + wide_skew<M>(move, cd)) & 63));
                lds_store(A, slot * 4u, half ? hi32(v[c]) : lo32(v[c]));
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const int k = 64 * h + c;  // destination column (FINAL: rank column)
            const uint32_t slot = (move == WM_FINAL) ? (uint32_t)(64 * k + lane + (64 * k) / M)
                                  : (move == WM_T)   ? (uint32_t)(h * MOVE_WORDS + 65 * c + lane)
                                                     : (uint32_t)(k * 64 + ((lane + wide_skew<M>(move, k)) & 63));
            const uint32_t w = lds_load(A, slot * 4u);
            v[c] = half ? pack(w, lo32(v[c])) : pack(hi32(v[c]), w);
        }
    }
}

template <int H>
__global__ __launch_bounds__(64 * H) __attribute__((amdgpu_waves_per_eu(2)))
void thm2_wide_kernel(SortArgs a, const int64_t* __restrict__ offs) {
    constexpr int M = 64 * H;
    constexpr int CAP = 64 * M;
    __shared__ __attribute__((aligned(16))) uint32_t A[wide_words<H>()];
    uint64_t* X = (uint64_t*)A;
    const int h = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (int64_t t = blockIdx.x; t < a.num_tiles; t += gridDim.x) {
        const int lane = (int)opaque((uint32_t)lane_id());
        const int64_t o = offs[t];
        const int64_t len = offs[t + 1] - o;
        if (len > CAP) {
            if (threadIdx.x == 0) atomicOr(a.err, ERR_TILE_TOO_LONG);
            continue;
        }
        const int n = (int)len;
        // ---- load: register c of lane L in wavefront h holds item 64 (64 h + c) + L (the
        // schedule sorts any placement: coalesced columns); padding sorts last.  Sixteen
        // columns at a time are staged through this wavefront's part of A (each lane
        // reads back its own words), which bounds the loads in flight.
        uint32_t* Aw = A + h * MOVE_WORDS;
        __syncthreads();  // every wavefront has read the previous tile's last move
        const rsrc_t rk = buffer_rsrc(a.keys_in + o, (uint32_t)(n > 0 ? n : 0) * 4u);  // 0 past the end
#pragma unroll 1
        for (int g = 0; g < R; g += 16) {
            uint32_t kk[16];
            buffer_load_columns<16>(rk, (uint32_t)lane * 4u + 256u * (uint32_t)(64 * h + g), kk);
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const uint32_t i = (uint32_t)(64 * (64 * h + g + j) + lane);
                lds_store(Aw, (uint32_t)(64 * (g + j) + lane) * 4u,
                          (i < (uint32_t)n) ? (a.f32 ? f32_to_ordered(kk[j]) : kk[j]) : 0xFFFFFFFFu);
            }
        }
        uint64_t v[R];
#pragma unroll
        for (int c = 0; c < R; ++c)
            v[c] = comp(lds_load(Aw, (uint32_t)(64 * c + lane) * 4u), (uint32_t)(64 * (64 * h + c) + lane));

#pragma unroll 1
        for (int p = 0; p < 13; ++p) {
            const WidePhase ph = kThm2Wide[p];
            // one register sort per phase: a column, or this wavefront's part of a row
            // (descending in odd wavefronts, for the merge across wavefronts)
            const bool row = ph.sort == SORT_ROW;
            const uint64_t m1 = (row && (h & 1)) ? COMP_MASK : 0ull;
            xor_all(v, mask_of(ph.pre, lane) ^ m1);
            row_sort_from(v, runs_start(ph.runs, H));
            xor_all(v, m1);
            if (row) wide_row_merge<H>(X, v, h, lane);
            xor_all(v, mask_of(ph.post, lane));
            wide_move<H>(A, v, ph.move, h, lane);
        }

        // ---- store: register c of lane L in wavefront h holds rank 64 (64 h + c) + L
        const int cb = 64 * h;
        store_sorted(a, o, 4096 * h, n, v, lane);
        if (a.fuse_pay) {
            uint32_t pos[R];
#pragma unroll
            for (int c = 0; c < R; ++c) pos[c] = comp_pos(v[c]);
            gather_payload<R>(a, o, n, pos, lane, [cb](int c, int ln) { return 64 * (cb + c) + ln; });
        }
    }
}

template <int H>
hipError_t launch_thm2_wide(const SortArgs& a, hipStream_t s) {
    auto kern = thm2_wide_kernel<H>;
    const int grid = persistent_grid((const void*)kern, 64 * H, 0, a.num_tiles);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * H), 0, s, a, a.offsets);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Batcher's bitonic sort of tiles of 4096 H keys, H = 2 or 4 wavefronts per tile
// (bitonic_sort_wide): wavefront h loads items 4096 h .. 4096 h + 4095 and stores ranks
// 4096 h .. 4096 h + 4095.
template <int H>
__global__ __launch_bounds__(64 * H) __attribute__((amdgpu_waves_per_eu(2)))
void bitonic_wide_kernel(SortArgs a, const int64_t* __restrict__ offs) {
    constexpr int CAP = 4096 * H;
    __shared__ __attribute__((aligned(16))) uint32_t A[wide_bitonic_words<H>()];
    const int h = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (int64_t t = blockIdx.x; t < a.num_tiles; t += gridDim.x) {
        const int lane = (int)opaque((uint32_t)lane_id());
        const int64_t o = offs[t];
        const int64_t len = offs[t + 1] - o;
        if (len > CAP) {
            if (threadIdx.x == 0) atomicOr(a.err, ERR_TILE_TOO_LONG);
            continue;
        }
        const int n = (int)len;
        const int nw = n > 4096 * h ? n - 4096 * h : 0;  // items of this wavefront's part
        // ---- load through this wavefront's own part of A (16 columns in flight)
        uint32_t* Aw = A + h * MOVE_WORDS;
        __syncthreads();  // every wavefront is done with the previous tile's exchanges
        const rsrc_t rk = buffer_rsrc(a.keys_in + o + 4096 * h, (uint32_t)nw * 4u);  // 0 past the end
#pragma unroll 1
        for (int g = 0; g < R; g += 16) {
            uint32_t kk[16];
            buffer_load_columns<16>(rk, (uint32_t)lane * 4u + 256u * (uint32_t)g, kk);
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int i = 64 * (g + j) + lane;
                lds_store(Aw, (uint32_t)i * 4u, (i < nw) ? (a.f32 ? f32_to_ordered(kk[j]) : kk[j]) : 0xFFFFFFFFu);
            }
        }
        uint64_t v[R];
#pragma unroll
        for (int c = 0; c < R; ++c)
            v[c] = comp(lds_load(Aw, (uint32_t)(64 * c + lane) * 4u), (uint32_t)(4096 * h + 64 * c + lane));

        bitonic_sort_wide<H>(A, v, h, lane);

        // ---- store: register c of lane L in wavefront h holds rank 4096 h + 64 c + L
        const int rb = 4096 * h;
        store_sorted(a, o, rb, n, v, lane);
        if (a.fuse_pay) {
            uint32_t pos[R];
#pragma unroll
            for (int c = 0; c < R; ++c) pos[c] = comp_pos(v[c]);
            gather_payload<R>(a, o, n, pos, lane, [rb](int c, int ln) { return rb + 64 * c + ln; });
        }
    }
}

template <int H>
hipError_t launch_bitonic_wide(const SortArgs& a, hipStream_t s) {
    auto kern = bitonic_wide_kernel<H>;
    const int grid = persistent_grid((const void*)kern, 64 * H, 0, a.num_tiles);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * H), 0, s, a, a.offsets);
    return hipGetLastError();
}

template <int SCHED>
hipError_t launch_s4096(const SortArgs& a, hipStream_t s) {
    auto kern = sort4096_kernel<SCHED>;
    const int grid = persistent_grid((const void*)kern, 64, 0, a.num_tiles);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64), 0, s, a, a.offsets);
    return hipGetLastError();
}

}  // namespace

int64_t sort_capacity(int sched) { (void)sched; return 16384; }

hipError_t launch_sort(const SortArgs& a, int64_t max_len, int sched, hipStream_t s) {
    if (a.num_tiles == 0) return hipSuccess;
    if (sched == 2) {
        if (max_len <= 4096) return launch_s4096<2>(a, s);
        if (max_len <= 8192) return launch_thm2_wide<2>(a, s);
        return launch_thm2_wide<4>(a, s);
    }
    if (sched == 3) {
        if (max_len <= 4096) return launch_s4096<3>(a, s);
        if (max_len <= 8192) return launch_bitonic_wide<2>(a, s);
        return launch_bitonic_wide<4>(a, s);
    }
    return launch_sort_split(a, max_len, s);
}

}  // namespace ts
