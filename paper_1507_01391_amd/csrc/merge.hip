// Sorting a batch of tiles of uneven length (1 .. 2^28 keys each) in a fixed sequence of
// launches that a stream capture can record once and replay.
//
// The tile-local problem is the paper's sorting problem (Sec. 1, "Problems of
// interest"); its schedules assume a w x m tile resident in one workgroup.  Tiles of up
// to 4096 keys are sorted in one wavefront (packed up to eight per wavefront), tiles of
// 4097 .. 32768 keys whole in one workgroup of 2, 4 or 8 wavefronts (the bitonic network
// spread over the wavefronts, bitonic_sort_wide: the tile stays resident, so every key
// is read and written once).  A longer tile is cut into 4096-key pieces, every piece
// is sorted in registers by the bitonic network of bitonic.hpp (conflict-free
// transposes through LDS), and sorted runs are merged pairwise, doubling the run length
// per round.  A
// merge step is the last level of the same bitonic network, applied to 4096 outputs at
// a time: a merge-path co-rank search picks the A and B ranges that produce them, A is
// loaded ascending and B descending (a bitonic sequence) and 12 merge stages sort it.
//
// Items are 64-bit composites  key << 28 | position,  distinct within a tile, so the
// result is the unique stable order.  A packing wavefront holds up to eight tiles of at
// most 512 keys (four of 1024, two of 2048): there the composite is
// slot << 44 | key << 12 | position, each tile owning a slot of 4096 / P positions,
// and its padding sorts to the end of its slot.  Both forms stay below 2^62, the range
// the networks of bitonic.hpp compare in.
//
// Sequence of launches (all on one stream, no host synchronisation):
//   1. clear the work counters (a fill kernel, so the sequence stays capturable);
//   2. bin: one thread per tile appends the tile to a packing bin or a workgroup bin,
//      or its pieces to the piece list and its output pieces to the list of every merge
//      round it needs;
//   3. sort: one persistent launch per bin and one for the pieces;
//   4. per merge round: co-rank search (one thread per output piece), then the merge.
// The last store of every tile writes keys, the permutation and the payload, gathered
// from the input by the permutation.
#include "bitonic.hpp"
#include "common.hpp"
#include "kernels.hpp"

namespace ts {

namespace {

using namespace bt;

constexpr int K = MERGE_PIECE;
constexpr int POS_BITS = MERGE_POS_BITS;
constexpr int PACKED_POS_BITS = 12;  // positions within a packing wavefront (< 4096)
constexpr uint64_t PAD = COMP_MASK;  // above every composite

int g_merge_pack = 1;
// Longest tile sorted whole by one workgroup (4096: none, every longer tile goes
// through pieces and merge rounds); tuning knob "merge_wide".
int g_merge_wide = 32768;

// Bins: 0 .. 3 pack 8 / 4 / 2 / 1 tiles of up to 512 / 1024 / 2048 / 4096 keys per
// wavefront; 4 .. 6 hold tiles of up to 8192 / 16384 / 32768 keys, one per workgroup of
// 2 / 4 / 8 wavefronts.  Counter word of bin b (the piece list counts at word 4).
constexpr int NUM_BINS = 7;
constexpr int BIN_THREADS = 1024;  // threads (tiles) per workgroup of merge_bin_kernel
TS_DEV int bin_counter(int b) { return b < 4 ? b : b + 1; }

// Composite with PB position bits: slot << (32 + PB) | key << PB | pos.
template <int PB>
TS_DEV uint64_t make_comp(uint32_t slot, uint32_t key, uint32_t pos) {
    return ((uint64_t)slot << (32 + PB)) | ((uint64_t)key << PB) | pos;
}
template <int PB>
TS_DEV uint32_t comp_key(uint64_t c) { return (uint32_t)(c >> PB); }
template <int PB>
TS_DEV uint32_t comp_pos(uint64_t c) { return (uint32_t)c & ((1u << PB) - 1u); }

TS_DEV uint64_t entry(int64_t tile, uint32_t j) { return ((uint64_t)tile << 16) | j; }
TS_DEV int64_t entry_tile(uint64_t e) { return (int64_t)(e >> 16); }
TS_DEV uint32_t entry_j(uint64_t e) { return (uint32_t)(e & 0xFFFFu); }

TS_DEV uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
TS_DEV int64_t uniform64(int64_t v) {
    const uint64_t u = (uint64_t)v;
    return (int64_t)(((uint64_t)uniform((uint32_t)(u >> 32)) << 32) | uniform((uint32_t)u));
}

// Append `cnt` entries (tile, 0 .. cnt-1) per lane to `list`, one atomic per wave.
// Entries past `cap` are dropped and reported (tiles overlapping in a malformed offset
// array could otherwise need more entries than the workspace holds).
TS_DEV void wave_append(uint32_t* counter, uint64_t* list, int64_t cap, uint32_t* err,
                        uint32_t cnt, int64_t tile, int lane) {
    uint32_t x = cnt;  // inclusive scan over the wave
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)x, d);
        if (lane >= d) x += y;
    }
    const uint32_t total = (uint32_t)__shfl((int)x, 63);
    if (total == 0) return;
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(counter, total);
    base = (uint32_t)__shfl((int)base, 0);
    const uint32_t start = base + x - cnt;
    const bool over = (int64_t)start + cnt > cap;
    flag_error(err, over, ERR_BAD_OFFSETS);
    for (uint32_t j = 0; j < cnt && (int64_t)(start + j) < cap; ++j) list[start + j] = entry(tile, j);
}


// One thread per tile.  The bin entries of a workgroup are counted in LDS first (one
// LDS atomic per wave and bin) and reserved with one global atomic per workgroup and
// bin: with a global atomic per wave the few bin counters serialised the launch.  The
// tile loop steps by whole workgroups, so every wave of a workgroup meets the same
// barriers.
__global__ __launch_bounds__(BIN_THREADS) void merge_bin_kernel(MergeArgs a) {
    __shared__ uint32_t wg_count[NUM_BINS], wg_base[NUM_BINS];
    const int lane = lane_id();
    const int64_t T = a.s.num_tiles;
    const int64_t stride = (int64_t)gridDim.x * BIN_THREADS;
    for (int64_t b0 = (int64_t)blockIdx.x * BIN_THREADS; b0 < T; b0 += stride) {
        const int64_t t = b0 + threadIdx.x;
        int64_t n = 0;
        bool bad = false;
        if (t < T) {
            const int64_t o = a.s.offsets[t];
            n = a.s.offsets[t + 1] - o;
            bad = o < 0 || n < 0 || o + n > a.total_len;  // would leave the run buffers
        }
        const bool too_long = !bad && n > a.max_len;
        flag_error(a.s.err, too_long, ERR_TILE_TOO_LONG);
        flag_error(a.s.err, bad, ERR_BAD_OFFSETS);
        if (too_long || bad) n = 0;
        int bin = -1;
        if (n > 0 && n <= K) bin = a.pack ? (n <= 512 ? 0 : n <= 1024 ? 1 : n <= 2048 ? 2 : 3) : 3;
        else if (n > K && n <= a.wide_max) bin = n <= 2 * K ? 4 : n <= 4 * K ? 5 : 6;
        if (threadIdx.x < NUM_BINS) wg_count[threadIdx.x] = 0u;
        __syncthreads();
        uint32_t slot = 0;  // this tile's place among the workgroup's entries of its bin
        for (int b = 0; b < NUM_BINS; ++b) {
            const uint64_t m = ballot(bin == b);
            if (m == 0) continue;
            const int leader = __builtin_ctzll(m);
            uint32_t wb = 0;
            if (lane == leader) wb = atomicAdd(&wg_count[b], (uint32_t)popc64(m));
            wb = (uint32_t)__shfl((int)wb, leader);
            if (bin == b) slot = wb + count_below(m);
        }
        __syncthreads();
        if (threadIdx.x < NUM_BINS && wg_count[threadIdx.x] > 0u)
            wg_base[threadIdx.x] = atomicAdd(&a.counters[bin_counter((int)threadIdx.x)], wg_count[threadIdx.x]);
        __syncthreads();
        if (bin >= 0) a.bins[bin * T + wg_base[bin] + slot] = entry(t, 0);
        const uint32_t np = (n > a.wide_max) ? (uint32_t)((n + K - 1) / K) : 0u;
        wave_append(&a.counters[4], a.pieces, a.cap, a.s.err, np, t, lane);
        for (int r = 0; r < a.rounds; ++r) {
            const uint32_t nr = (n > ((int64_t)K << r)) ? np : 0u;
            wave_append(&a.counters[8 + r], a.round_lists + (int64_t)r * a.cap, a.cap, a.s.err, nr, t,
                        lane);
        }
        __syncthreads();  // wg_count and wg_base are reused by the next group of tiles
    }
}

// ---------------------------------------------------------------------------------
// Final stores of registers c0 .. c0+NC-1 of one tile: register c0 + c of lane L holds
// rank rb + 64 c + L, valid below `nvalid`.  Keys and positions are written straight
// from the composites; the payload is gathered through the positions 16 registers at a
// time, every load of a group issued before any is used (a load per register inside
// its own branch would wait for each one in turn).
// `narrow`: every payload offset of the tile (position x elem_stride x 4 bytes) fits
// in 32 bits, so gathers use a wave-uniform base plus 32-bit offsets.  PB: position
// bits of the composites.
template <int NC, int PB = POS_BITS>
TS_DEV void store_final_regs(const SortArgs& s, int64_t o, int64_t rb, int nvalid,
                             const uint64_t (&v)[R], int c0, int lane, bool narrow) {
    const int ln = (int)opaque((uint32_t)lane);
    const PayloadRef& p = s.pay;
    const uint32_t nv = (uint32_t)(nvalid > 0 ? nvalid : 0);
    const uint32_t off = (uint32_t)ln * 4u;  // byte offset of column 0; column c at + 256 c
    // keys and positions through buffer resources over the piece's outputs: stores of
    // ranks >= nvalid are dropped by the range check; afterwards only the positions stay
    // live
    uint32_t pos_of[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) pos_of[c] = comp_pos<PB>(v[c0 + c]);
    if (s.keys_out) {
        const rsrc_t r = buffer_rsrc(s.keys_out + o + rb, nv * 4u);
        if (s.f32) {
#pragma unroll
            for (int c = 0; c < NC; ++c) buffer_store(r, off + 256u * c, ordered_to_f32(comp_key<PB>(v[c0 + c])));
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) buffer_store(r, off + 256u * c, comp_key<PB>(v[c0 + c]));
        }
    }
    if (s.perm_out) {
        const rsrc_t r = buffer_rsrc(s.perm_out + o + rb, nv * 4u);
#pragma unroll
        for (int c = 0; c < NC; ++c) buffer_store(r, off + 256u * c, pos_of[c]);
    }
    if (p.channels == 0) return;
    constexpr int G = NC < 16 ? NC : 16;
#pragma unroll 1
    for (uint32_t ch = 0; ch < p.channels; ++ch) {
        const int lc = (int)opaque((uint32_t)ln);
        const uint32_t* pin = p.in + (int64_t)ch * p.cs + o * p.es;           // tile item 0
        uint32_t* pout = p.out + (int64_t)ch * p.cs + (o + rb) * p.es;        // rank rb
        const uint32_t es4 = (uint32_t)p.es * 4u;
        if (narrow) {
            // gather through the positions (the whole tile is addressable with 32-bit
            // offsets), stores through a buffer over the piece's outputs
            const rsrc_t rin = buffer_rsrc(pin, 0xFFFFFFFFu);
            const rsrc_t rout = buffer_rsrc(pout, nv * es4);
            const uint32_t loff = (uint32_t)lc * es4;
#pragma unroll
            for (int g = 0; g < NC; g += G) {
                uint32_t pv[G];
#pragma unroll
                for (int j = 0; j < G; ++j) {
                    const int q = 64 * (g + j) + lc;
                    const uint32_t src = (q < nvalid) ? pos_of[g + j] * es4 : 0u;
                    pv[j] = __builtin_amdgcn_raw_buffer_load_b32(rin, (int)src, 0, 0);
                }
#pragma unroll
                for (int j = 0; j < G; ++j) buffer_store(rout, loff + (uint32_t)(64 * (g + j)) * es4, pv[j]);
            }
        } else {
#pragma unroll
            for (int g = 0; g < NC; g += G) {
                uint32_t pv[G];
#pragma unroll
                for (int j = 0; j < G; ++j) {
                    const int q = 64 * (g + j) + lc;
                    pv[j] = *((q < nvalid) ? pin + (int64_t)pos_of[g + j] * p.es : pin);
                }
#pragma unroll
                for (int j = 0; j < G; ++j) {
                    const int q = 64 * (g + j) + lc;
                    if (q < nvalid) pout[(int64_t)q * p.es] = pv[j];
                }
            }
        }
    }
}

TS_DEV bool narrow_payload(const MergeArgs& a) {
    return (uint64_t)a.max_len * (uint64_t)a.s.pay.es * 4u <= (uint64_t(1) << 32);
}

// Tile of bin entry e (or none past the bin's count): offset and length, wave-uniform.
TS_DEV void bin_tile(const MergeArgs& a, int bin, uint32_t cnt, uint32_t e, int64_t& o, int& n) {
    o = 0;
    n = 0;
    if (e < cnt) {
        const int64_t t = entry_tile(a.bins[(int64_t)bin * a.s.num_tiles + e]);
        o = uniform64(a.s.offsets[t]);
        n = (int)uniform((uint32_t)(a.s.offsets[t + 1] - o));
    }
}

// Stage CPS columns (keys of positions 64 j + lane, j < CPS) of one tile into A at
// word `w0 + 64 j + lane`, 16 columns per batch of loads; positions >= n get the
// maximal key.
template <int CPS>
TS_DEV void stage_keys(uint32_t* A, const SortArgs& s, int64_t o, int n, int w0, int lane) {
    constexpr int G = CPS < 16 ? CPS : 16;
    const rsrc_t rk = buffer_rsrc(s.keys_in + o, (uint32_t)(n > 0 ? n : 0) * 4u);  // 0 past the end
#pragma unroll 1
    for (int g = 0; g < CPS; g += G) {
        uint32_t kk[G];
        buffer_load_columns<G>(rk, (uint32_t)lane * 4u + 256u * (uint32_t)g, kk);
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const uint32_t i = (uint32_t)(64 * (g + j) + lane);
            const uint32_t key = ((int)i < n) ? (s.f32 ? f32_to_ordered(kk[j]) : kk[j]) : 0xFFFFFFFFu;
            lds_store(A, (uint32_t)(w0 + (int)i) * 4u, key);
        }
    }
}

// Packed bin: P tiles, tile s at slot s (positions s*C .. s*C + C-1, C = 4096 / P).
template <int P>
TS_DEV void load_packed(uint32_t* A, uint64_t (&v)[R], const MergeArgs& a, int bin, uint32_t cnt,
                        uint32_t item, int lane) {
    constexpr int CPS = 64 / P;  // columns per slot
#pragma unroll
    for (int sl = 0; sl < P; ++sl) {
        int64_t o;
        int n;
        bin_tile(a, bin, cnt, item * P + sl, o, n);
        stage_keys<CPS>(A, a.s, o, n, sl * CPS * 64, lane);
    }
#pragma unroll
    for (int c = 0; c < R; ++c) {
        const uint32_t i = (uint32_t)(64 * c + lane);
        v[c] = make_comp<PACKED_POS_BITS>((uint32_t)(c / CPS), lds_load(A, i * 4u),
                                            (uint32_t)(64 * (c % CPS) + lane));
    }
}

template <int P>
TS_DEV void store_packed(const uint64_t (&v)[R], const MergeArgs& a, int bin, uint32_t cnt,
                         uint32_t item, int lane) {
    constexpr int CPS = 64 / P;
#pragma unroll
    for (int sl = 0; sl < P; ++sl) {
        int64_t o;
        int n;
        bin_tile(a, bin, cnt, item * P + sl, o, n);
        store_final_regs<CPS, PACKED_POS_BITS>(a.s, o, 0, n, v, sl * CPS, lane, narrow_payload(a));
    }
}

// Piece j of a long tile: positions j*4096 .. ; sorted runs go to run0.
TS_DEV void piece_range(const MergeArgs& a, uint64_t e, int64_t& o, int& n, uint32_t& base) {
    const int64_t t = entry_tile(e);
    const uint32_t j = entry_j(e);
    const int64_t to = uniform64(a.s.offsets[t]);
    const int64_t tn = uniform64(a.s.offsets[t + 1] - to);
    base = j * (uint32_t)K;
    o = to + base;
    const int64_t rem = tn - (int64_t)base;
    n = (int)(rem < K ? rem : K);
}

// KIND 0 .. 3: packing bin KIND (8, 4, 2, 1 tiles per wavefront); KIND 4: pieces of
// long tiles.  One launch per kind keeps every kernel straight-line code.
template <int KIND>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
void merge_sort_kernel(MergeArgs a) {
    __shared__ uint32_t A[MOVE_WORDS];
    constexpr int P = KIND < 4 ? (8 >> KIND) : 1;
    uint32_t cnt = uniform(a.counters[KIND]);
    if (KIND == 4 && cnt > (uint32_t)a.cap) cnt = (uint32_t)a.cap;
    const uint32_t items = (cnt + P - 1) / P;
    for (uint32_t item = blockIdx.x; item < items; item += gridDim.x) {
        const int lane = (int)opaque((uint32_t)lane_id());
        uint64_t v[R];
        if constexpr (KIND < 4) {
            load_packed<P>(A, v, a, KIND, cnt, item, lane);
        } else {
            int64_t o;
            int n;
            uint32_t base;
            piece_range(a, a.pieces[item], o, n, base);
            stage_keys<64>(A, a.s, o, n, 0, lane);
#pragma unroll
            for (int c = 0; c < R; ++c) {
                const uint32_t i = (uint32_t)(64 * c + lane);
                v[c] = make_comp<POS_BITS>(0u, lds_load(A, i * 4u), base + i);
            }
        }
        bitonic_sort4096(A, v, lane);
        if constexpr (KIND < 4) {
            store_packed<P>(v, a, KIND, cnt, item, lane);
        } else {
            int64_t o;
            int n;
            uint32_t base;
            piece_range(a, a.pieces[item], o, n, base);
            const int ln = (int)opaque((uint32_t)lane);
            uint64_t* rb = a.run0 + o;
#pragma unroll
            for (int c = 0; c < R; ++c) {
                const int r = 64 * c + ln;
                if (r < n) *(uint64_t*)((char*)rb + (uint32_t)r * 8u) = v[c];
            }
        }
    }
}

// Workgroup bins (4, 5, 6): one tile of up to 4096 H keys per workgroup of H wavefronts,
// sorted whole by bitonic_sort_wide; wavefront h loads items 4096 h .. and stores ranks
// 4096 h .. (keys, permutation and payload).
template <int H>
__global__ __launch_bounds__(64 * H) __attribute__((amdgpu_waves_per_eu(2)))
void merge_wide_kernel(MergeArgs a) {
    constexpr int BIN = H == 2 ? 4 : H == 4 ? 5 : 6;
    __shared__ __attribute__((aligned(16))) uint32_t A[wide_bitonic_words<H>()];
    const int h = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t cnt = uniform(a.counters[bin_counter(BIN)]);
    for (uint32_t item = blockIdx.x; item < cnt; item += gridDim.x) {
        const int lane = (int)opaque((uint32_t)lane_id());
        int64_t o;
        int n;
        bin_tile(a, BIN, cnt, item, o, n);
        const int nw = n > 4096 * h ? n - 4096 * h : 0;  // items of this wavefront's part
        uint32_t* Aw = A + h * MOVE_WORDS;
        __syncthreads();  // the previous tile's exchanges are done
        stage_keys<64>(Aw, a.s, o + 4096 * h, nw, 0, lane);
        uint64_t v[R];
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const uint32_t i = (uint32_t)(64 * c + lane);
            v[c] = make_comp<POS_BITS>(0u, lds_load(Aw, i * 4u), (uint32_t)(4096 * h) + i);
        }
        bitonic_sort_wide<H>(A, v, h, lane);
        store_final_regs<R>(a.s, o, 4096 * h, nw, v, 0, lane, narrow_payload(a));
    }
}

// ---------------------------------------------------------------------------------
// Merge round r: runs of length L = 4096 << r are merged in pairs.  Output piece u of a
// tile covers outputs u*4096 .. of the pair p = u >> (r+1) that starts at ps.
struct PieceGeom {
    int64_t o, n;      // tile
    int64_t ps;        // pair start (tile position)
    int64_t la, lb;    // lengths of the pair's two runs (lb may be 0)
    int64_t d0, d1;    // output range within the pair
    bool last;         // this round finishes the tile
};

TS_DEV PieceGeom piece_geom(const MergeArgs& a, uint64_t e, int r) {
    PieceGeom g;
    const int64_t t = entry_tile(e);
    const int64_t u = entry_j(e);
    g.o = a.s.offsets[t];
    g.n = a.s.offsets[t + 1] - g.o;
    const int64_t L = (int64_t)K << r;
    g.ps = (u >> (r + 1)) * 2 * L;
    const int64_t rest = g.n - g.ps;
    g.la = rest < L ? rest : L;
    g.lb = rest - g.la < L ? rest - g.la : L;
    g.d0 = u * K - g.ps;
    const int64_t d1 = g.d0 + K;
    g.d1 = d1 < g.la + g.lb ? d1 : g.la + g.lb;
    g.last = 2 * L >= g.n;
    return g;
}

// Number of A elements among the d smallest of the union of A and B (all distinct).
TS_DEV int64_t corank(const uint64_t* A, int64_t la, const uint64_t* B, int64_t lb, int64_t d) {
    int64_t lo = d - lb > 0 ? d - lb : 0;
    int64_t hi = d < la ? d : la;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (A[mid] > B[d - 1 - mid]) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void merge_corank_kernel(MergeArgs a, int r) {
    const uint32_t cnt = a.counters[8 + r] < (uint32_t)a.cap ? a.counters[8 + r] : (uint32_t)a.cap;
    const uint64_t* list = a.round_lists + (int64_t)r * a.cap;
    int32_t* cr = a.coranks + (int64_t)r * a.cap * 2;
    const uint64_t* in = (r & 1) ? a.run1 : a.run0;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += gridDim.x * blockDim.x) {
        const PieceGeom g = piece_geom(a, list[e], r);
        const uint64_t* A = in + g.o + g.ps;
        const uint64_t* B = A + ((int64_t)K << r);
        cr[2 * (int64_t)e] = (int32_t)corank(A, g.la, B, g.lb, g.d0);
        cr[2 * (int64_t)e + 1] = (int32_t)corank(A, g.la, B, g.lb, g.d1);
    }
}

// LAST = true handles the output pieces of tiles that this round finishes (final keys,
// permutation and payload), LAST = false the others (runs for the next round); the two
// are separate launches so that each is a straight-line kernel.
template <bool LAST>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
void merge_round_kernel(MergeArgs a, int r) {
    __shared__ uint32_t A[MOVE_WORDS];
    const uint32_t cnt = uniform(a.counters[8 + r] < (uint32_t)a.cap ? a.counters[8 + r] : (uint32_t)a.cap);
    const uint64_t* list = a.round_lists + (int64_t)r * a.cap;
    const int32_t* cr = a.coranks + (int64_t)r * a.cap * 2;
    const uint64_t* in = (r & 1) ? a.run1 : a.run0;
    uint64_t* out_run = (r & 1) ? a.run0 : a.run1;
    for (uint32_t w = blockIdx.x; w < cnt; w += gridDim.x) {
        const PieceGeom g = piece_geom(a, list[w], r);
        if (g.last != LAST) continue;
        const int lane = (int)opaque((uint32_t)lane_id());
        const int64_t i0 = uniform((uint32_t)cr[2 * (int64_t)w]);
        const int64_t i1 = uniform((uint32_t)cr[2 * (int64_t)w + 1]);
        const int la = (int)(i1 - i0);                        // from run A
        const int lb = (int)((g.d1 - g.d0) - la);             // from run B
        const int64_t k0 = g.d0 - i0;
        // element q of the bitonic sequence: A ascending, padding, B descending; all
        // addresses are 32-bit offsets from the pair's first composite
        const uint64_t* base = in + uniform64(g.o + g.ps);
        const uint32_t offA = (uint32_t)i0;
        const uint32_t offB = (uint32_t)(((int64_t)K << r) + k0 + (K - 1));
        uint64_t v[R];
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const int q = 64 * c + lane;
            const bool inA = q < la;
            const bool inB = q >= K - lb;
            const uint32_t idx = inA ? offA + (uint32_t)q : (inB ? offB - (uint32_t)q : 0u);
            const uint64_t x = *(const uint64_t*)((const char*)base + idx * 8u);
            v[c] = (inA || inB) ? x : PAD;
            if ((c & 15) == 15) __builtin_amdgcn_sched_barrier(0);  // bound live addresses
        }
        bitonic_merge4096(A, v, lane);
        const int ln = (int)opaque((uint32_t)lane);
        const int64_t ob = g.ps + g.d0;  // tile position of output rank 0
        const int nout = (int)(g.d1 - g.d0);
        if (LAST) {
            store_final_regs<R>(a.s, g.o, ob, nout, v, 0, lane, narrow_payload(a));
        } else {
            uint64_t* ob_ptr = out_run + g.o + ob;
#pragma unroll
            for (int c = 0; c < R; ++c) {
                const int q = 64 * c + ln;
                if (q < nout) ob_ptr[q] = v[c];
            }
        }
    }
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int rounds_for(int64_t max_len) {
    int r = 0;
    while (((int64_t)K << r) < max_len) ++r;
    return r;
}

}  // namespace

void set_merge_pack(int v) { g_merge_pack = v; }
void set_merge_wide(int v) { g_merge_wide = v; }

MergeLayout merge_layout(int64_t num_tiles, int64_t total_len, int64_t max_len) {
    MergeLayout L{};
    // merge rounds only for tiles longer than the workgroup bins take
    L.rounds = max_len > g_merge_wide ? rounds_for(max_len) : 0;
    L.cap = total_len / K + num_tiles + 1;
    size_t off = 256;  // header: error word and counters
    L.bins = off;
    off += align256((size_t)num_tiles * NUM_BINS * 8);
    L.pieces = off;
    off += align256((size_t)L.cap * 8);
    L.round_lists = off;
    off += align256((size_t)L.rounds * L.cap * 8);
    L.coranks = off;
    off += align256((size_t)L.rounds * L.cap * 8);
    L.run0 = off;
    off += align256(L.rounds >= 1 ? (size_t)total_len * 8 : 0);
    L.run1 = off;
    off += align256(L.rounds >= 2 ? (size_t)total_len * 8 : 0);
    L.total = off;
    return L;
}

hipError_t launch_sort_merge(const SortArgs& s, int64_t total_len, int64_t max_len, void* ws,
                             hipStream_t st) {
    if (s.num_tiles == 0) return hipSuccess;
    const MergeLayout L = merge_layout(s.num_tiles, total_len, max_len);
    char* w = (char*)ws;
    MergeArgs a{};
    a.s = s;
    a.counters = (uint32_t*)ws + MERGE_COUNTER_WORD;
    a.bins = (uint64_t*)(w + L.bins);
    a.pieces = (uint64_t*)(w + L.pieces);
    a.round_lists = (uint64_t*)(w + L.round_lists);
    a.coranks = (int32_t*)(w + L.coranks);
    a.run0 = (uint64_t*)(w + L.run0);
    a.run1 = (uint64_t*)(w + L.run1);
    a.cap = L.cap;
    a.rounds = L.rounds;
    a.pack = g_merge_pack;
    a.max_len = max_len;
    a.total_len = total_len;
    a.wide_max = g_merge_wide > K ? g_merge_wide : K;

    hipError_t e = launch_fill_zero(a.counters, MERGE_COUNTER_BYTES, st);
    if (e != hipSuccess) return e;
    {
        int64_t g = (s.num_tiles + BIN_THREADS - 1) / BIN_THREADS;
        if (g > 1024) g = 1024;
        hipLaunchKernelGGL(merge_bin_kernel, dim3((unsigned)g), dim3(BIN_THREADS), 0, st, a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    {
        // the workgroup bins (whole tiles of up to 32768 keys), largest first
        if (max_len > K && g_merge_wide > K) {
            hipLaunchKernelGGL(merge_wide_kernel<8>, dim3(persistent_grid((const void*)merge_wide_kernel<8>, 512, 0,
                                                                          s.num_tiles)),
                               dim3(512), 0, st, a);
            hipLaunchKernelGGL(merge_wide_kernel<4>, dim3(persistent_grid((const void*)merge_wide_kernel<4>, 256, 0,
                                                                          s.num_tiles)),
                               dim3(256), 0, st, a);
            hipLaunchKernelGGL(merge_wide_kernel<2>, dim3(persistent_grid((const void*)merge_wide_kernel<2>, 128, 0,
                                                                          s.num_tiles)),
                               dim3(128), 0, st, a);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        // pieces (the longest chains of work), then the packing bins
        const void* kinds[5] = {(const void*)merge_sort_kernel<4>, (const void*)merge_sort_kernel<3>,
                                (const void*)merge_sort_kernel<2>, (const void*)merge_sort_kernel<1>,
                                (const void*)merge_sort_kernel<0>};
        const int64_t bound[5] = {L.cap, s.num_tiles, s.num_tiles, s.num_tiles, s.num_tiles};
        for (int k = 0; k < 5; ++k) {
            const int g = persistent_grid(kinds[k], 64, 0, bound[k]);
            switch (k) {
                case 0: hipLaunchKernelGGL(merge_sort_kernel<4>, dim3(g), dim3(64), 0, st, a); break;
                case 1: hipLaunchKernelGGL(merge_sort_kernel<3>, dim3(g), dim3(64), 0, st, a); break;
                case 2: hipLaunchKernelGGL(merge_sort_kernel<2>, dim3(g), dim3(64), 0, st, a); break;
                case 3: hipLaunchKernelGGL(merge_sort_kernel<1>, dim3(g), dim3(64), 0, st, a); break;
                default: hipLaunchKernelGGL(merge_sort_kernel<0>, dim3(g), dim3(64), 0, st, a); break;
            }
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    for (int r = 0; r < L.rounds; ++r) {
        int64_t gc = (L.cap + 255) / 256;
        if (gc > 2048) gc = 2048;
        hipLaunchKernelGGL(merge_corank_kernel, dim3((unsigned)gc), dim3(256), 0, st, a, r);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        for (int last = 0; last < 2; ++last) {
            auto kern = last ? merge_round_kernel<true> : merge_round_kernel<false>;
            const int g = persistent_grid((const void*)kern, 64, 0, L.cap);
            hipLaunchKernelGGL(kern, dim3(g), dim3(64), 0, st, a, r);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

}  // namespace ts
