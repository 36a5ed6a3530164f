// Stable w-way partition of tiles held in LDS, without LDS bank conflicts.
//
// Problem: Afshani & Sitchinava, Sec. 1 ("Problems of interest", partition) and
// the abstract (partitioning = sorting an input with n/w copies of each label).
//
// Schedule ("alternating-direction binary split"): one pass per label bit,
// least significant first.  A pass reads the tile in its current order, 64
// consecutive items per wave instruction ("column"), and writes the items whose
// bit is 0 forward from the front of the tile and the items whose bit is 1
// backward from the back.  After k columns the zero block ends at z and the one
// block starts at N - (64k - z); both heads therefore sit on the same bank
// residue (N is a multiple of 64), and the next column's zeros (forward from
// that residue) and ones (backward from it) cover 64 cyclically consecutive
// item slots: one per bank, i.e. every write instruction respects the paper's
// Conflict Avoidance Condition (Sec. 1).  Reading the result zero block forward
// and one block backward ("virtual order") restores input order inside each
// half, so each pass is a stable split and nbits passes are an LSD radix sort on
// the label -- the stable partition.  The virtual-order reads are conflict-free
// for the same reason (a column meets the turning point at most once, and the
// two pieces cover complementary residues).  The alternation of directions plays
// the role of the "alternating order" rows of Lemma 1 (Sec. 2).
//
// Per tile: labels and one payload word are packed in a 64-bit item
// (hi = source position << 16 | label, lo = payload) and live in registers
// between passes; LDS holds one copy of the tile (8 bytes per item).  The next
// tile's labels and payload are loaded into registers while the current tile is
// being split, so HBM latency overlaps the LDS work.
#include <algorithm>
#include <cstdint>

#include "common.hpp"
#include "kernels.hpp"

namespace ts {

namespace {

// Arguments of the split kernel, for its three uses: the stable partition (MODE 0: item
// = label + position + one payload word), the LSD radix sort of 32-bit keys in a tile
// (MODE 1: item = ordered key + position) and one pass of the device-wide radix sort
// (MODE 2: item = ordered key + payload word; the tile is split on one digit and every
// digit block is stored at its place in the whole array).
struct SplitArgs {
    const uint32_t* keys_in;    // labels or keys
    uint32_t* keys_out;
    const uint32_t* pay_in;     // MODE 0 only, one channel
    uint32_t* pay_out;
    int64_t pay_es;
    uint32_t has_pay;
    int32_t* perm_out;
    int64_t num_tiles;
    uint32_t num_classes;       // MODE 0: labels must be below this
    int nbits;                  // bits to split on
    uint32_t validate;
    uint32_t f32;               // MODE 1: keys are binary32 patterns; MODE 2: map them on load
    uint32_t* err;
    // MODE 2 only
    int shift;                  // the digit is bits shift .. shift + nbits - 1 of the key
    uint32_t f32_out;           // map ordered keys back to binary32 on store
    const uint32_t* hist;       // [RADIX_DIGITS][num_tiles] digit counts of every tile
    const uint32_t* goff;       // [RADIX_DIGITS][num_tiles] exclusive prefix of hist in that order
    int64_t n_total;            // length of the whole array (destinations are below it)
    // Payload words gathered from global memory at the store (out[v] = in[position of
    // rank v]): MODE 1 for small batches, where a second launch costs more; MODE 0 for the
    // channels after the first
    PayloadRef gpay;
};

template <int CPW>
struct TileLoad {
    int64_t o;   // first item of the tile
    int n;       // tile length (or -1 when there is no tile)
    uint32_t lab[CPW];
    uint32_t pay[CPW];
};

// Issue the global loads of one tile (no waits) through buffer resources over the
// tile: lanes past the end read 0 (the hardware range check) and are replaced by
// padding later.
template <int CPW, int CAP, bool NT = false>
TS_DEV void issue_tile_load(const SplitArgs& a, const int64_t* __restrict__ offs, int64_t t,
                            int w, int lane, TileLoad<CPW>& L) {
    // Branch-free: an absent tile reads the offsets of tile 0 and loads nothing, so the
    // previous contents of L never have to be kept alive.
    const bool exists = t < a.num_tiles;
    const int64_t tt = exists ? t : 0;
    const int64_t o = offs[tt];
    const int64_t len = offs[tt + 1] - o;
    L.o = o;
    L.n = !exists ? -1 : ((len > CAP) ? -2 : (int)len);
    const uint32_t nn = (uint32_t)((L.n > 0) ? L.n : 0);
    const uint32_t off = ((uint32_t)(64 * w * CPW) + (uint32_t)lane) * 4u;
    buffer_load_columns<CPW, NT>(buffer_rsrc(a.keys_in + o, nn * 4u), off, L.lab);
    const uint32_t es = (uint32_t)a.pay_es;
    const rsrc_t rp = buffer_rsrc(a.pay_in + o * (int64_t)es, a.has_pay ? nn * es * 4u : 0u);
    if (es == 1) buffer_load_columns<CPW, NT>(rp, off, L.pay);
    else buffer_load_columns_strided<CPW, NT>(rp, off * es, 256u * es, L.pay);
}

template <int NW, int CAP, int WPE, int MODE, int PF = -1, int NTM = 0>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(WPE > 0 ? WPE : 1)))
void split_kernel(SplitArgs a, const int64_t* __restrict__ offs) {
    constexpr int CPW = CAP / 64 / NW;  // columns per wave
    constexpr bool NTL = (NTM & 1) != 0, NTS = (NTM & 2) != 0;  // streaming loads / stores
    // Whether the next tile's loads are issued before this tile is split (PF = 1 / 0).
    // By default narrow, uncapped waves prefetch and the rest load each tile when they
    // start it (WPE < 0: never prefetch).
    constexpr bool PREFETCH = PF >= 0 ? PF == 1 : (CPW <= 16 && WPE == 0);
    __shared__ uint64_t A[CAP];
    __shared__ int wz[NW];
    const int lane0 = lane_id();
    const int w0 = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t lmask = (MODE == 0) ? (1u << a.nbits) - 1u : 0xFFFFFFFFu;
    const bool has_pay = a.has_pay != 0;

    TileLoad<CPW> L;
    // A radix pass runs one workgroup per tile (grid = num_tiles), XCD-contiguous: the
    // digit blocks of neighbouring tiles share cache lines of the output and of the
    // count tables.
    int64_t t = (MODE == 2) ? xcd_contiguous(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    issue_tile_load<CPW, CAP, NTL>(a, offs, t, w0, lane0, L);

    for (; t < a.num_tiles; t += gridDim.x) {
        // lane-derived values (positions, addresses) are recomputed per tile rather
        // than hoisted out of the tile loop and kept live across it
        const int lane = (int)opaque((uint32_t)lane0);
        const int w = opaque_s(w0);
        const int64_t o = L.o;
        const int n = L.n;
        if (n == -2) {  // longer than this kernel's capacity: skip and flag
            if (threadIdx.x == 0) atomicOr(a.err, ERR_TILE_TOO_LONG);
            issue_tile_load<CPW, CAP, NTL>(a, offs, t + gridDim.x, w, lane, L);
            continue;
        }
        // The tile is padded to the kernel capacity: every wave always owns CPW full
        // columns, so all loop bounds and branches below are wave-uniform constants.
        constexpr int N = CAP;

        // ---- items of this tile: column k, lane l holds item 64k + l.  Padding items
        //      carry the largest label (key) and a position >= n, so they end up last.
        uint64_t e[CPW];
        bool bad = false;
#pragma unroll
        for (int j = 0; j < CPW; ++j) {
            const int i = 64 * (w * CPW + j) + lane;
            uint32_t lab = lmask, pay = 0;
            if (i < n) {
                lab = L.lab[j];
                if (MODE == 0) {
                    bad |= lab >= a.num_classes;
                    lab &= lmask;
                    pay = L.pay[j];
                } else if (a.f32) {
                    lab = f32_to_ordered(lab);
                }
                if (MODE == 2) pay = has_pay ? L.pay[j] : (uint32_t)(o + i);  // no payload: the index
            }
            e[j] = (MODE == 0) ? pack(((uint32_t)i << 16) | lab, pay)
                               : pack(lab, MODE == 2 ? pay : (uint32_t)i);
        }
        if (a.validate) flag_error(a.err, bad, ERR_BAD_LABEL);

        // ---- radix pass: lane l, quarter q stands for digit d = 64q + l; its count and
        //      output offset in this tile are loaded now, so that they arrive while the
        //      tile is split
        constexpr int RQ = (MODE == 2) ? RADIX_DIGITS / 64 : 1;
        uint32_t rcnt[RQ], rgoff[RQ];
        if constexpr (MODE == 2) {
#pragma unroll
            for (int q = 0; q < RQ; ++q) {
                const int64_t idx = (int64_t)(64 * q + lane) * a.num_tiles + t;
                rcnt[q] = a.hist[idx];
                rgoff[q] = a.goff[idx];
            }
        }

        // ---- prefetch the next tile while this one is split in LDS
        if (PREFETCH) issue_tile_load<CPW, CAP, NTL>(a, offs, t + gridDim.x, w, lane, L);

        // ---- one stable split per label bit.  Addresses are byte offsets into A built from
        //      one lane-dependent register plus wave-uniform scalars and the DS immediate
        //      offset, so no per-column address registers stay live across passes.
        const uint32_t lane8 = (uint32_t)lane * 8u;
        const uint32_t neg_lane8 = 0u - lane8;
        const uint32_t fwd_base = lane8 + (uint32_t)(w * CPW * 512);  // column j at + 512 j
        const int bit0 = (MODE == 2) ? a.shift : 0;
        for (int b = 0; b < a.nbits; ++b) {
            // Zero masks of this wave's columns; zeros before this wave's first column (zb)
            // and in the whole tile (zt).
            constexpr bool KEEP = (NW > 1);  // masks are kept between the two loops
            uint64_t zm[KEEP ? CPW : 1];
            int zb = 0, zt = 0;
            if (KEEP) {
                int zc = 0;
#pragma unroll
                for (int j = 0; j < CPW; ++j) {
                    zm[j] = ballot(((hi32(e[j]) >> (b + bit0)) & 1u) == 0u);
                    zc += popc64(zm[j]);
                }
                if (lane == 0) wz[w] = zc;
                __syncthreads();  // every wave has read the previous pass and posted its count
                // lane q < NW holds wave q's count in the low half and, when q < w, again in
                // the high half; one prefix sum over the first NW lanes yields zt and zb
                const uint32_t mine = (lane < NW) ? (uint32_t)wz[lane] : 0u;
                const uint32_t both = row_prefix_sum<NW>(mine | ((lane < w) ? mine << 16 : 0u));
                const uint32_t s = (uint32_t)__builtin_amdgcn_readlane((int)both, NW - 1);
                zt = (int)(s & 0xFFFFu);
                zb = (int)(s >> 16);
            }
            if (NW == 1) wave_lds_fence();  // the previous pass's reads stay before these writes
            // Write: a zero of column k goes to z + r0 and a one to N-1-(64k-z)-(lane-r0),
            // with z the zeros before the column and r0 the zeros in lower lanes; i.e. to
            // z + r0 + (one ? N-1-64k-lane : 0), the bracket folded into the rank count.
            int z = zb;  // zeros before the current column (whole tile, in order)
#pragma unroll
            for (int j = 0; j < CPW; ++j) {
                const int k = w * CPW + j;
                const uint64_t zj = KEEP ? zm[KEEP ? j : 0] : ballot(((hi32(e[j]) >> (b + bit0)) & 1u) == 0u);
                const uint32_t one_off = zero_if_mask(zj, (uint32_t)(N - 1 - 64 * k) - (uint32_t)lane);
                const uint32_t pos = count_below_plus(zj, one_off) + (uint32_t)z;
                lds_store(A, pos * 8u, e[j]);
                z += popc64(zj);
            }
            if (NW == 1) zt = z;
            if (NW > 1) __syncthreads();  // the split tile is complete
            else wave_lds_fence();
            // Read back in virtual order: zero block forward, then one block backward.
            const uint32_t rev_base =
                (uint32_t)__builtin_amdgcn_readfirstlane((N - 1 + zt - 64 * w * CPW - 64 * (CPW - 1)) * 8) +
                neg_lane8;  // column j (reversed) at + 512 (CPW-1-j)
            // The turning point zt falls inside at most one wave's columns: the others take
            // one uniform branch for all of theirs.
            const int first = 64 * w * CPW;
            if (first + 64 * CPW <= zt) {
#pragma unroll
                for (int j = 0; j < CPW; ++j) e[j] = lds_load(A, fwd_base + 512u * j);
            } else if (first >= zt) {
#pragma unroll
                for (int j = 0; j < CPW; ++j) e[j] = lds_load(A, rev_base + 512u * (CPW - 1 - j));
            } else {
#pragma unroll
                for (int j = 0; j < CPW; ++j)
                    e[j] = lds_load(A, (lane < zt - first - 64 * j) ? fwd_base + 512u * j
                                                                   : rev_base + 512u * (CPW - 1 - j));
            }
        }

        if constexpr (MODE == 2) {
            // ---- digit d's block of this tile goes to goff[d][t] onward; in the split
            //      tile it starts after the blocks of the smaller digits, so the item of
            //      digit d at tile rank v goes to v + delta[d], delta[d] = goff[d][t] -
            //      (counts of the digits below d).  Every item fetches delta of its digit
            //      from lane d mod 64 of quarter d / 64 with ds_bpermute (no bank conflicts).
            uint32_t delta[RQ];
            uint32_t below = 0;  // counts of the digits of the previous quarters
#pragma unroll
            for (int q = 0; q < RQ; ++q) {
                const uint32_t inc = wave_inclusive_scan_u32(rcnt[q]);
                delta[q] = rgoff[q] - (below + inc - rcnt[q]);
                below += (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
            }
            const int ls = (int)opaque((uint32_t)lane);
            const uint32_t dmask = (1u << a.nbits) - 1u;
            const uint32_t ntot = (uint32_t)a.n_total;
            uint32_t dst[CPW];
            bool bad = false;  // counts that disagree with the tile: not stored, recorded
#pragma unroll
            for (int j = 0; j < CPW; ++j) {
                const uint32_t v = (uint32_t)(64 * (w * CPW + j) + ls);
                const uint32_t d = (hi32(e[j]) >> a.shift) & dmask;
                const int src = (int)((d & 63u) * 4u);
                uint32_t dl = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)delta[0]);
#pragma unroll
                for (int q = 1; q < RQ; ++q) {
                    const uint32_t x = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)delta[q]);
                    dl = ((d >> 6) == (uint32_t)q) ? x : dl;
                }
                const bool real = v < (uint32_t)n;
                const uint32_t g = dl + v;
                bad |= real && g >= ntot;
                dst[j] = (real && g < ntot) ? g : ntot;  // ntot: past the end, dropped
            }
            if (a.n_total <= (int64_t)0x3FFFFFFF) {
                // byte offsets fit in 32 bits: buffer stores over the whole output, the
                // hardware range check drops the ones at ntot
                const rsrc_t rk = buffer_rsrc(a.keys_out, ntot * 4u);
#pragma unroll
                for (int j = 0; j < CPW; ++j) {
                    const uint32_t h = hi32(e[j]);
                    buffer_store<false>(rk, dst[j] * 4u, a.f32_out ? ordered_to_f32(h) : h);
                }
                if (a.pay_out) {
                    const rsrc_t rp = buffer_rsrc(a.pay_out, ntot * 4u);
#pragma unroll
                    for (int j = 0; j < CPW; ++j) buffer_store<false>(rp, dst[j] * 4u, lo32(e[j]));
                }
            } else {
#pragma unroll
                for (int j = 0; j < CPW; ++j) {
                    if (dst[j] < ntot) {
                        const uint32_t h = hi32(e[j]);
                        a.keys_out[dst[j]] = a.f32_out ? ordered_to_f32(h) : h;
                        if (a.pay_out) a.pay_out[dst[j]] = lo32(e[j]);
                    }
                }
            }
            if (a.validate) flag_error(a.err, bad, ERR_BAD_OFFSETS);
        } else
        // ---- store in order (coalesced: column k covers items 64k .. 64k+63), one
        //      uniform branch per output; stores past the end of the tile are dropped by
        //      the buffer range check
        {
            const int ls = (int)opaque((uint32_t)lane);
            const uint32_t off = ((uint32_t)(64 * w * CPW) + (uint32_t)ls) * 4u;
            const uint32_t nb = (uint32_t)n * 4u;
            uint32_t v[CPW];
            if (a.keys_out) {
                const rsrc_t r = buffer_rsrc(a.keys_out + o, nb);
#pragma unroll
                for (int j = 0; j < CPW; ++j) {
                    const uint32_t h = hi32(e[j]);
                    v[j] = (MODE == 0) ? (h & 0xFFFFu) : (a.f32 ? ordered_to_f32(h) : h);
                }
#pragma unroll
                for (int j = 0; j < CPW; ++j) buffer_store<NTS>(r, off + 256u * j, v[j]);
            }
            if (MODE == 0 && has_pay) {
                const uint32_t es = (uint32_t)a.pay_es;
                const rsrc_t r = buffer_rsrc(a.pay_out + o * (int64_t)es, nb * es);
                if (es == 1) {
#pragma unroll
                    for (int j = 0; j < CPW; ++j) buffer_store<NTS>(r, off + 256u * j, lo32(e[j]));
                } else {
#pragma unroll
                    for (int j = 0; j < CPW; ++j) buffer_store<NTS>(r, off * es + 256u * es * j, lo32(e[j]));
                }
            }
            if (a.perm_out) {
                const rsrc_t r = buffer_rsrc(a.perm_out + o, nb);
#pragma unroll
                for (int j = 0; j < CPW; ++j) v[j] = (MODE == 0) ? (hi32(e[j]) >> 16) : lo32(e[j]);
#pragma unroll
                for (int j = 0; j < CPW; ++j) buffer_store<NTS>(r, off + 256u * j, v[j]);
            }
            if (MODE != 2 && a.gpay.out != nullptr) {
                // rank v takes the words of its source position; both stay inside the tile
                // (MODE 0: the payload channels after the first, which rides in the item)
                const int64_t es = a.gpay.es, cs = a.gpay.cs;
                for (uint32_t c = 0; c < a.gpay.channels; ++c) {
                    const uint32_t* src = a.gpay.in + o * es + (int64_t)c * cs;
                    uint32_t* dst = a.gpay.out + o * es + (int64_t)c * cs;
                    // ranks below n hold real items, whose positions are below n; the
                    // padding ranks load and store nothing
#pragma unroll
                    for (int j = 0; j < CPW; ++j) {
                        const int r = 64 * (w * CPW + j) + ls;
                        const uint32_t from = (MODE == 0) ? (hi32(e[j]) >> 16) : lo32(e[j]);
                        v[j] = (r < n) ? src[(int64_t)from * es] : 0u;
                    }
#pragma unroll
                    for (int j = 0; j < CPW; ++j) {
                        const int r = 64 * (w * CPW + j) + ls;
                        if (r < n) dst[(int64_t)r * es] = v[j];
                    }
                }
            }
        }
        if (!PREFETCH) issue_tile_load<CPW, CAP, NTL>(a, offs, t + gridDim.x, w, lane, L);
    }
}

// ONESHOT: one workgroup per tile (the hardware dispatcher overlaps the tiles of the
// workgroups resident on a CU) instead of a persistent grid.
template <int NW, int CAP, int WPE = 0, int MODE = 0, int PF = -1, int NTM = 0, bool ONESHOT = false>
hipError_t launch_split(const SplitArgs& a, const int64_t* offs, hipStream_t s) {
    auto kern = split_kernel<NW, CAP, WPE, MODE, PF, NTM>;
    const int grid = ONESHOT ? (int)std::min<int64_t>(a.num_tiles, INT32_MAX)
                             : persistent_grid((const void*)kern, NW * 64, 0, a.num_tiles);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NW * 64), 0, s, a, offs);
    return hipGetLastError();
}

// Launch shape for the kernels without a tuned variant table (tuning knob "oneshot"):
// 1 (default) one workgroup per tile with streaming global accesses, 0 a persistent
// grid that loads the next tile while it splits the current one.
int g_oneshot = 1;

template <int NW, int CAP, int WPE = 0, int MODE = 0>
hipError_t launch_split_shaped(const SplitArgs& a, const int64_t* offs, hipStream_t s) {
    return g_oneshot ? launch_split<NW, CAP, WPE, MODE, 0, 3, true>(a, offs, s)
                     : launch_split<NW, CAP, WPE, MODE>(a, offs, s);
}

}  // namespace

void set_oneshot(int v) { g_oneshot = v; }
bool tile_oneshot() { return g_oneshot != 0; }

int64_t partition_split_capacity() { return 16384; }

// Kernel variant for 4096-item tiles (tuning knob "partition_waves_4096"); the default
// is one 8-wave workgroup per tile, four resident per CU.
static int g_part_nw4096 = 168;
void set_partition_waves(int nw) { g_part_nw4096 = nw; }

hipError_t launch_partition_split(const PartitionArgs& p, int64_t max_len, hipStream_t s) {
    if (p.num_tiles == 0) return hipSuccess;
    SplitArgs a{};
    a.keys_in = p.labels_in;
    a.keys_out = p.labels_out;
    a.pay_in = p.pay.in;
    a.pay_out = p.pay.out;
    a.pay_es = p.pay.es;
    a.has_pay = p.pay.channels > 0;
    a.perm_out = p.perm_out;
    a.num_tiles = p.num_tiles;
    a.num_classes = p.num_classes;
    a.nbits = p.nbits;
    a.validate = p.validate;
    a.err = p.err;
    if (p.pay.channels > 1)
        a.gpay = PayloadRef{p.pay.in + p.pay.cs, p.pay.out + p.pay.cs, p.pay.channels - 1, p.pay.es, p.pay.cs};
    const int64_t* o = p.offsets;
    if (max_len <= 1024) return launch_split_shaped<4, 1024>(a, o, s);
    if (max_len <= 2048) return launch_split_shaped<4, 2048>(a, o, s);
    if (max_len <= 4096) {
        switch (g_part_nw4096) {
            case 1: return launch_split<1, 4096>(a, o, s);
            case 2: return launch_split<2, 4096>(a, o, s);
            case 4: return launch_split<4, 4096>(a, o, s);
            case 16: return launch_split<16, 4096>(a, o, s);
            // persistent grids: 1xx = 8 or 4 waves with registers capped for xx/2 waves per SIMD
            case 104: return launch_split<4, 4096, 4>(a, o, s);         // 4 waves, 4 workgroups per CU
            case 106: return launch_split<8, 4096, 6, 0, 1>(a, o, s);   // 3 workgroups per CU, prefetch
            case 108: return launch_split<8, 4096, 8>(a, o, s);         // 4 workgroups per CU
            // one workgroup per tile, streaming loads and stores (176: plain accesses)
            case 164: return launch_split<4, 4096, 4, 0, 0, 3, true>(a, o, s);
            case 166: return launch_split<8, 4096, 6, 0, 0, 3, true>(a, o, s);
            case 168: return launch_split<8, 4096, 8, 0, 0, 3, true>(a, o, s);
            case 176: return launch_split<8, 4096, 6, 0, 0, 0, true>(a, o, s);
            default: return launch_split_shaped<8, 4096>(a, o, s);
        }
    }
    if (max_len <= 8192) return launch_split_shaped<8, 8192>(a, o, s);
    return launch_split_shaped<16, 16384>(a, o, s);
}

hipError_t launch_radix_pass(const RadixPass& r, hipStream_t s) {
    if (r.num_tiles == 0) return hipSuccess;
    SplitArgs a{};
    a.keys_in = r.keys_in;
    a.keys_out = r.keys_out;
    a.pay_in = r.pay_in;
    a.pay_out = r.pay_out;
    a.pay_es = 1;
    a.has_pay = r.pay_in != nullptr;
    a.num_tiles = r.num_tiles;
    a.nbits = r.nbits;
    a.f32 = r.f32_in;
    a.err = r.err;
    a.shift = r.shift;
    a.f32_out = r.f32_out;
    a.hist = r.hist;
    a.goff = r.goff;
    a.n_total = r.n_total;
    a.validate = 1;
    static_assert(RADIX_TILE_KEYS == 4096 && RADIX_TILE_PAY == 8192, "the pass kernel's tile sizes");
    if (r.tile == RADIX_TILE_PAY) return launch_split<16, 8192, 8, 2, 0, 1, true>(a, r.offsets, s);
    return launch_split<8, 4096, 8, 2, 0, 1, true>(a, r.offsets, s);
}

hipError_t launch_sort_split(const SortArgs& q, int64_t max_len, hipStream_t s) {
    if (q.num_tiles == 0) return hipSuccess;
    SplitArgs a{};
    a.keys_in = q.keys_in;
    a.keys_out = q.keys_out;
    a.perm_out = q.perm_out;
    a.num_tiles = q.num_tiles;
    a.nbits = 32;
    a.f32 = q.f32;
    a.err = q.err;
    if (q.fuse_pay) a.gpay = q.pay;
    const int64_t* o = q.offsets;
    if (max_len <= 1024) return launch_split_shaped<4, 1024, 0, 1>(a, o, s);
    if (max_len <= 2048) return launch_split_shaped<4, 2048, 0, 1>(a, o, s);
    // up to about one tile per CU the sort is latency-bound: 16 waves halve each wave's
    // columns per pass
    if (max_len <= 4096 && q.num_tiles <= 256) return launch_split_shaped<16, 4096, 0, 1>(a, o, s);
    if (max_len <= 4096) return launch_split_shaped<8, 4096, 0, 1>(a, o, s);
    if (max_len <= 8192) return launch_split_shaped<8, 8192, 0, 1>(a, o, s);
    return launch_split_shaped<16, 16384, 0, 1>(a, o, s);
}

}  // namespace ts
