// Conflict-free routing of a tile of 64-bit items to given destinations inside LDS.
//
// This is the permutation problem of Afshani & Sitchinava (Sec. 1, "Problems of
// interest": an item labelled (i, j) goes to slot j of bank i), solved by
// reducing it to a balanced partition by destination bank class followed by an
// in-bank placement.  Items are 64 bits, so a slot s occupies the bank pair
// 2s mod 64, two slots share banks iff they are congruent modulo 32, and a 64-bit write
// is served 16 lanes at a time: 16 lanes whose destinations are distinct modulo 16 are
// also distinct modulo 32.  The class of a destination is dst mod 16.
//
//  1. Four binary splits, most significant class bit first.  At level L the tile is
//     2^L equal segments; every segment sends the items whose next class bit is 0
//     forward from its front and those whose bit is 1 backward from its back.
//     Because the destinations form a permutation, each half receives exactly
//     half the items, so segment boundaries stay at fixed multiples of the
//     column size, and every column's 64 writes land on 64 cyclically
//     consecutive slots: distinct banks for any phase grouping (the same argument
//     as the partition kernel's split).  Reads are linear.
//  2. After the splits, group g (4m = N/16 consecutive slots) holds exactly the 4m
//     items bound for class g.  Lane l = 16q + g (q = 0 .. 3) takes quarter q of group
//     g: in placement step t it reads item q m + ((t + g + 16 q) mod m) of the group (the
//     32 lanes of a read phase meet residues t + g and t + g + 16 modulo 32, all
//     distinct) and writes it to its destination slot, of class g: the 16 lanes of a
//     64-bit write phase reach 16 distinct classes.
//
// The high word of an item is its key: the destination class (dst mod 16) in bits
// 31..28, dst / 16 in bits 27..18 and a 14-bit source index in bits 13..0.  With the
// class bits on top, all items of a level-L segment share the key's top L bits (the
// segment index), so the class bit split at that level is one unsigned comparison
// against a per-segment threshold.  The tile is padded to the capacity; padding items
// must carry the unused destinations so that every class still receives exactly N/16
// items.
//
// A routing can be recorded (every column's ballot at every level, the zeros before
// each wave at the levels whose segments span waves, and every item's placement slot)
// and replayed for further data that travels the same way: the replayed items need
// no destination field, so two 32-bit payload channels share one 64-bit item, and
// the addresses are the recorded ones, so the replay is as conflict-free.
#pragma once

#include "common.hpp"

namespace ts {

// Split levels of a routing: 16 destination classes.
constexpr int ROUTE_LEVELS = 4;

// Key of an item bound for slot dst (< 16384) with source index src (< 16384).
TS_DEV uint32_t route_key(uint32_t dst, uint32_t src) {
    return ((dst & 15u) << 28) | ((dst >> 4) << 18) | src;
}
TS_DEV uint32_t key_dst(uint32_t key) { return (((key >> 18) & 0x3FFu) << 4) | (key >> 28); }
TS_DEV uint32_t key_src(uint32_t key) { return key & 0x3FFFu; }

template <int NW, int CAP>
struct Router {
    static constexpr int NCOL = CAP / 64;   // columns of the tile
    static constexpr int CPW = NCOL / NW;   // columns per wave
    static constexpr int M = CAP / 64;      // a quarter of the items of a class
    static constexpr int LOG_NCOL = __builtin_ctz(NCOL);
    static_assert(CPW * NW == NCOL, "capacity must split evenly over the waves");
    static_assert(M >= 64, "tiles of at least 64 x 64 items");
    static_assert(CAP <= 16384, "keys hold 14-bit slots and sources");
    static constexpr int KEEP_MAX = 8;      // above this, ballots are recomputed (scalar registers)

    // Record of one routing (lives in LDS next to A).
    struct Plan {
        uint64_t bal[ROUTE_LEVELS][NCOL];   // ballot of every column at every level
        int zb[ROUTE_LEVELS][NW];           // zeros of the segment before each wave's first column
    };

    // One binary split (level L, class bit 3 - L) of every segment.  MODE 0: route;
    // 1: route and record into *plan; 2: replay the split recorded in *plan.
    //
    // Column k (k_in = k mod segment columns) writes a zero to seg_base + z + r0 and a one
    // to seg_end - 1 - (64 k_in - z) - (lane - r0), z the segment's zeros before the
    // column and r0 the zeros in lower lanes; i.e. to seg_base + z + r0 +
    // (one ? 64 (seg_cols - k_in) - 1 - lane : 0), the bracket folded into the rank count.
    template <int L, int MODE>
    static TS_DEV void split_level(uint64_t* A, int* wz, uint64_t (&e)[CPW], int w_in, int lane, Plan* plan) {
        const int w = opaque_s(w_in);              // per-level column constants stay local
        constexpr int seg_cols = NCOL >> L;        // columns per segment
        constexpr bool shared = seg_cols > CPW;    // segment spans several waves
        constexpr bool keep = CPW <= KEEP_MAX;     // zero masks kept between the two loops
        const uint32_t lane8 = opaque((uint32_t)lane * 8u);
        const uint32_t own_base = lane8 + (uint32_t)(w * CPW * 512);  // column j at + 512 j
        auto zero_mask = [&](int j) -> uint64_t {
            if constexpr (MODE == 2) {
                const uint64_t bv = plan->bal[L][w * CPW + j];  // same word for every lane
                // (readfirstlane returns a signed int: widen through uint32_t)
                return ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(hi32(bv)) << 32) |
                       (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(lo32(bv));
            } else {
                // segment index = the key's top L bits; the split bit follows them
                const uint32_t seg = (uint32_t)((w * CPW + j) >> (LOG_NCOL - L));
                const uint32_t thr = (L == 0 ? 0u : (seg << ((32 - L) & 31))) | (1u << (31 - L));
                return ballot(hi32(e[j]) < thr);
            }
        };
        uint64_t zm[keep ? CPW : 1];
        int zb = 0;  // zeros of this segment in columns before this wave's first column
        if constexpr (shared) {
            if constexpr (MODE == 2) {
                zb = (int)__builtin_amdgcn_readfirstlane((uint32_t)plan->zb[L][w]);
                __syncthreads();  // every wave has read the previous level
            } else {
                int zc = 0;
#pragma unroll
                for (int j = 0; j < CPW; ++j) {
                    const uint64_t m = zero_mask(j);
                    if constexpr (keep) zm[j] = m;
                    zc += popc64(m);
                }
                if (lane == 0) wz[w] = zc;
                __syncthreads();  // all waves have read the previous level and posted counts
                // lanes first .. w-1 (the earlier waves of this wave's segment) hold their
                // counts; a prefix sum over the first NW lanes adds them up
                constexpr int wps = seg_cols / CPW;  // waves per segment (a power of two)
                const int first = w & ~(wps - 1);
                const uint32_t mine = (lane >= first && lane < w) ? (uint32_t)wz[lane] : 0u;
                zb = (int)__builtin_amdgcn_readlane((int)row_prefix_sum<NW>(mine), NW - 1);
                if (MODE == 1 && lane == 0) plan->zb[L][w] = zb;
            }
        } else {
            wave_lds_fence();  // the previous level's reads stay before these writes
        }
        int z = zb;
#pragma unroll
        for (int j = 0; j < CPW; ++j) {
            const int k = w * CPW + j;                          // global column
            const int kin = shared ? (k & (seg_cols - 1)) : (j & (seg_cols - 1));
            if (!shared && kin == 0) z = 0;                     // a new wave-local segment
            const uint64_t m = (keep && shared && MODE != 2) ? zm[keep ? j : 0] : zero_mask(j);
            if (MODE == 1 && lane == 0) plan->bal[L][k] = m;
            const uint32_t one_off = zero_if_mask(m, (uint32_t)(64 * (seg_cols - kin) - 1) - (uint32_t)lane);
            const uint32_t pos = count_below_plus(m, one_off) + (uint32_t)(64 * (k - kin) + z);
            lds_store(A, pos * 8u, e[j]);
            z += popc64(m);
        }
        if (shared) __syncthreads();  // the level is complete in every segment
        else wave_lds_fence();
#pragma unroll
        for (int j = 0; j < CPW; ++j) e[j] = lds_load(A, own_base + 512u * j);
    }

    template <int MODE>
    static TS_DEV void split_levels(uint64_t* A, int* wz, uint64_t (&e)[CPW], int w, int lane, Plan* plan) {
        split_level<0, MODE>(A, wz, e, w, lane, plan);
        split_level<1, MODE>(A, wz, e, w, lane, plan);
        split_level<2, MODE>(A, wz, e, w, lane, plan);
        split_level<3, MODE>(A, wz, e, w, lane, plan);
        static_assert(ROUTE_LEVELS == 4, "four class bits");
    }

    // Placement: group g = slots [4Mg, 4M(g+1)) holds the items for class g.  Wave w
    // performs steps t = w*CPW + j; lane l = 16q + g reads item qM + ((t + g + 16q) mod M)
    // of group g and then writes it to its destination (class g).
    static TS_DEV void gather_groups(const uint64_t* A, uint64_t (&e)[CPW], int w, int lane) {
        __syncthreads();  // every wave's groups are complete
        const int lane_o = (int)opaque((uint32_t)lane);
        const uint32_t g = (uint32_t)lane_o & 15u, q = (uint32_t)lane_o >> 4;
        const uint32_t base = g * (4 * M) + q * M;
        const uint32_t rot = g + 16u * q;
#pragma unroll
        for (int j = 0; j < CPW; ++j) {
            const int t = w * CPW + j;
            const uint32_t slot = base + (((uint32_t)t + rot) & (uint32_t)(M - 1));
            e[j] = lds_load(A, slot * 8u);
        }
        __syncthreads();  // all groups read before any slot is overwritten
    }

    // Route e[] (column w*CPW + j of the current order in e[j]) so that on return the
    // LDS array A holds every item at its destination slot.  Contains barriers: every
    // wave of the workgroup must call it.  With RECORD the routing is written to *plan
    // and pdst[j] receives the slot of the item this lane places in step w*CPW + j.
    template <bool RECORD = false>
    static TS_DEV void route(uint64_t* A, int* wz, uint64_t (&e)[CPW], int w, int lane,
                             Plan* plan = nullptr, uint32_t* pdst = nullptr) {
        split_levels<RECORD ? 1 : 0>(A, wz, e, w, lane, plan);
        gather_groups(A, e, w, lane);
#pragma unroll
        for (int j = 0; j < CPW; ++j) {
            const uint32_t dst = key_dst(hi32(e[j]));
            if (RECORD) pdst[j] = dst;
            lds_store(A, dst * 8u, e[j]);
        }
        __syncthreads();  // A holds the tile in destination order
    }

    // Move e[] exactly as the recorded routing moved its items (e[j] in column
    // w*CPW + j of the original order); on return A holds them at their destinations.
    // Contains barriers: every wave of the workgroup must call it.
    static TS_DEV void replay(uint64_t* A, const Plan* plan, uint64_t (&e)[CPW],
                              const uint32_t* pdst, int w, int lane) {
        split_levels<2>(A, nullptr, e, w, lane, const_cast<Plan*>(plan));
        gather_groups(A, e, w, lane);
#pragma unroll
        for (int j = 0; j < CPW; ++j) lds_store(A, pdst[j] * 8u, e[j]);
        __syncthreads();
    }
};

}  // namespace ts
