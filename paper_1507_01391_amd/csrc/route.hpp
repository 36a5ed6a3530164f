// Conflict-free routing of a tile of 64-bit items to given destinations inside LDS.
//
// This is the permutation problem of Afshani & Sitchinava (Sec. 1, "Problems of
// interest": an item labelled (i, j) goes to slot j of bank i), solved by
// reducing it to a balanced w-way partition by destination bank followed by an
// in-bank placement:
//
//  1. Six binary splits, most significant bank bit first.  At level L the tile is
//     2^L equal segments; every segment sends the items whose next bank bit is 0
//     forward from its front and those whose bit is 1 backward from its back.
//     Because the destinations form a permutation, each half receives exactly
//     half the items, so segment boundaries stay at fixed multiples of the
//     column size, and every column's 64 writes land on 64 cyclically
//     consecutive slots: one per bank, for any phase grouping (the same
//     argument as the partition kernel's split).  Reads are linear.
//  2. After the splits, group g (m = N/64 consecutive slots) holds exactly the m
//     items bound for bank g.  In placement step t lane l reads item
//     (t + l) mod m of group l (a skewed, conflict-free read) and writes it to
//     its destination slot, which lies in bank l: every lane writes its own bank.
//
// Items carry the destination in the low 16 bits of their high word.  The tile
// is padded to the capacity; padding items must carry the unused destinations
// so that every bank still receives exactly N/64 items.
//
// A routing can be recorded (every column's ballot at every level, the zeros before
// each wave at the levels whose segments span waves, and every item's placement slot)
// and replayed for further data that travels the same way: the replayed items need
// no destination field, so two 32-bit payload channels share one 64-bit item, and
// the addresses are the recorded ones, so the replay is as conflict-free.
#pragma once

#include "common.hpp"

namespace ts {

template <int NW, int CAP>
struct Router {
    static constexpr int NCOL = CAP / 64;   // columns of the tile
    static constexpr int CPW = NCOL / NW;   // columns per wave
    static constexpr int M = CAP / 64;      // items per bank
    static_assert(CPW * NW == NCOL, "capacity must split evenly over the waves");
    static_assert(M >= 64, "tiles of at least 64 x 64 items");

    // Record of one routing (lives in LDS next to A).
    struct Plan {
        uint64_t bal[6][NCOL];   // ballot of every column at every level
        int zb[6][NW];           // zeros of the segment before each wave's first column
    };

    // Route e[] (column w*CPW + j of the current order in e[j]) so that on return the
    // LDS array A holds every item at its destination slot.  Contains barriers: every
    // wave of the workgroup must call it.  With RECORD the routing is written to *plan
    // and pdst[j] receives the slot of the item this lane places in step w*CPW + j.
    template <bool RECORD = false>
    static TS_DEV void route(uint64_t* A, int* wz, uint64_t (&e)[CPW], int w, int lane,
                             Plan* plan = nullptr, uint32_t* pdst = nullptr) {
#pragma unroll 1
        for (int L = 0; L < 6; ++L) {
            const uint32_t lane8 = opaque((uint32_t)lane * 8u);
            const uint32_t neg_lane8 = 0u - lane8;
            const uint32_t own_base = lane8 + (uint32_t)(w * CPW * 512);  // column j at + 512 j
            const int bit = 5 - L;                 // bank bit split at this level
            const int seg_cols = NCOL >> L;        // columns per segment
            const bool shared = seg_cols > CPW;    // segment spans several waves
            int zb = 0;  // zeros of this segment in columns before this wave's first column
            if (shared) {
                int zc = 0;
#pragma unroll
                for (int j = 0; j < CPW; ++j) zc += 64 - popc64(ballot((hi32(e[j]) >> bit) & 1u));
                if (lane == 0) wz[w] = zc;
                __syncthreads();  // all waves have read the previous level and posted counts
                const int waves_per_seg = seg_cols / CPW;
                const int first = (w / waves_per_seg) * waves_per_seg;
                const int mine = (lane < NW) ? wz[lane] : 0;
#pragma unroll
                for (int q = 0; q < NW; ++q) {
                    const int v = __builtin_amdgcn_readlane(mine, q);
                    zb += (q >= first && q < w) ? v : 0;
                }
                if (RECORD && lane == 0) plan->zb[L][w] = zb;
            }
            if (!shared) wave_lds_fence();  // the previous level's reads stay before these writes
            int z = zb;
#pragma unroll
            for (int j = 0; j < CPW; ++j) {
                const int k = w * CPW + j;         // global column
                const int kin = k % seg_cols;      // column inside its segment
                if (!shared && kin == 0) z = 0;    // a new wave-local segment starts
                const int seg_base = k - kin;      // first column of the segment
                // ballot recomputed here rather than kept from the count loop (registers)
                const uint64_t bal = ballot((hi32(e[j]) >> bit) & 1u);
                if (RECORD && lane == 0) plan->bal[L][k] = bal;
                const uint32_t r0 = count_below(~bal);
                // zero: seg_base*64 + z + rank0; one: seg_end - 1 - (64 kin - z) - (lane - rank0)
                const uint32_t z8 = (uint32_t)__builtin_amdgcn_readfirstlane((seg_base * 64 + z) * 8);
                const uint32_t d8 = (uint32_t)__builtin_amdgcn_readfirstlane((seg_cols * 64 - 1 - 64 * kin) * 8);
                const uint32_t a0 = r0 * 8u + z8;
                const uint32_t a1 = a0 + neg_lane8 + d8;
                lds_store(A, select_by_mask(bal, a0, a1), e[j]);
                z += 64 - popc64(bal);
            }
            if (shared) __syncthreads();  // the level is complete in every segment
            else wave_lds_fence();
#pragma unroll
            for (int j = 0; j < CPW; ++j) e[j] = lds_load(A, own_base + 512u * j);
        }
        // ---- placement: group g = slots [g*M, (g+1)*M) holds the items for bank g.
        //      Wave w performs steps t = w*CPW + j; lane l reads item (t + l) mod M of
        //      group l and later writes it to its destination (bank l).
        __syncthreads();  // every wave's groups are complete
        const int lane_o = (int)opaque((uint32_t)lane);
#pragma unroll
        for (int j = 0; j < CPW; ++j) {
            const int t = w * CPW + j;
            const uint32_t slot = (uint32_t)lane_o * M + (uint32_t)((t + lane_o) & (M - 1));
            e[j] = lds_load(A, slot * 8u);
        }
        __syncthreads();  // all groups read before any slot is overwritten
#pragma unroll
        for (int j = 0; j < CPW; ++j) {
            const uint32_t dst = hi32(e[j]) & (uint32_t)(CAP - 1);
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
#pragma unroll 1
        for (int L = 0; L < 6; ++L) {
            const uint32_t lane8 = opaque((uint32_t)lane * 8u);
            const uint32_t neg_lane8 = 0u - lane8;
            const uint32_t own_base = lane8 + (uint32_t)(w * CPW * 512);
            const int seg_cols = NCOL >> L;
            const bool shared = seg_cols > CPW;
            int zb = 0;
            if (shared) {
                zb = (int)__builtin_amdgcn_readfirstlane((uint32_t)plan->zb[L][w]);
                __syncthreads();  // every wave has read the previous level
            } else {
                wave_lds_fence();
            }
            int z = zb;
#pragma unroll
            for (int j = 0; j < CPW; ++j) {
                const int k = w * CPW + j;
                const int kin = k % seg_cols;
                if (!shared && kin == 0) z = 0;
                const int seg_base = k - kin;
                const uint64_t bv = plan->bal[L][k];  // same word for every lane
                // (readfirstlane returns a signed int: widen through uint32_t)
                const uint64_t bal = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(hi32(bv)) << 32) |
                                     (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(lo32(bv));
                const uint32_t r0 = count_below(~bal);
                const uint32_t z8 = (uint32_t)__builtin_amdgcn_readfirstlane((seg_base * 64 + z) * 8);
                const uint32_t d8 = (uint32_t)__builtin_amdgcn_readfirstlane((seg_cols * 64 - 1 - 64 * kin) * 8);
                const uint32_t a0 = r0 * 8u + z8;
                const uint32_t a1 = a0 + neg_lane8 + d8;
                lds_store(A, select_by_mask(bal, a0, a1), e[j]);
                z += 64 - popc64(bal);
            }
            if (shared) __syncthreads();
            else wave_lds_fence();
#pragma unroll
            for (int j = 0; j < CPW; ++j) e[j] = lds_load(A, own_base + 512u * j);
        }
        __syncthreads();
        const int lane_o = (int)opaque((uint32_t)lane);
#pragma unroll
        for (int j = 0; j < CPW; ++j) {
            const int t = w * CPW + j;
            const uint32_t slot = (uint32_t)lane_o * M + (uint32_t)((t + lane_o) & (M - 1));
            e[j] = lds_load(A, slot * 8u);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < CPW; ++j) lds_store(A, pdst[j] * 8u, e[j]);
        __syncthreads();
    }
};

}  // namespace ts
