// Device helpers shared by the tile kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

#define TS_DEV __device__ __forceinline__

namespace ts {

constexpr int WAVE = 64;

TS_DEV int lane_id() {
    return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

TS_DEV uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Number of set bits of `mask` in lanes below the calling lane.
TS_DEV uint32_t count_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Same, plus an addend (folded into the mbcnt accumulator).
TS_DEV uint32_t count_below_plus(uint64_t mask, uint32_t add) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, add));
}

TS_DEV int popc64(uint64_t m) { return __popcll(m); }

// Make the compiler treat v as changed here, so values derived from it are computed
// inside the enclosing loop instead of being hoisted and kept live in registers.
TS_DEV uint32_t opaque(uint32_t v) {
    asm volatile("" : "+v"(v));
    return v;
}

// The same for a wave-uniform value (kept in a scalar register): values derived from
// it are recomputed with scalar instructions where they are used instead of being
// hoisted, which can run out of scalar registers and spill them to vector lanes.
TS_DEV int opaque_s(int v) {
    asm volatile("" : "+s"(v));
    return v;
}
TS_DEV int64_t opaque_s64(int64_t v) {
    asm volatile("" : "+s"(v));
    return v;
}

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on XCD b % 8),
// each with its own L2.  For a grid of g workgroups with one tile each, this gives XCD
// x one contiguous range of tiles, taken in order: tiles that write neighbouring parts
// of one cache line then run on the same XCD at about the same time.  A bijection of
// [0, g): XCD x holds g/8 (+1 if x < g%8) workgroups and its range starts at
// x*(g/8) + min(x, g%8).
TS_DEV int64_t xcd_contiguous(int64_t b, int64_t g) {
    const int64_t x = b & 7, i = b >> 3, q = g >> 3, r = g & 7;
    return x * q + (x < r ? x : r) + i;
}

// Cross-lane exchange through LDS inside one wavefront.  The LDS executes a
// wavefront's instructions in order, so no hardware wait is needed; what must be
// stopped is the compiler moving loads and stores across this point: it reasons per
// lane, and where it can prove a lane's own later read disjoint from its earlier
// writes (a fixed transpose, say) it may hoist the read above writes by other lanes.
TS_DEV void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-lane select driven by a wave mask (e.g. a ballot): lane bit set -> if1, else if0.
// One v_cndmask with the mask as its SGPR-pair condition.
TS_DEV uint32_t select_by_mask(uint64_t mask, uint32_t if0, uint32_t if1) {
    uint32_t r;
    asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(if0), "v"(if1), "s"(mask));
    return r;
}

// Lane bit of `mask` set -> 0, else if0 (one v_cndmask with an inline-constant operand).
TS_DEV uint32_t zero_if_mask(uint64_t mask, uint32_t if0) {
    uint32_t r;
    asm("v_cndmask_b32_e64 %0, %1, 0, %2" : "=v"(r) : "v"(if0), "s"(mask));
    return r;
}

// Sum of v over lanes 0 .. L-1 (L a power of two, at most 16), valid in lane L-1:
// an inclusive prefix sum inside the first DPP row.
template <int L, int S = 1>
TS_DEV uint32_t row_prefix_sum(uint32_t v) {
    static_assert(L >= 1 && L <= 16 && (L & (L - 1)) == 0, "one DPP row, power of two");
    if constexpr (S < L) {
        v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x110 | S, 0xF, 0xF, true);  // row_shr:S
        return row_prefix_sum<L, 2 * S>(v);
    } else {
        return v;
    }
}

// Inclusive prefix sum across the 64 lanes of a wavefront (all lanes active), in DPP:
// a prefix sum inside each row of 16 lanes, then lane 15 of rows 0 and 2 is added to
// rows 1 and 3 (row_bcast:15) and lane 31 to rows 2 and 3 (row_bcast:31).  Rows left
// out by the row mask read 0 (`old`), so they add nothing.
TS_DEV uint32_t wave_inclusive_scan_u32(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false); // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false); // row_bcast:31
    return v;
}

// Issue CPW coalesced 32-bit global loads of one tile, column j = items 64*(c0+j) + lane,
// with no waits between them and no branches around them.  Element g of the tile is at
// base[(o + g) * stride].  Lanes past the end (and every lane when n <= 0) read from
// `fallback` -- any always-readable address -- and the caller ignores those values.
// Unit stride uses a wave-uniform tile pointer and 32-bit byte offsets (scalar-base
// addressing); other strides use 64-bit addresses.
// NT: streaming (nontemporal) loads, for data read exactly once.
template <int CPW, bool NT = false, typename T>
TS_DEV void load_columns(const T* __restrict__ base, int64_t stride, int64_t o, int n, int c0,
                         int lane, T (&out)[CPW], const void* fallback) {
    const bool any = n > 0;
    const uint32_t nn = any ? (uint32_t)n : 0u;  // a negative n loads nothing
    if (stride == 1) {
        const char* tb = any ? (const char*)(base + o) : (const char*)fallback;
#pragma unroll
        for (int j = 0; j < CPW; ++j) {
            const uint32_t i = (uint32_t)(64 * (c0 + j) + lane);
            const uint32_t off = (i < nn) ? i * (uint32_t)sizeof(T) : 0u;
            const T* p = (const T*)(tb + off);
            out[j] = NT ? __builtin_nontemporal_load(p) : *p;
        }
    } else {
#pragma unroll
        for (int j = 0; j < CPW; ++j) {
            const int i = 64 * (c0 + j) + lane;
            const T* p = (i < n) ? base + (o + i) * stride : (const T*)fallback;
            out[j] = NT ? __builtin_nontemporal_load(p) : *p;
        }
    }
}

// Buffer resource over `bytes` bytes from `base` (raw addressing, 4-byte granules):
// loads at offsets past the end return 0 and stores there are dropped by the
// hardware range check, so the edge of a tile needs no per-lane masks or fallback
// addresses.  Every access below takes a byte offset; column j of a wave is the
// per-lane offset plus an immediate.
typedef __amdgpu_buffer_rsrc_t rsrc_t;

TS_DEV rsrc_t buffer_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

// CPW columns of 32-bit words: out[j] = word at byte lane_off + 256 j (0 past the end).
template <int CPW, bool NT = false>
TS_DEV void buffer_load_columns(rsrc_t r, uint32_t lane_off, uint32_t (&out)[CPW]) {
#pragma unroll
    for (int j = 0; j < CPW; ++j)
        out[j] = __builtin_amdgcn_raw_buffer_load_b32(r, (int)(lane_off + 256u * j), 0, NT ? 2 : 0);
}

// The same with a run-time column stride in bytes (elements `stride` words apart).
template <int CPW, bool NT = false>
TS_DEV void buffer_load_columns_strided(rsrc_t r, uint32_t lane_off, uint32_t col_bytes, uint32_t (&out)[CPW]) {
#pragma unroll
    for (int j = 0; j < CPW; ++j)
        out[j] = __builtin_amdgcn_raw_buffer_load_b32(r, (int)(lane_off + col_bytes * j), 0, NT ? 2 : 0);
}

// CPW columns of 16-bit values: out[j] = value at byte lane_off + 128 j (0 past the end).
template <int CPW, bool NT = false>
TS_DEV void buffer_load_columns16(rsrc_t r, uint32_t lane_off, uint32_t (&out)[CPW]) {
#pragma unroll
    for (int j = 0; j < CPW; ++j)
        out[j] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, (int)(lane_off + 128u * j), 0, NT ? 2 : 0);
}

template <bool NT = false>
TS_DEV void buffer_store(rsrc_t r, uint32_t byte_off, uint32_t v) {
    __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)byte_off, 0, NT ? 2 : 0);
}

template <bool NT = false>
TS_DEV void buffer_store16(rsrc_t r, uint32_t byte_off, uint32_t v) {
    __builtin_amdgcn_raw_buffer_store_b16((unsigned short)v, r, (int)byte_off, 0, NT ? 2 : 0);
}

// Store element g = 64*c + lane of a tile (g < n) at base[(o + g) * stride]; NT: a
// streaming (nontemporal) store.
template <bool NT = false, typename T>
TS_DEV void store_item(T* __restrict__ base, int64_t stride, int64_t o, int g, T v) {
    T* p = (stride == 1) ? (T*)((char*)(base + o) + (uint32_t)g * (uint32_t)sizeof(T)) : base + (o + g) * stride;
    if (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// LDS accesses at a byte offset from the start of an LDS array.
template <typename T>
TS_DEV T lds_load(const T* base, uint32_t byte_off) {
    return *(const T*)((const char*)base + byte_off);
}
template <typename T>
TS_DEV void lds_store(T* base, uint32_t byte_off, T v) {
    *(T*)((char*)base + byte_off) = v;
}

// A 64-bit LDS load kept whole.  When only one half of a loaded 64-bit slot is used,
// the compiler narrows the load to 32 bits at a two-word stride, which puts lanes L
// and L+16 of a 32-lane phase on one bank; this keeps the conflict-free 64-bit access.
template <typename T>
TS_DEV uint64_t lds_load_u64_whole(const T* base, uint32_t byte_off) {
    uint64_t v = *(const uint64_t*)((const char*)base + byte_off);
    asm volatile("" : "+v"(v));
    return v;
}

// CPW 64-bit LDS loads issued back to back, then kept whole (see lds_load_u64_whole)
// all together, so their latencies overlap.
template <int CPW, typename T>
TS_DEV void lds_load_columns_whole(const T* base, uint32_t byte_off, uint32_t col_bytes, uint64_t (&out)[CPW]) {
#pragma unroll
    for (int j = 0; j < CPW; ++j) out[j] = *(const uint64_t*)((const char*)base + byte_off + col_bytes * j);
#pragma unroll
    for (int j = 0; j < CPW; ++j) asm volatile("" : "+v"(out[j]));
}

TS_DEV uint32_t hi32(uint64_t x) { return (uint32_t)(x >> 32); }
TS_DEV uint32_t lo32(uint64_t x) { return (uint32_t)x; }
TS_DEV uint64_t pack(uint32_t hi, uint32_t lo) { return ((uint64_t)hi << 32) | lo; }

// Order-preserving map of binary32 bit patterns to uint32 (and back).
TS_DEV uint32_t f32_to_ordered(uint32_t b) {
    uint32_t flip = (uint32_t)((int32_t)b >> 31) | 0x80000000u;
    return b ^ flip;
}
TS_DEV uint32_t ordered_to_f32(uint32_t u) {
    uint32_t flip = ((u >> 31) - 1u) | 0x80000000u;
    return u ^ flip;
}

// Record an error bit once per wave.
TS_DEV void flag_error(uint32_t* err, bool bad, uint32_t bit) {
    uint64_t any = ballot(bad);
    if (any != 0 && lane_id() == (int)(__builtin_ctzll(any))) atomicOr(err, bit);
}

}  // namespace ts
