// Tile-local permutation without LDS bank conflicts (Afshani & Sitchinava, Sec. 1,
// "Problems of interest", permutation).  The routing itself is in route.hpp.
//
//   SCATTER  out[pi[i]] = in[i]: item (in[i], destination pi[i]) is routed once.
//   GATHER   out[i] = in[pi[i]]: first the index i is routed to slot pi[i], which
//            leaves inv[q] (the output slot that wants in[q]) at every slot q; then
//            (in[q], destination inv[q]) is routed.  The first routing is shared by
//            all payload channels.
// Item keys carry the source index beside the destination (route_key), so either
// direction can also write the inverse permutation at no extra routing: a scatter's
// caller can then undo it with another scatter instead of a two-routing gather.
#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"
#include "route.hpp"

namespace ts {

namespace {

// REPLAY (for two or more channels): the first channel is routed and recorded, the
// other channels replay the record two per 64-bit item.  The channels are the optional
// aux channel (first) and the payload channels.
//
// Global accesses go through buffer resources over the tile (pi, inv_out, and each
// payload channel when its elements are contiguous): lanes past the end of the tile
// read 0 and their stores are dropped by the hardware range check, so no per-lane
// bounds test or address select is spent on them.
template <int NW, int CAP, bool GATHER, int WPE, bool REPLAY, bool NT>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(WPE > 0 ? WPE : 1)))
void permute_split_kernel(PermuteArgs a, const int64_t* __restrict__ offs) {
    using R = Router<NW, CAP>;
    constexpr int CPW = R::CPW;
    __shared__ uint64_t A[CAP];
    __shared__ int wz[NW];
    __shared__ typename std::conditional<REPLAY, typename R::Plan, int>::type plan;
    const int lane0 = lane_id();
    const int w0 = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    constexpr bool gather = GATHER;
    const uint32_t has_aux = a.aux.in != nullptr ? 1u : 0u;
    const uint32_t nch = a.pay.channels + has_aux;  // channels to move
    const bool with_pay = nch > 0;

    for (int64_t t = blockIdx.x; t < a.num_tiles; t += gridDim.x) {
        // lane- and wave-derived values are recomputed per tile instead of being hoisted
        // out of the tile loop (and spilled)
        const int lane = (int)opaque((uint32_t)lane0);
        const int w = opaque_s(w0);
        const int64_t o = offs[t];
        const int64_t len = offs[t + 1] - o;
        if (len > CAP) {
            if (threadIdx.x == 0) atomicOr(a.err, ERR_TILE_TOO_LONG);
            continue;
        }
        const int n = (int)len;
        const uint32_t nb = (uint32_t)(n > 0 ? n : 0);
        // byte offset of item 64 (w*CPW) + lane in 32-bit and 16-bit arrays; column j
        // adds 256 j / 128 j
        const uint32_t off32 = ((uint32_t)(64 * w * CPW) + (uint32_t)lane) * 4u;
        const uint32_t off16 = off32 >> 1;
        const rsrc_t rpi = a.pi16 ? buffer_rsrc((const uint16_t*)a.pi + o, nb * 2u)
                                  : buffer_rsrc(a.pi + o, nb * 4u);
        // resources of the outputs are built where they are used (from opaque copies of
        // the tile offset), not kept in scalar registers across the routing
        // channel c (the aux channel first, when there is one, then the payload
        // channels): words (o + g) * es + c' * cs; a buffer over the tile's n * es words
        // (the host keeps that below 2^32 bytes).  The aux channel has unit stride.
        auto chan_es = [&](uint32_t c) { return (has_aux && c == 0) ? 1u : (uint32_t)a.pay.es; };
        auto pay_rsrc = [&](bool out, uint32_t c) {
            const int64_t oo = opaque_s64(o);
            if (has_aux && c == 0) return buffer_rsrc((out ? a.aux.out : a.aux.in) + oo, nb * 4u);
            const uint32_t* base = out ? a.pay.out : a.pay.in;
            const uint32_t es = (uint32_t)a.pay.es;
            return buffer_rsrc(base + (int64_t)(c - has_aux) * a.pay.cs + oo * (int64_t)es, nb * es * 4u);
        };
        // lane offsets are passed in from an opaque copy of the lane taken where the
        // access happens, so the compiler neither keeps per-column offsets live across a
        // routing nor shares them with values computed before it
        auto load_pay = [&](uint32_t c, uint32_t lane_off, uint32_t (&xv)[CPW]) {
            const rsrc_t r = pay_rsrc(false, c);
            const uint32_t es = chan_es(c);
            if (es == 1) buffer_load_columns<CPW, NT>(r, lane_off, xv);
            else buffer_load_columns_strided<CPW, NT>(r, lane_off * es, 256u * es, xv);
        };
        // stores of whole columns, one uniform branch per call: lo32 (hi = false) or
        // hi32 (hi = true) of x[j] to channel c; index values v[j] to inv_out
        auto store_pay = [&](uint32_t c, uint32_t lane_off, const uint64_t (&x)[CPW], bool hi) {
            const rsrc_t r = pay_rsrc(true, c);
            const uint32_t es = chan_es(c);
            if (es == 1) {
#pragma unroll
                for (int j = 0; j < CPW; ++j) buffer_store<NT>(r, lane_off + 256u * j, hi ? hi32(x[j]) : lo32(x[j]));
            } else {
#pragma unroll
                for (int j = 0; j < CPW; ++j)
                    buffer_store<NT>(r, lane_off * es + 256u * es * j, hi ? hi32(x[j]) : lo32(x[j]));
            }
        };
        auto store_inv_cols = [&](uint32_t lane_off, const uint32_t (&v)[CPW]) {
            const int64_t oo = opaque_s64(o);
            if (a.inv16) {
                const rsrc_t r = buffer_rsrc((uint16_t*)a.inv_out + oo, nb * 2u);
#pragma unroll
                for (int j = 0; j < CPW; ++j) buffer_store16<NT>(r, (lane_off >> 1) + 128u * j, v[j]);
            } else {
                const rsrc_t r = buffer_rsrc(a.inv_out + oo, nb * 4u);
#pragma unroll
                for (int j = 0; j < CPW; ++j) buffer_store<NT>(r, lane_off + 256u * j, v[j]);
            }
        };
        auto lane_off_at = [&](int l) { return ((uint32_t)(64 * w * CPW) + (uint32_t)l) * 4u; };

        // ---- destinations: item i (column k, lane l; i = 64k + l) goes to pi[i];
        //      padding items i >= n keep their own index, so the destinations always
        //      form a permutation of [0, CAP).
        uint32_t dst[CPW];
        {
            uint32_t piv[CPW];
            if (a.pi16) buffer_load_columns16<CPW, NT>(rpi, off16, piv);
            else buffer_load_columns<CPW, NT>(rpi, off32, piv);
#pragma unroll
            for (int j = 0; j < CPW; ++j) {
                const int i = 64 * (w * CPW + j) + lane;
                dst[j] = (i < n) ? (piv[j] & (uint32_t)(CAP - 1)) : (uint32_t)i;
            }
            if (a.validate) {  // one branch for the whole check
                bool bad = false;
#pragma unroll
                for (int j = 0; j < CPW; ++j)
                    bad |= (64 * (w * CPW + j) + lane < n) && (piv[j] >= (uint32_t)n);  // also catches q < 0
                flag_error(a.err, bad, ERR_BAD_PERM);
            }
        }

        uint64_t e[CPW];
        if (gather) {
            // route the request index i to slot pi[i]: slot q then holds inv[q]
#pragma unroll
            for (int j = 0; j < CPW; ++j) {
                const int i = 64 * (w * CPW + j) + lane;
                e[j] = pack(route_key(dst[j], 0u), (uint32_t)i);
            }
            R::route(A, wz, e, w, lane);
            const int lg = (int)opaque((uint32_t)lane);
            lds_load_columns_whole<CPW>(A, (uint32_t)lg * 8u + (uint32_t)(w * CPW * 512), 512u, e);
            if (a.validate) {
                bool bad = false;
#pragma unroll
                for (int j = 0; j < CPW; ++j) bad |= key_dst(hi32(e[j])) != (uint32_t)(64 * (w * CPW + j) + lg);
                flag_error(a.err, bad, ERR_BAD_PERM);
            }
#pragma unroll
            for (int j = 0; j < CPW; ++j) dst[j] = lo32(e[j]);  // inv[q] for q = 64k + l
            if (a.inv_out) store_inv_cols(lane_off_at(lg), dst);
#pragma unroll
            for (int j = 0; j < CPW; ++j) dst[j] = route_key(dst[j], 0u);
            __syncthreads();  // A is reused by the next routing
        } else {
            // the source index rides in the key (for inv_out)
#pragma unroll
            for (int j = 0; j < CPW; ++j) dst[j] = route_key(dst[j], (uint32_t)(64 * (w * CPW + j) + lane));
        }

        // a scatter asked only for the inverse still routes once (with no payload);
        // with REPLAY only channel 0 is routed here
        const uint32_t nroute = REPLAY ? 1u : ((!gather && a.inv_out && nch == 0) ? 1u : nch);
        uint32_t pdst[REPLAY ? CPW : 1];
#pragma unroll 1
        for (uint32_t c = 0; c < nroute; ++c) {
            const int lc = (int)opaque((uint32_t)lane);
            uint32_t xv[CPW];
            if (with_pay) load_pay(c, lane_off_at(lc), xv);
            else
#pragma unroll
                for (int j = 0; j < CPW; ++j) xv[j] = 0u;
#pragma unroll
            for (int j = 0; j < CPW; ++j) e[j] = pack(dst[j], xv[j]);
            if constexpr (REPLAY) R::template route<true>(A, wz, e, w, lane, &plan, pdst);
            else R::route(A, wz, e, w, lane);
            const int ls = (int)opaque((uint32_t)lane);
            lds_load_columns_whole<CPW>(A, (uint32_t)ls * 8u + (uint32_t)(w * CPW * 512), 512u, e);
            if (a.validate && c == 0 && !gather) {
                bool bad = false;
#pragma unroll
                for (int j = 0; j < CPW; ++j) bad |= key_dst(hi32(e[j])) != (uint32_t)(64 * (w * CPW + j) + ls);
                flag_error(a.err, bad, ERR_BAD_PERM);
            }
            if (with_pay) store_pay(c, lane_off_at(ls), e, false);
            if (!gather && c == 0 && a.inv_out) {
                uint32_t src[CPW];
#pragma unroll
                for (int j = 0; j < CPW; ++j) src[j] = key_src(hi32(e[j]));
                store_inv_cols(lane_off_at(ls), src);
            }
            __syncthreads();  // A is reused by the next channel / tile
        }
        if constexpr (REPLAY) {
#pragma unroll 1
            for (uint32_t c = 1; c < nch; c += 2) {
                const int lc = (int)opaque((uint32_t)lane);
                const bool two = c + 1 < nch;
                uint32_t x0[CPW], x1[CPW];
                load_pay(c, lane_off_at(lc), x0);
                load_pay(two ? c + 1 : c, lane_off_at(lc), x1);
#pragma unroll
                for (int j = 0; j < CPW; ++j) e[j] = pack(x1[j], x0[j]);
                R::replay(A, &plan, e, pdst, w, lane);
                const int ls = (int)opaque((uint32_t)lane);
                lds_load_columns_whole<CPW>(A, (uint32_t)ls * 8u + (uint32_t)(w * CPW * 512), 512u, e);
                store_pay(c, lane_off_at(ls), e, false);
                if (two) store_pay(c + 1, lane_off_at(ls), e, true);
                __syncthreads();  // A is reused by the next pair / tile
            }
        }
    }
}

// ONESHOT: one workgroup per tile instead of a persistent grid; NT: streaming global
// loads and stores (every word is read or written once).
template <int NW, int CAP, int WPE = 0, bool ONESHOT = false, bool NT = false>
hipError_t launch_perm(const PermuteArgs& a, hipStream_t s) {
    const bool replay = a.pay.channels + (a.aux.in != nullptr ? 1u : 0u) >= 2;
    auto kern = (a.direction == 1)
                    ? (replay ? permute_split_kernel<NW, CAP, true, WPE, true, NT>
                              : permute_split_kernel<NW, CAP, true, WPE, false, NT>)
                    : (replay ? permute_split_kernel<NW, CAP, false, WPE, true, NT>
                              : permute_split_kernel<NW, CAP, false, WPE, false, NT>);
    const int grid = ONESHOT ? (int)std::min<int64_t>(a.num_tiles, INT32_MAX)
                             : persistent_grid((const void*)kern, NW * 64, 0, a.num_tiles);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NW * 64), 0, s, a, a.offsets);
    return hipGetLastError();
}

template <int NW, int CAP, int WPE = 0>
hipError_t launch_perm_shaped(const PermuteArgs& a, hipStream_t s) {
    return tile_oneshot() ? launch_perm<NW, CAP, WPE, true, true>(a, s) : launch_perm<NW, CAP, WPE>(a, s);
}

}  // namespace

int64_t permute_split_capacity() { return 16384; }

// Kernel variant for 8192-item tiles (tuning knob "permute_variant").  Persistent grids:
// 0 = 16 waves, registers as the compiler likes; 1 = 16 waves capped at 64 registers
// (two workgroups per CU); 2 = 8 waves.  One workgroup per tile, 16 waves capped at 64
// registers: 6 = streaming loads and stores (default), 7 = plain accesses; 8 = the
// persistent form of 6; 9 = one workgroup of 8 waves per tile, streaming accesses; 10 =
// 4 waves (32 columns each) and 11 = 8 waves with registers for three per SIMD, likewise;
// 12 = 8 waves with registers for two per SIMD and 13 = 8 waves with no register cap.
static int g_perm_variant = 6;
void set_permute_variant(int v) { g_perm_variant = v; }

hipError_t launch_permute_split(const PermuteArgs& a, int64_t max_len, hipStream_t s) {
    if (a.num_tiles == 0) return hipSuccess;
    if (max_len <= 4096) return g_perm_variant == 1 ? launch_perm_shaped<8, 4096, 6>(a, s) : launch_perm_shaped<8, 4096>(a, s);
    if (max_len <= 8192) {
        if (g_perm_variant == 1) return launch_perm<16, 8192, 8>(a, s);
        if (g_perm_variant == 2) return launch_perm<8, 8192>(a, s);
        if (g_perm_variant == 6) return launch_perm<16, 8192, 8, true, true>(a, s);
        if (g_perm_variant == 7) return launch_perm<16, 8192, 8, true, false>(a, s);
        if (g_perm_variant == 8) return launch_perm<16, 8192, 8, false, true>(a, s);
        if (g_perm_variant == 9) return launch_perm<8, 8192, 4, true, true>(a, s);
        if (g_perm_variant == 10) return launch_perm<4, 8192, 2, true, true>(a, s);
        if (g_perm_variant == 11) return launch_perm<8, 8192, 3, true, true>(a, s);
        if (g_perm_variant == 12) return launch_perm<8, 8192, 2, true, true>(a, s);
        if (g_perm_variant == 13) return launch_perm<8, 8192, 0, true, true>(a, s);
        return launch_perm<16, 8192>(a, s);
    }
    return launch_perm_shaped<16, 16384>(a, s);
}

}  // namespace ts
