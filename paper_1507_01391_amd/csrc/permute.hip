// Tile-local permutation without LDS bank conflicts (Afshani & Sitchinava, Sec. 1,
// "Problems of interest", permutation).  The routing itself is in route.hpp.
//
//   SCATTER  out[pi[i]] = in[i]: item (in[i], destination pi[i]) is routed once.
//   GATHER   out[i] = in[pi[i]]: first the index i is routed to slot pi[i], which
//            leaves inv[q] (the output slot that wants in[q]) at every slot q; then
//            (in[q], destination inv[q]) is routed.  The first routing is shared by
//            all payload channels.
// Items carry the source index beside the destination (destination in the low 16
// bits of the high word, source in the high 16), so either direction can also write
// the inverse permutation at no extra routing: a scatter's caller can then undo it
// with another scatter instead of a two-routing gather.
#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"
#include "route.hpp"

namespace ts {

namespace {

// REPLAY (for two or more payload channels): channel 0 is routed and recorded, the
// other channels replay the record two per 64-bit item.
template <int NW, int CAP, bool GATHER, int WPE, bool REPLAY, bool NT>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(WPE > 0 ? WPE : 1)))
void permute_split_kernel(PermuteArgs a, const int64_t* __restrict__ offs) {
    using R = Router<NW, CAP>;
    constexpr int CPW = R::CPW;
    __shared__ uint64_t A[CAP];
    __shared__ int wz[NW];
    __shared__ typename std::conditional<REPLAY, typename R::Plan, int>::type plan;
    const int lane0 = lane_id();
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    constexpr bool gather = GATHER;

    for (int64_t t = blockIdx.x; t < a.num_tiles; t += gridDim.x) {
        const int lane = (int)opaque((uint32_t)lane0);
        const uint32_t own_base = (uint32_t)lane * 8u + (uint32_t)(w * CPW * 512);
        const int64_t o = offs[t];
        const int64_t len = offs[t + 1] - o;
        if (len > CAP) {
            if (threadIdx.x == 0) atomicOr(a.err, ERR_TILE_TOO_LONG);
            continue;
        }
        const int n = (int)len;

        // ---- destinations: item i (column k, lane l; i = 64k + l) goes to pi[i];
        //      padding items i >= n keep their own index, so the destinations always
        //      form a permutation of [0, CAP).
        uint32_t dst[CPW];
        bool bad = false;
        int32_t piv[CPW];
        load_columns<CPW, NT>(a.pi, 1, o, n, w * CPW, lane, piv, offs);
#pragma unroll
        for (int j = 0; j < CPW; ++j) {
            const int i = 64 * (w * CPW + j) + lane;
            const int32_t q = piv[j];
            bad |= (i < n) && (q < 0 || q >= n);
            dst[j] = (i < n) ? ((uint32_t)q & (uint32_t)(CAP - 1)) : (uint32_t)i;
        }
        if (a.validate) flag_error(a.err, bad, ERR_BAD_PERM);

        uint64_t e[CPW];
        if (gather) {
            // route the request index i to slot pi[i]: slot q then holds inv[q]
#pragma unroll
            for (int j = 0; j < CPW; ++j) {
                const int i = 64 * (w * CPW + j) + lane;
                e[j] = pack(dst[j], (uint32_t)i);
            }
            R::route(A, wz, e, w, lane);
#pragma unroll
            for (int j = 0; j < CPW; ++j) {
                const int q = 64 * (w * CPW + j) + lane;
                const uint64_t x = lds_load_u64_whole(A, own_base + 512u * j);
                if (a.validate) flag_error(a.err, (hi32(x) & (CAP - 1)) != (uint32_t)q, ERR_BAD_PERM);
                dst[j] = lo32(x);  // inv[q] for q = 64k + l
                if (a.inv_out && q < n) store_item<NT>(a.inv_out, 1, o, q, (int32_t)dst[j]);
            }
            __syncthreads();  // A is reused by the next routing
        } else {
            // the source index rides above the destination (for inv_out)
#pragma unroll
            for (int j = 0; j < CPW; ++j) dst[j] |= (uint32_t)(64 * (w * CPW + j) + lane) << 16;
        }

        // a scatter asked only for the inverse still routes once (with no payload);
        // with REPLAY only channel 0 is routed here
        const uint32_t nroute = REPLAY ? 1u
                                       : ((!gather && a.inv_out && a.pay.channels == 0) ? 1u : a.pay.channels);
        uint32_t pdst[REPLAY ? CPW : 1];
#pragma unroll 1
        for (uint32_t c = 0; c < nroute; ++c) {
            // per-column addresses are recomputed per channel instead of being kept
            // live (or spilled) across the whole channel loop
            const int lc = (int)opaque((uint32_t)lane);
            const uint32_t own_c = (uint32_t)lc * 8u + (uint32_t)(w * CPW * 512);
            const int64_t cbase = (int64_t)c * a.pay.cs;
            const bool with_pay = a.pay.channels > 0;
            uint32_t xv[CPW];
            load_columns<CPW, NT>(a.pay.in + (with_pay ? cbase : 0), a.pay.es, o, with_pay ? n : 0, w * CPW,
                              lc, xv, offs);
#pragma unroll
            for (int j = 0; j < CPW; ++j) e[j] = pack(dst[j], xv[j]);
            if constexpr (REPLAY) R::template route<true>(A, wz, e, w, lane, &plan, pdst);
            else R::route(A, wz, e, w, lane);
#pragma unroll
            for (int j = 0; j < CPW; ++j) {
                const int v = 64 * (w * CPW + j) + lc;
                const uint64_t x = lds_load_u64_whole(A, own_c + 512u * j);
                if (a.validate && c == 0 && !gather)
                    flag_error(a.err, (hi32(x) & (CAP - 1)) != (uint32_t)v, ERR_BAD_PERM);
                if (v < n) {
                    if (with_pay) store_item<NT>(a.pay.out + cbase, a.pay.es, o, v, lo32(x));
                    if (!gather && c == 0 && a.inv_out) store_item<NT>(a.inv_out, 1, o, v, (int32_t)(hi32(x) >> 16));
                }
            }
            __syncthreads();  // A is reused by the next channel / tile
        }
        if constexpr (REPLAY) {
#pragma unroll 1
            for (uint32_t c = 1; c < a.pay.channels; c += 2) {
                const int lc = (int)opaque((uint32_t)lane);
                const uint32_t own_c = (uint32_t)lc * 8u + (uint32_t)(w * CPW * 512);
                const bool two = c + 1 < a.pay.channels;
                const int64_t cb0 = (int64_t)c * a.pay.cs;
                const int64_t cb1 = two ? cb0 + a.pay.cs : cb0;
                uint32_t x0[CPW], x1[CPW];
                load_columns<CPW, NT>(a.pay.in + cb0, a.pay.es, o, n, w * CPW, lc, x0, offs);
                load_columns<CPW, NT>(a.pay.in + cb1, a.pay.es, o, n, w * CPW, lc, x1, offs);
#pragma unroll
                for (int j = 0; j < CPW; ++j) e[j] = pack(x1[j], x0[j]);
                R::replay(A, &plan, e, pdst, w, lane);
#pragma unroll
                for (int j = 0; j < CPW; ++j) {
                    const int v = 64 * (w * CPW + j) + lc;
                    const uint64_t x = lds_load_u64_whole(A, own_c + 512u * j);
                    if (v < n) {
                        store_item<NT>(a.pay.out + cb0, a.pay.es, o, v, lo32(x));
                        if (two) store_item<NT>(a.pay.out + cb1, a.pay.es, o, v, hi32(x));
                    }
                }
                __syncthreads();  // A is reused by the next pair / tile
            }
        }
    }
}

// ONESHOT: one workgroup per tile instead of a persistent grid; NT: streaming global
// loads and stores (every word is read or written once).
template <int NW, int CAP, int WPE = 0, bool ONESHOT = false, bool NT = false>
hipError_t launch_perm(const PermuteArgs& a, hipStream_t s) {
    const bool replay = a.pay.channels >= 2;
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
// persistent form of 6.
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
        return launch_perm<16, 8192>(a, s);
    }
    return launch_perm_shaped<16, 16384>(a, s);
}

}  // namespace ts
