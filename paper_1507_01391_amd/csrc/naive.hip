// Baseline kernels: the same problems solved the plain way, with a direct LDS
// scatter to each item's computed destination.  The destinations of one wave
// instruction are data dependent, so several lanes often hit one bank (bank
// conflicts).  They exist only to be measured beside the conflict-free kernels.
#include <algorithm>
#include <cstdint>

#include "common.hpp"
#include "kernels.hpp"

namespace ts {

namespace {

// Launch shape of the naive kernels (tuning knob): a persistent grid, or one
// workgroup per tile.
static int g_naive_oneshot = 0;

int naive_grid(const void* kern, int threads, int64_t tiles) {
    return g_naive_oneshot ? (int)std::min<int64_t>(tiles, INT32_MAX)
                           : persistent_grid(kern, threads, 0, tiles);
}


// Inclusive prefix sum across the 64 lanes of a wave.
TS_DEV int wave_inclusive_scan(int v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

// Stable partition: per-column multisplit ranks (label match by ballots), running
// per-class counts per wave, then one direct scatter into LDS.
template <int NW, int CAP>
__global__ __launch_bounds__(NW * 64) void partition_naive_kernel(PartitionArgs a) {
    constexpr int CPW = CAP / 64 / NW;
    __shared__ uint64_t A[CAP];
    __shared__ int cnt[NW][64];
    __shared__ int start[NW][64];
    const int lane = lane_id();
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t lmask = (1u << a.nbits) - 1u;
    const bool has_pay = a.pay.channels > 0;
    const int wv = w;
    uint32_t Llab[CPW], Lpay[CPW];
    int64_t Lo = 0;
    int Ln = -1;
    auto issue = [&](int64_t tt) {
        const bool exists = tt < a.num_tiles;
        const int64_t t0 = exists ? tt : 0;
        Lo = a.offsets[t0];
        const int64_t len = a.offsets[t0 + 1] - Lo;
        Ln = !exists ? -1 : ((len > CAP) ? -2 : (int)len);
        const int nn = (Ln > 0) ? Ln : 0;
        load_columns<CPW>(a.labels_in, 1, Lo, nn, wv * CPW, lane, Llab, a.offsets);
        load_columns<CPW>(a.pay.in, a.pay.es, Lo, has_pay ? nn : 0, wv * CPW, lane, Lpay, a.offsets);
    };
    int64_t t = blockIdx.x;
    issue(t);
    for (; t < a.num_tiles; t += gridDim.x) {
        const int64_t o = Lo;
        const int n = Ln;
        if (n == -2) {
            if (threadIdx.x == 0) atomicOr(a.err, ERR_TILE_TOO_LONG);
            issue(t + gridDim.x);
            continue;
        }
        uint64_t e[CPW];
        int rank[CPW];
        cnt[w][lane] = 0;
        uint32_t labs[CPW], pays[CPW];
#pragma unroll
        for (int j = 0; j < CPW; ++j) { labs[j] = Llab[j]; pays[j] = Lpay[j]; }
        issue(t + gridDim.x);
#pragma unroll
        for (int j = 0; j < CPW; ++j) {
            const int i = 64 * (wv * CPW + j) + lane;
            uint32_t lab = lmask, pay = 0;
            const bool real = i < n;
            if (real) {
                lab = labs[j] & lmask;
                pay = pays[j];
            }
            e[j] = pack(((uint32_t)i << 16) | lab, pay);
            uint64_t match = ballot(real);
            for (int b = 0; b < a.nbits; ++b) {
                const uint64_t bb = ballot((lab >> b) & 1u);
                match &= ((lab >> b) & 1u) ? bb : ~bb;
            }
            rank[j] = 0;
            if (real) {
                const int inr = (int)count_below(match);
                const int tot = popc64(match);
                const int base = cnt[w][lab];
                rank[j] = base + inr;
                if (inr == tot - 1) cnt[w][lab] = base + tot;
            }
        }
        __syncthreads();
        if (w == 0) {
            int run = 0;
            int tot = 0;
            for (int q = 0; q < NW; ++q) tot += cnt[q][lane];
            const int excl = wave_inclusive_scan(tot) - tot;
            run = excl;
            for (int q = 0; q < NW; ++q) {
                start[q][lane] = run;
                run += cnt[q][lane];
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < CPW; ++j) {
            const int i = 64 * (w * CPW + j) + lane;
            if (i < n) {
                const uint32_t lab = hi32(e[j]) & 0xFFFFu;
                A[start[w][lab] + rank[j]] = e[j];  // direct scatter: bank conflicts
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < CPW; ++j) {
            const int v = 64 * (w * CPW + j) + lane;
            if (v < n) {
                const uint64_t x = A[v];
                const uint32_t h = hi32(x);
                if (a.labels_out) a.labels_out[o + v] = h & 0xFFFFu;
                if (has_pay) a.pay.out[(o + v) * a.pay.es] = lo32(x);
                if (a.perm_out) a.perm_out[o + v] = (int32_t)(h >> 16);
            }
        }
        __syncthreads();
    }
}

template <int NW, int CAP>
hipError_t launch_pn(const PartitionArgs& a, hipStream_t s) {
    auto kern = partition_naive_kernel<NW, CAP>;
    const int grid = naive_grid((const void*)kern, NW * 64, a.num_tiles);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NW * 64), 0, s, a);
    return hipGetLastError();
}

// Permutation by a direct LDS scatter (SCATTER: A[pi[i]] = in[i], then linear reads)
// or a direct LDS gather (GATHER: A[q] = in[q], then out[i] = A[pi[i]]).
template <int NW, int CAP>
__global__ __launch_bounds__(NW * 64) void permute_naive_kernel(PermuteArgs a) {
    constexpr int CPW = CAP / 64 / NW;
    __shared__ uint32_t A[CAP];
    const int lane = lane_id();
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (int64_t t = blockIdx.x; t < a.num_tiles; t += gridDim.x) {
        const int64_t o = a.offsets[t];
        const int64_t len = a.offsets[t + 1] - o;
        if (len > CAP) {
            if (threadIdx.x == 0) atomicOr(a.err, ERR_TILE_TOO_LONG);
            continue;
        }
        const int n = (int)len;
        int32_t pidx[CPW];
        if (a.pi16) {
            uint16_t p16[CPW];
            load_columns<CPW>((const uint16_t*)a.pi, 1, o, n, w * CPW, lane, p16, a.offsets);
#pragma unroll
            for (int j = 0; j < CPW; ++j) pidx[j] = (int32_t)p16[j];
        } else {
            load_columns<CPW>(a.pi, 1, o, n, w * CPW, lane, pidx, a.offsets);
        }
#pragma unroll
        for (int j = 0; j < CPW; ++j) pidx[j] &= (CAP - 1);
        if (a.inv_out) {  // inv[pi[i]] = i, a direct scatter to global memory
#pragma unroll
            for (int j = 0; j < CPW; ++j) {
                const int i = 64 * (w * CPW + j) + lane;
                if (i < n) {
                    if (a.inv16) ((uint16_t*)a.inv_out)[o + pidx[j]] = (uint16_t)i;
                    else a.inv_out[o + pidx[j]] = i;
                }
            }
        }
        for (uint32_t c = 0; c < a.pay.channels; ++c) {
            const int64_t cb = (int64_t)c * a.pay.cs;
            uint32_t xv[CPW];
            load_columns<CPW>(a.pay.in + cb, a.pay.es, o, n, w * CPW, lane, xv, a.offsets);
#pragma unroll
            for (int j = 0; j < CPW; ++j) {
                const int i = 64 * (w * CPW + j) + lane;
                if (i < n) {
                    if (a.direction == 0) A[pidx[j]] = xv[j];   // direct scatter: bank conflicts
                    else A[i] = xv[j];
                }
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < CPW; ++j) {
                const int i = 64 * (w * CPW + j) + lane;
                if (i < n) {
                    const uint32_t v = (a.direction == 0) ? A[i] : A[pidx[j]];  // gather: conflicts
                    store_item(a.pay.out + cb, a.pay.es, o, i, v);
                }
            }
            __syncthreads();
        }
    }
}

template <int NW, int CAP>
hipError_t launch_pmn(const PermuteArgs& a, hipStream_t s) {
    auto kern = permute_naive_kernel<NW, CAP>;
    const int grid = naive_grid((const void*)kern, NW * 64, a.num_tiles);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NW * 64), 0, s, a);
    return hipGetLastError();
}

// LSD radix sort with 4-bit digits: per pass, per-column multisplit ranks and one
// direct LDS scatter (bank conflicts).  Items are (ordered key, position); the tile
// is padded to the capacity with keys 0xFFFFFFFF and positions >= n.
template <int NW, int CAP>
__global__ __launch_bounds__(NW * 64) void sort_naive_kernel(SortArgs a) {
    constexpr int CPW = CAP / 64 / NW;
    __shared__ uint64_t A[CAP];
    __shared__ int cnt[NW][16];
    __shared__ int start[NW][16];
    const int lane = lane_id();
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (int64_t t = blockIdx.x; t < a.num_tiles; t += gridDim.x) {
        const int64_t o = a.offsets[t];
        const int64_t len = a.offsets[t + 1] - o;
        if (len > CAP) {
            if (threadIdx.x == 0) atomicOr(a.err, ERR_TILE_TOO_LONG);
            continue;
        }
        const int n = (int)len;
        uint32_t kv[CPW];
        load_columns<CPW>(a.keys_in, 1, o, n, w * CPW, lane, kv, a.offsets);
        uint64_t e[CPW];
#pragma unroll
        for (int j = 0; j < CPW; ++j) {
            const int i = 64 * (w * CPW + j) + lane;
            const uint32_t key = (i < n) ? (a.f32 ? f32_to_ordered(kv[j]) : kv[j]) : 0xFFFFFFFFu;
            e[j] = pack(key, (uint32_t)i);
        }
#pragma unroll 1
        for (int pass = 0; pass < 8; ++pass) {
            const int sh = 4 * pass;
            if (lane < 16) cnt[w][lane] = 0;
            int rank[CPW];
#pragma unroll
            for (int j = 0; j < CPW; ++j) {
                const uint32_t d = (hi32(e[j]) >> sh) & 15u;
                uint64_t match = ~0ull;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const uint64_t bb = ballot((d >> b) & 1u);
                    match &= ((d >> b) & 1u) ? bb : ~bb;
                }
                const int inr = (int)count_below(match);
                const int tot = popc64(match);
                const int base = cnt[w][d];
                rank[j] = base + inr;
                if (inr == tot - 1) cnt[w][d] = base + tot;
            }
            __syncthreads();
            if (w == 0 && lane < 16) {
                int tot = 0;
                for (int q = 0; q < NW; ++q) tot += cnt[q][lane];
                int excl = 0;
                for (int d2 = 0; d2 < 16; ++d2) {
                    const int td = __shfl(tot, d2, 64);
                    excl += (d2 < lane) ? td : 0;
                }
                int run = excl;
                for (int q = 0; q < NW; ++q) {
                    start[q][lane] = run;
                    run += cnt[q][lane];
                }
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < CPW; ++j) {
                const uint32_t d = (hi32(e[j]) >> sh) & 15u;
                A[start[w][d] + rank[j]] = e[j];  // direct scatter: bank conflicts
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < CPW; ++j) e[j] = A[64 * (w * CPW + j) + lane];
            __syncthreads();
        }
#pragma unroll
        for (int j = 0; j < CPW; ++j) {
            const int v = 64 * (w * CPW + j) + lane;
            if (v < n) {
                const uint32_t key = hi32(e[j]);
                if (a.keys_out) store_item(a.keys_out, 1, o, v, a.f32 ? ordered_to_f32(key) : key);
                if (a.perm_out) store_item(a.perm_out, 1, o, v, (int32_t)lo32(e[j]));
            }
        }
    }
}

template <int NW, int CAP>
hipError_t launch_sn(const SortArgs& a, hipStream_t s) {
    auto kern = sort_naive_kernel<NW, CAP>;
    const int grid = naive_grid((const void*)kern, NW * 64, a.num_tiles);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NW * 64), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sort_naive(const SortArgs& a, int64_t max_len, hipStream_t s) {
    if (a.num_tiles == 0) return hipSuccess;
    if (max_len <= 1024) return launch_sn<4, 1024>(a, s);
    if (max_len <= 2048) return launch_sn<4, 2048>(a, s);
    if (max_len <= 4096) return launch_sn<8, 4096>(a, s);
    if (max_len <= 8192) return launch_sn<8, 8192>(a, s);
    return launch_sn<16, 16384>(a, s);
}

hipError_t launch_permute_naive(const PermuteArgs& a, int64_t max_len, hipStream_t s) {
    if (a.num_tiles == 0) return hipSuccess;
    if (max_len <= 4096) return launch_pmn<8, 4096>(a, s);
    if (max_len <= 8192) return launch_pmn<8, 8192>(a, s);
    return launch_pmn<16, 16384>(a, s);
}

void set_naive_oneshot(int v) { g_naive_oneshot = v; }

hipError_t launch_partition_naive(const PartitionArgs& a, int64_t max_len, hipStream_t s) {
    if (a.num_tiles == 0) return hipSuccess;
    if (max_len <= 1024) return launch_pn<4, 1024>(a, s);
    if (max_len <= 2048) return launch_pn<4, 2048>(a, s);
    if (max_len <= 4096) return launch_pn<8, 4096>(a, s);
    if (max_len <= 8192) return launch_pn<8, 8192>(a, s);
    return launch_pn<16, 16384>(a, s);
}

}  // namespace ts
