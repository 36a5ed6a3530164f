// Device-wide stable sort of one array of 32-bit keys (with an optional payload word
// or the permutation), built on the conflict-free partition of tiles.
//
// Afshani & Sitchinava (Sec. 1) note that partitioning is the step of a quicksort with
// pivots: every row sends its items to the bucket of their range.  Here the buckets are
// the values of a 6-bit digit of the key and the sort is LSD: six passes (digits of 6,
// 6, 6, 6, 6 and 2 bits).  A pass
//   1. counts every tile's digits (tile t, digit d -> hist[d][t]),
//   2. takes the exclusive prefix of hist in digit-major order (goff[d][t]: where tile
//      t's block of digit d starts in the output array),
//   3. partitions every tile on the digit with its conflict-free binary splits
//      (partition.hip, MODE 2) and stores each digit block at goff.
// Tiles hold 4096 keys when the keys travel alone and 8192 items when a payload word
// or the permutation travels with them (radix_tile).
// Each tile partition is stable and the blocks of one digit are laid out in tile order,
// so every pass is a stable partition of the whole array and six passes sort it.
#include <algorithm>
#include <cstdint>

#include "common.hpp"
#include "kernels.hpp"

namespace ts {

namespace {

constexpr int HIST_CPL = 64;  // keys per lane: one wavefront per 4096 keys of a tile
static_assert(RADIX_DIGITS == 64, "lane d sums the counts of digit d");

// offs[t] = min(t * 4096, n) for t = 0 .. T.
__global__ void radix_offsets_kernel(int64_t* offs, int64_t T, int64_t n, int tile) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t <= T) offs[t] = std::min<int64_t>(t * tile, n);
}

// hist[d][t] = number of keys of tile t whose digit is d (digits >= 2^nbits: 0).  One
// wavefront per 4096 keys of the tile.  Lane l counts its 64 keys into a column of its
// own of its wave's LDS table (word 64 d + l): the 64 adds of one instruction hit 64
// distinct words whose banks (word mod 32) differ inside each 32-lane half, so there are
// no bank conflicts.  Lane d then sums row d with 64-bit reads in the order skewed by d,
// so that the 32 lanes of a phase read 8-byte slots 32 d + ((k + d) mod 32): distinct
// modulo 32; the waves' row sums are added through LDS, one word per lane.
// With `limit` > 0 (a device partition with validation), keys >= limit set ERR_BAD_LABEL.
template <int HIST_W>
__global__ __launch_bounds__(64 * HIST_W) void radix_hist_kernel(const uint32_t* __restrict__ keys, int64_t n,
                                                                 int64_t T, int shift, int nbits, uint32_t f32,
                                                                 uint32_t* __restrict__ hist, uint32_t limit,
                                                                 uint32_t* __restrict__ err) {
    __shared__ uint64_t cnt[HIST_W][RADIX_DIGITS * 64 / 2];
    __shared__ uint32_t part[HIST_W][64];
    const int lane = lane_id();
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t t = xcd_contiguous(blockIdx.x, gridDim.x);  // grid = T, one tile each
    const int64_t o = t * (4096 * HIST_W) + (int64_t)w * 4096;
    const uint32_t len = (uint32_t)std::max<int64_t>(0, std::min<int64_t>(4096, n - o));
    uint32_t k[HIST_CPL];
    buffer_load_columns<HIST_CPL, true>(buffer_rsrc(keys + std::min<int64_t>(o, n), len * 4u),
                                        (uint32_t)lane * 4u, k);
    // clear: lane l writes slot 64 r + l (words 128 r + 2l, +1): 16 lanes of a 64-bit
    // write phase cover 16 consecutive slots
#pragma unroll
    for (int r = 0; r < RADIX_DIGITS / 2; ++r) lds_store(cnt[w], (uint32_t)(64 * r + lane) * 8u, uint64_t(0));
    wave_lds_fence();
    if (limit != 0u) {  // labels of a validated device partition (keys are not binary32 there)
        uint32_t bad = 0;
#pragma unroll
        for (int j = 0; j < HIST_CPL; ++j) bad |= (64u * j + (uint32_t)lane < len && k[j] >= limit) ? 1u : 0u;
        flag_error(err, bad != 0u, ERR_BAD_LABEL);
    }
    const uint32_t dmask = (1u << nbits) - 1u;
    uint32_t* words = (uint32_t*)cnt[w];
#pragma unroll
    for (int j = 0; j < HIST_CPL; ++j) {
        const uint32_t i = (uint32_t)(64 * j + lane);
        const uint32_t key = f32 ? f32_to_ordered(k[j]) : k[j];
        if (i < len) atomicAdd(&words[((key >> shift) & dmask) * 64u + (uint32_t)lane], 1u);
    }
    wave_lds_fence();
    uint32_t sum = 0;
#pragma unroll
    for (int q = 0; q < 32; ++q) {
        const uint64_t v = lds_load_u64_whole(cnt[w], (uint32_t)(32 * lane + ((q + lane) & 31)) * 8u);
        sum += lo32(v) + hi32(v);
    }
    if constexpr (HIST_W > 1) {
        part[w][lane] = sum;
        __syncthreads();
        if (w != 0) return;
        sum = 0;
#pragma unroll
        for (int q = 0; q < HIST_W; ++q) sum += part[q][lane];
    }
    hist[(int64_t)lane * T + t] = sum;
}

// Exclusive prefix sum of m words in three launches: per-block sums, a scan of the block
// sums (one workgroup), and the per-block scan with its offset.
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_PER_THREAD = 16;
constexpr int SCAN_BLOCK = SCAN_THREADS * SCAN_PER_THREAD;

// Exclusive scan of one value per thread over the workgroup; *total receives the sum.
template <int THREADS>
TS_DEV uint32_t block_exclusive_scan(uint32_t v, uint32_t* total) {
    __shared__ uint32_t wsum[THREADS / 64];
    const int lane = lane_id();
    const int w = (int)(threadIdx.x >> 6);
    const uint32_t inc = wave_inclusive_scan_u32(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int q = 0; q < THREADS / 64; ++q) {
        const uint32_t s = wsum[q];
        before += (q < w) ? s : 0u;
        all += s;
    }
    __syncthreads();  // wsum is reused by the next call
    *total = all;
    return before + inc - v;
}

__global__ __launch_bounds__(SCAN_THREADS) void scan_sums_kernel(const uint32_t* __restrict__ in, int64_t m,
                                                                  uint32_t* __restrict__ bsum) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK + (int64_t)threadIdx.x * SCAN_PER_THREAD;
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_PER_THREAD; ++i) s += (base + i < m) ? in[base + i] : 0u;
    uint32_t total;
    block_exclusive_scan<SCAN_THREADS>(s, &total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// One workgroup scans nb block sums in place (chunks of 1024 with a running carry).
__global__ __launch_bounds__(1024) void scan_block_sums_kernel(uint32_t* __restrict__ bsum, int64_t nb) {
    uint32_t carry = 0;
    for (int64_t c = 0; c < nb; c += 1024) {
        const int64_t i = c + threadIdx.x;
        const uint32_t v = (i < nb) ? bsum[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_exclusive_scan<1024>(v, &total);
        if (i < nb) bsum[i] = carry + ex;
        carry += total;
    }
}

__global__ __launch_bounds__(SCAN_THREADS) void scan_apply_kernel(const uint32_t* __restrict__ in, int64_t m,
                                                                   const uint32_t* __restrict__ bsum,
                                                                   uint32_t* __restrict__ out) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK + (int64_t)threadIdx.x * SCAN_PER_THREAD;
    uint32_t v[SCAN_PER_THREAD];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_PER_THREAD; ++i) {
        v[i] = (base + i < m) ? in[base + i] : 0u;
        s += v[i];
    }
    uint32_t total;
    uint32_t run = bsum[blockIdx.x] + block_exclusive_scan<SCAN_THREADS>(s, &total);
#pragma unroll
    for (int i = 0; i < SCAN_PER_THREAD; ++i) {
        if (base + i < m) out[base + i] = run;
        run += v[i];
    }
}

void launch_hist(int tile, const uint32_t* keys, int64_t n, int64_t T, int shift, int nbits, uint32_t f32,
                 uint32_t* hist, uint32_t limit, uint32_t* err, hipStream_t s) {
    if (tile == 8192)
        hipLaunchKernelGGL(radix_hist_kernel<2>, dim3((unsigned)T), dim3(128), 0, s, keys, n, T, shift, nbits, f32,
                           hist, limit, err);
    else
        hipLaunchKernelGGL(radix_hist_kernel<1>, dim3((unsigned)T), dim3(64), 0, s, keys, n, T, shift, nbits, f32,
                           hist, limit, err);
}

}  // namespace

DeviceSortLayout device_sort_layout(int64_t n, int tile, bool with_pay, bool pingpong) {
    DeviceSortLayout L{};
    const int64_t T = (n + tile - 1) / tile;
    const int64_t m = (int64_t)RADIX_DIGITS * T;
    const int64_t nb = (m + SCAN_BLOCK - 1) / SCAN_BLOCK;
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    size_t off = 256;  // header: error word
    L.offsets = off;
    off += al((size_t)(T + 1) * 8);
    L.hist = off;
    off += al((size_t)m * 4);
    L.goff = off;
    off += al((size_t)m * 4);
    L.bsum = off;
    off += al((size_t)nb * 4);
    L.keys = off;
    off += al(pingpong ? (size_t)n * 4 : 0);
    L.pay = off;
    off += al(pingpong && with_pay ? (size_t)n * 4 : 0);
    L.total = off;
    return L;
}

hipError_t launch_device_sort(const DeviceSortArgs& d, void* ws, hipStream_t s) {
    const int64_t n = d.n;
    if (n == 0) return hipSuccess;
    const bool carry = d.pay_in != nullptr || d.perm_out != nullptr;  // a payload word travels
    const int tile = radix_tile(carry);
    const DeviceSortLayout L = device_sort_layout(n, tile, carry);
    char* w = (char*)ws;
    int64_t* offs = (int64_t*)(w + L.offsets);
    uint32_t* hist = (uint32_t*)(w + L.hist);
    uint32_t* goff = (uint32_t*)(w + L.goff);
    uint32_t* bsum = (uint32_t*)(w + L.bsum);
    uint32_t* tk = (uint32_t*)(w + L.keys);
    uint32_t* tp = carry ? (uint32_t*)(w + L.pay) : nullptr;
    const int64_t T = (n + tile - 1) / tile;
    const int64_t m = (int64_t)RADIX_DIGITS * T;
    const int64_t nb = (m + SCAN_BLOCK - 1) / SCAN_BLOCK;
    uint32_t* out_pay = d.pay_out ? d.pay_out : (uint32_t*)d.perm_out;  // final payload words

    hipLaunchKernelGGL(radix_offsets_kernel, dim3((unsigned)((T + 1 + 255) / 256)), dim3(256), 0, s, offs, T, n, tile);
    hipError_t e = hipGetLastError();
    // buffers: in -> ws, ws -> out, out -> ws, ..., ws -> out
    constexpr int kPasses = RADIX_PASSES;
    static_assert(kPasses % 2 == 0, "an even number of passes ends in the output");
    for (int p = 0; p < kPasses && e == hipSuccess; ++p) {
        const bool to_ws = (p % 2) == 0;
        const uint32_t* kin = p == 0 ? d.keys_in : (to_ws ? d.keys_out : tk);
        const uint32_t* pin = p == 0 ? d.pay_in : (to_ws ? out_pay : tp);
        uint32_t* kout = to_ws ? tk : d.keys_out;
        uint32_t* pout = carry ? (to_ws ? tp : out_pay) : nullptr;
        const uint32_t f32_in = (p == 0) ? d.f32 : 0u;
        launch_hist(tile, kin, n, T, RADIX_BITS * p, std::min(RADIX_BITS, 32 - RADIX_BITS * p), f32_in, hist, 0u,
                    d.err, s);
        hipLaunchKernelGGL(scan_sums_kernel, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, hist, m, bsum);
        hipLaunchKernelGGL(scan_block_sums_kernel, dim3(1), dim3(1024), 0, s, bsum, nb);
        hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, hist, m, bsum, goff);
        e = hipGetLastError();
        if (e != hipSuccess) break;
        RadixPass r{};
        r.keys_in = kin;
        r.keys_out = kout;
        r.pay_in = pin;  // NULL in pass 0 without a payload: the kernel carries the index
        r.pay_out = pout;
        r.offsets = offs;
        r.num_tiles = T;
        r.shift = RADIX_BITS * p;
        r.nbits = std::min(RADIX_BITS, 32 - RADIX_BITS * p);
        r.f32_in = f32_in;
        r.f32_out = (p == kPasses - 1) ? d.f32 : 0u;
        r.hist = hist;
        r.goff = goff;
        r.n_total = n;
        r.err = d.err;
        r.tile = tile;
        e = launch_radix_pass(r, s);
    }
    return e;
}

hipError_t launch_device_partition(const DeviceSortArgs& d, int nbits, uint32_t num_classes,
                                   bool validate, void* ws, hipStream_t s) {
    const int64_t n = d.n;
    if (n == 0) return hipSuccess;
    const bool carry = d.pay_in != nullptr || d.perm_out != nullptr;
    const int tile = radix_tile(carry);
    const DeviceSortLayout L = device_sort_layout(n, tile, carry, false);
    char* w = (char*)ws;
    int64_t* offs = (int64_t*)(w + L.offsets);
    uint32_t* hist = (uint32_t*)(w + L.hist);
    uint32_t* goff = (uint32_t*)(w + L.goff);
    uint32_t* bsum = (uint32_t*)(w + L.bsum);
    const int64_t T = (n + tile - 1) / tile;
    const int64_t m = (int64_t)RADIX_DIGITS * T;
    const int64_t nb = (m + SCAN_BLOCK - 1) / SCAN_BLOCK;
    hipLaunchKernelGGL(radix_offsets_kernel, dim3((unsigned)((T + 1 + 255) / 256)), dim3(256), 0, s, offs, T, n, tile);
    launch_hist(tile, d.keys_in, n, T, 0, nbits, 0u, hist, validate ? num_classes : 0u, d.err, s);
    hipLaunchKernelGGL(scan_sums_kernel, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, hist, m, bsum);
    hipLaunchKernelGGL(scan_block_sums_kernel, dim3(1), dim3(1024), 0, s, bsum, nb);
    hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, hist, m, bsum, goff);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    RadixPass r{};
    r.keys_in = d.keys_in;
    r.keys_out = d.keys_out;
    r.pay_in = d.pay_in;  // NULL: the kernel carries the index (for perm_out)
    r.pay_out = d.pay_out ? d.pay_out : (uint32_t*)d.perm_out;
    r.offsets = offs;
    r.num_tiles = T;
    r.shift = 0;
    r.nbits = nbits;
    r.hist = hist;
    r.goff = goff;
    r.n_total = n;
    r.err = d.err;
    r.tile = tile;
    return launch_radix_pass(r, s);
}

}  // namespace ts
