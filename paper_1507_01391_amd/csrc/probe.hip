// Measurement kernels: an LDS access probe (bank count, width and phase
// behaviour of gfx950 LDS, read by the SQ_LDS_BANK_CONFLICT counter and by
// s_memtime) and a plain HBM copy (the achievable-bandwidth reference).
#include <cstdint>

#include "common.hpp"
#include "kernels.hpp"

namespace ts {

namespace {

constexpr int PROBE_WORDS = 16384;  // 64 KiB of LDS

template <int OP, int WIDTH>
__global__ __launch_bounds__(1024) void lds_probe_kernel(const uint32_t* lane_words, int iters,
                                                         uint64_t* cycles_out, uint32_t* sink) {
    __shared__ uint32_t L[PROBE_WORDS];
    const int lane = lane_id();
    const int wave = (int)(threadIdx.x >> 6);
    for (int i = threadIdx.x; i < PROBE_WORDS; i += blockDim.x) L[i] = (uint32_t)i * 2654435761u;
    __syncthreads();
    uint32_t word = lane_words[lane] % PROBE_WORDS;
    word &= ~(uint32_t)(WIDTH - 1);
    // LDS byte address of L[word] (address space 3), so the array is really allocated
    // and every access stays inside it.
    typedef __attribute__((address_space(3))) uint32_t lds_u32;
    const uint32_t byte = (uint32_t)(uintptr_t)((lds_u32*)&L[word]);
    uint32_t acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0;
    const uint64_t t0 = __builtin_amdgcn_s_memtime();
    for (int it = 0; it < iters; ++it) {
        if (OP == 0) {
            if (WIDTH == 1) {
                uint32_t v0, v1, v2, v3;
                asm volatile(
                    "ds_read_b32 %0, %4\n"
                    "ds_read_b32 %1, %4\n"
                    "ds_read_b32 %2, %4\n"
                    "ds_read_b32 %3, %4\n"
                    "s_waitcnt lgkmcnt(0)\n"
                    : "=v"(v0), "=v"(v1), "=v"(v2), "=v"(v3)
                    : "v"(byte)
                    : "memory");
                acc0 ^= v0;
                acc1 ^= v1;
                acc2 ^= v2;
                acc3 ^= v3;
            } else if (WIDTH == 2) {
                uint64_t v0, v1, v2, v3;
                asm volatile(
                    "ds_read_b64 %0, %4\n"
                    "ds_read_b64 %1, %4\n"
                    "ds_read_b64 %2, %4\n"
                    "ds_read_b64 %3, %4\n"
                    "s_waitcnt lgkmcnt(0)\n"
                    : "=v"(v0), "=v"(v1), "=v"(v2), "=v"(v3)
                    : "v"(byte)
                    : "memory");
                acc0 ^= (uint32_t)v0 ^ (uint32_t)(v1 >> 32);
                acc1 ^= (uint32_t)v2 ^ (uint32_t)(v3 >> 32);
            } else {
                typedef uint32_t u4 __attribute__((ext_vector_type(4)));
                u4 v0, v1;
                asm volatile(
                    "ds_read_b128 %0, %2\n"
                    "ds_read_b128 %1, %2\n"
                    "s_waitcnt lgkmcnt(0)\n"
                    : "=v"(v0), "=v"(v1)
                    : "v"(byte)
                    : "memory");
                acc0 ^= v0.x ^ v1.w;
                acc1 ^= v0.y ^ v1.z;
            }
        } else if (OP == 1) {
            const uint32_t d = (uint32_t)it ^ (uint32_t)lane;
            if (WIDTH == 1) {
                asm volatile(
                    "ds_write_b32 %0, %1\n"
                    "ds_write_b32 %0, %1\n"
                    "ds_write_b32 %0, %1\n"
                    "ds_write_b32 %0, %1\n"
                    "s_waitcnt lgkmcnt(0)\n"
                    :
                    : "v"(byte), "v"(d)
                    : "memory");
            } else if (WIDTH == 2) {
                const uint64_t dd = ((uint64_t)d << 32) | d;
                asm volatile(
                    "ds_write_b64 %0, %1\n"
                    "ds_write_b64 %0, %1\n"
                    "ds_write_b64 %0, %1\n"
                    "ds_write_b64 %0, %1\n"
                    "s_waitcnt lgkmcnt(0)\n"
                    :
                    : "v"(byte), "v"(dd)
                    : "memory");
            } else {
                typedef uint32_t u4 __attribute__((ext_vector_type(4)));
                u4 dd = {d, d, d, d};
                asm volatile(
                    "ds_write_b128 %0, %1\n"
                    "ds_write_b128 %0, %1\n"
                    "s_waitcnt lgkmcnt(0)\n"
                    :
                    : "v"(byte), "v"(dd)
                    : "memory");
            }
        } else {
            const uint32_t src = (lane_words[lane] & 63u) * 4u;
            uint32_t v0, v1, v2, v3;
            const uint32_t x = (uint32_t)it + (uint32_t)lane;
            asm volatile(
                "ds_bpermute_b32 %0, %4, %5\n"
                "ds_bpermute_b32 %1, %4, %5\n"
                "ds_bpermute_b32 %2, %4, %5\n"
                "ds_bpermute_b32 %3, %4, %5\n"
                "s_waitcnt lgkmcnt(0)\n"
                : "=v"(v0), "=v"(v1), "=v"(v2), "=v"(v3)
                : "v"(src), "v"(x)
                : "memory");
            acc0 ^= v0;
            acc1 ^= v1;
            acc2 ^= v2;
            acc3 ^= v3;
        }
    }
    const uint64_t t1 = __builtin_amdgcn_s_memtime();
    const int gw = (int)blockIdx.x * (int)(blockDim.x >> 6) + wave;
    if (lane == 0) cycles_out[gw] = t1 - t0;
    __syncthreads();
    sink[gw * 64 + lane] = acc0 ^ acc1 ^ acc2 ^ acc3 ^ L[(lane * 97u + (uint32_t)wave) % PROBE_WORDS];
}

template <int OP, int WIDTH>
hipError_t launch_probe_t(const uint32_t* lane_words, int iters, int waves, int groups,
                          uint64_t* cycles_out, uint32_t* sink, hipStream_t s) {
    hipLaunchKernelGGL((lds_probe_kernel<OP, WIDTH>), dim3(groups), dim3(waves * 64), 0, s,
                       lane_words, iters, cycles_out, sink);
    return hipGetLastError();
}

// Copy: every workgroup moves one contiguous chunk of 256 x COPY_U 16-byte vectors with
// streaming loads and stores, all loads issued before the first store; the last
// chunk may be partial.
typedef uint32_t v4u __attribute__((ext_vector_type(4)));
constexpr int COPY_U = 8;
constexpr size_t COPY_CHUNK = 256 * COPY_U;

__global__ __launch_bounds__(256) void copy_kernel(const v4u* __restrict__ src,
                                                   v4u* __restrict__ dst, size_t n16) {
    const size_t c = (size_t)blockIdx.x * COPY_CHUNK;
    if (c + COPY_CHUNK <= n16) {
        v4u r[COPY_U];
#pragma unroll
        for (int u = 0; u < COPY_U; ++u) r[u] = __builtin_nontemporal_load(src + c + u * 256 + threadIdx.x);
#pragma unroll
        for (int u = 0; u < COPY_U; ++u) __builtin_nontemporal_store(r[u], dst + c + u * 256 + threadIdx.x);
    } else {
        for (size_t i = c + threadIdx.x; i < n16; i += 256) dst[i] = src[i];
    }
}

__global__ void copy_tail_kernel(const uint8_t* src, uint8_t* dst, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

__global__ void fill_zero_kernel(uint32_t* p, size_t nwords) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < nwords; i += stride) p[i] = 0u;
}

}  // namespace

hipError_t launch_lds_probe(const uint32_t* lane_words, int op, int width, int iters, int waves,
                            int groups, uint64_t* cycles_out, uint32_t* sink, hipStream_t s) {
    if (op == 0 && width == 1) return launch_probe_t<0, 1>(lane_words, iters, waves, groups, cycles_out, sink, s);
    if (op == 0 && width == 2) return launch_probe_t<0, 2>(lane_words, iters, waves, groups, cycles_out, sink, s);
    if (op == 0 && width == 4) return launch_probe_t<0, 4>(lane_words, iters, waves, groups, cycles_out, sink, s);
    if (op == 1 && width == 1) return launch_probe_t<1, 1>(lane_words, iters, waves, groups, cycles_out, sink, s);
    if (op == 1 && width == 2) return launch_probe_t<1, 2>(lane_words, iters, waves, groups, cycles_out, sink, s);
    if (op == 1 && width == 4) return launch_probe_t<1, 4>(lane_words, iters, waves, groups, cycles_out, sink, s);
    if (op == 2) return launch_probe_t<2, 1>(lane_words, iters, waves, groups, cycles_out, sink, s);
    return hipErrorInvalidValue;
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
    const size_t n16 = bytes / 16;
    if (n16) {
        const size_t grid = (n16 + COPY_CHUNK - 1) / COPY_CHUNK;
        if (grid > (size_t)INT32_MAX) return hipErrorInvalidValue;
        hipLaunchKernelGGL(copy_kernel, dim3((unsigned)grid), dim3(256), 0, s, (const v4u*)src, (v4u*)dst, n16);
    }
    const size_t tail = bytes - n16 * 16;
    if (tail) {
        hipLaunchKernelGGL(copy_tail_kernel, dim3(1), dim3(64), 0, s,
                           (const uint8_t*)src + n16 * 16, (uint8_t*)dst + n16 * 16, tail);
    }
    return hipGetLastError();
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
    const size_t nw = bytes / 4;
    if (nw == 0) return hipSuccess;
    const int grid = (int)((nw + 255) / 256 < 1024 ? (nw + 255) / 256 : 1024);
    hipLaunchKernelGGL(fill_zero_kernel, dim3(grid), dim3(256), 0, s, (uint32_t*)p, nw);
    return hipGetLastError();
}

namespace {

// One workgroup per tile (grid-stride over tiles), threads stride over the tile.
__global__ __launch_bounds__(256) void label_check_kernel(const uint32_t* __restrict__ labels,
                                                          const int64_t* __restrict__ offs,
                                                          int64_t num_tiles, uint32_t num_classes,
                                                          uint32_t* err) {
    for (int64_t t = blockIdx.x; t < num_tiles; t += gridDim.x) {
        const int64_t o = offs[t];
        const int64_t n = offs[t + 1] - o;
        bool bad = false;
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) bad |= labels[o + i] >= num_classes;
        flag_error(err, bad, ERR_BAD_LABEL);
    }
}

}  // namespace

hipError_t launch_label_check(const uint32_t* labels, const int64_t* offsets, int64_t num_tiles,
                              uint32_t num_classes, uint32_t* err, hipStream_t s) {
    if (num_tiles == 0) return hipSuccess;
    const int64_t g = num_tiles < 8192 ? num_tiles : 8192;
    hipLaunchKernelGGL(label_check_kernel, dim3((unsigned)g), dim3(256), 0, s, labels, offsets,
                       num_tiles, num_classes, err);
    return hipGetLastError();
}


}  // namespace ts
