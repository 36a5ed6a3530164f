// tile_sort_noalloc: tile_sort for callers that cannot allocate device memory (code under
// stream capture, tight serving loops, harnesses that forbid hipMalloc).  The scratch
// that tile_sort keeps in the caller's workspace -- the error word, the merge schedule's
// work counters and bin lists, the permutation of a payload without perm_out -- lives
// here in one static device array per GPU instead.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "../../include/tilesort.h"
#include "kernels.hpp"

namespace {

// 32 MiB per GPU, held until the process ends.  Every call on a GPU uses the same array
// (calls that overlap on one GPU race on it).
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on each GPU (the array's name in host code is only a
// handle for the runtime), looked up once per device with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// dst |= src, one word (the error bits of this call, for the caller).
__global__ void or_error_word_kernel(const uint32_t* src, uint32_t* dst) {
    if (threadIdx.x == 0 && src[0] != 0u) atomicOr(dst, src[0]);
}

int scratch_of_current_device(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return ts::set_error(TS_ERR_HIP, "tile_sort_noalloc: hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices) return ts::set_error(TS_ERR_UNSUPPORTED, "tile_sort_noalloc: device index >= 64");
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[dev] == nullptr) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            char msg[160];
            snprintf(msg, sizeof msg, "tile_sort_noalloc: hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            return ts::set_error(TS_ERR_HIP, msg);
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return TS_OK;
}

}  // namespace

extern "C" ts_status tile_sort_noalloc(const uint32_t* keys_in, uint32_t* keys_out, const uint32_t* payload_in,
                                       uint32_t* payload_out, uint32_t channels, int64_t elem_stride,
                                       int64_t chan_stride, int32_t* perm_out, const int64_t* tile_offsets,
                                       int64_t num_tiles, int64_t total_len, int64_t max_tile_len,
                                       uint32_t flags, uint32_t* err_out, void* stream) {
    const size_t need = ts_workspace_bytes(TS_OP_SORT, flags, num_tiles, total_len, max_tile_len, channels);
    if (need > kScratchBytes) {
        char msg[200];
        snprintf(msg, sizeof msg,
                 "tile_sort_noalloc: this call needs %zu bytes of scratch; the static scratch holds %zu",
                 need, kScratchBytes);
        return (ts_status)ts::set_error(TS_ERR_WORKSPACE, msg);
    }
    void* ws = nullptr;
    const int st = scratch_of_current_device(&ws);
    if (st != TS_OK) return (ts_status)st;
    hipStream_t s = (hipStream_t)stream;
    // the header (error word, counters) starts at zero on every call; a fill kernel, not
    // a memset node, so the call stays capturable
    hipError_t e = ts::launch_fill_zero(ws, 256, s);
    if (e != hipSuccess) return (ts_status)ts::set_error(TS_ERR_HIP, "tile_sort_noalloc: clearing the scratch header failed");
    const ts_status r = tile_sort(keys_in, keys_out, payload_in, payload_out, channels, elem_stride, chan_stride,
                                  perm_out, tile_offsets, num_tiles, total_len, max_tile_len, flags, ws,
                                  kScratchBytes, stream);
    if (r != TS_OK || err_out == nullptr) return r;
    hipLaunchKernelGGL(or_error_word_kernel, dim3(1), dim3(64), 0, s, (const uint32_t*)ws, err_out);
    if ((e = hipGetLastError()) != hipSuccess)
        return (ts_status)ts::set_error(TS_ERR_HIP, "tile_sort_noalloc: error word copy failed");
    return TS_OK;
}
