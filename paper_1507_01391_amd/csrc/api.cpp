// C interface of libtilesort.so: argument checks, kernel selection and error
// reporting.  The declarations and their documentation are in include/tilesort.h.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>

#include "../../include/tilesort.h"
#include "kernels.hpp"

namespace {

thread_local std::string g_last_error;

ts_status fail(ts_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
ts_status fail(ts_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

ts_status hip_status(hipError_t e, const char* what) {
    if (e == hipSuccess) return TS_OK;
    return fail(TS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

static_assert(TS_ERRBIT_TILE_TOO_LONG == ts::ERR_TILE_TOO_LONG && TS_ERRBIT_BAD_LABEL == ts::ERR_BAD_LABEL &&
                  TS_ERRBIT_BAD_PERM == ts::ERR_BAD_PERM && TS_ERRBIT_BAD_OFFSETS == ts::ERR_BAD_OFFSETS,
              "the error bits of the C interface are the kernels' bits");

// Workspace layout: word 0 = error bits; words 1..63 reserved (counters); 256 bytes total.
constexpr size_t kWorkspaceBytes = 256;

int sched_of(uint32_t flags) { return (int)((flags >> 8) & 0xFu); }

// Schedules TS_SCHED_AUTO picks for tile_sort, by max_tile_len up to 4096, 8192 and
// 16384 (longer tiles always take the merge schedule).  Set by the autotuner through
// ts_tune("sort_plan_<len>", schedule).
int g_sort_plan[3] = {TS_SCHED_BITONIC, TS_SCHED_MERGE, TS_SCHED_MERGE};

// AUTO sorts a batch of at most this many tiles of up to 4096 keys with SPLIT: eight
// waves per tile finish one tile sooner than one wave running a network, while large
// batches are throughput-bound and take the tuned plan (tuning knob "sort_small_batch").
int64_t g_sort_small_batch = 1024;

int resolve_sort_sched(uint32_t flags, int64_t max_len, int64_t num_tiles) {
    const int s = sched_of(flags);
    if (s != TS_SCHED_AUTO) return s;
    if (max_len <= 4096) return num_tiles <= g_sort_small_batch ? TS_SCHED_SPLIT : g_sort_plan[0];
    if (max_len <= 8192) return g_sort_plan[1];
    if (max_len <= 16384) return g_sort_plan[2];
    return TS_SCHED_MERGE;
}

int bits_for(uint32_t classes) {
    int b = 0;
    while ((1u << b) < classes) ++b;
    return b;
}

ts_status check_common(const int64_t* offsets, int64_t num_tiles, int64_t max_len,
                       void* workspace, size_t ws_bytes) {
    if (num_tiles < 0) return fail(TS_ERR_INVALID, "num_tiles < 0");
    if (num_tiles > 0 && offsets == nullptr) return fail(TS_ERR_INVALID, "tile_offsets is NULL");
    if (max_len < 0) return fail(TS_ERR_INVALID, "max_tile_len < 0");
    if (workspace == nullptr) return fail(TS_ERR_WORKSPACE, "workspace is NULL");
    if (ws_bytes < kWorkspaceBytes)
        return fail(TS_ERR_WORKSPACE, "workspace too small (%zu < %zu bytes)", ws_bytes, kWorkspaceBytes);
    return TS_OK;
}

ts_status check_payload(const uint32_t* in, const uint32_t* out, uint32_t channels, int64_t es,
                        int64_t cs, bool need_out) {
    if (channels == 0) return TS_OK;
    if (in == nullptr) return fail(TS_ERR_INVALID, "payload_in is NULL with channels > 0");
    if (need_out && out == nullptr) return fail(TS_ERR_INVALID, "payload_out is NULL with channels > 0");
    if (es < 0 || cs < 0) return fail(TS_ERR_INVALID, "negative payload stride");
    if (channels > 1 && cs == 0) return fail(TS_ERR_INVALID, "chan_stride == 0 with channels > 1");
    if (in == out) return fail(TS_ERR_INVALID, "payload_in and payload_out alias");
    return TS_OK;
}

}  // namespace

namespace ts {

int set_error(int st, const char* msg) {
    g_last_error = msg;
    return st;
}

int num_cus() {
    static int cus = [] {
        int dev = 0, v = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
            v = 256;
        return v;
    }();
    return cus;
}

int persistent_grid(const void* kernel, int block_threads, size_t dyn_lds, int64_t work) {
    static std::mutex mu;
    static std::unordered_map<const void*, int> cache;
    int per_cu = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(kernel);
        if (it == cache.end()) {
            int b = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kernel, block_threads, dyn_lds) != hipSuccess || b <= 0)
                b = 1;
            cache[kernel] = b;
            per_cu = b;
        } else {
            per_cu = it->second;
        }
    }
    int64_t g = (int64_t)per_cu * num_cus();
    if (work < g) g = work;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace ts

extern "C" {

const char* ts_last_error(void) { return g_last_error.c_str(); }

const char* ts_version(void) { return "tilesort 0.1 (gfx950)"; }

size_t ts_workspace_bytes(int op, uint32_t flags, int64_t num_tiles, int64_t total_len,
                          int64_t max_tile_len, uint32_t channels) {
    if (op == TS_OP_DEVICE_SORT)
        return total_len > 0 ? ts::device_sort_layout(total_len, ts::radix_tile(channels > 0), channels > 0).total
                             : kWorkspaceBytes;
    if (op == TS_OP_DEVICE_PARTITION)
        // the count tables of the smaller tiles: enough for either tile size
        return total_len > 0 ? ts::device_sort_layout(total_len, ts::RADIX_TILE_KEYS, false, false).total
                             : kWorkspaceBytes;
    if (op != TS_OP_SORT || num_tiles <= 0 || total_len < 0) return kWorkspaceBytes;
    const int sched = resolve_sort_sched(flags, max_tile_len, num_tiles);
    if (sched == TS_SCHED_MERGE) return ts::merge_layout(num_tiles, total_len, max_tile_len).total;
    // a payload without perm_out keeps the permutation in the workspace
    if (channels > 0) return kWorkspaceBytes + (size_t)total_len * 4u;
    return kWorkspaceBytes;
}

ts_status ts_workspace_init(void* workspace, size_t workspace_bytes, void* stream) {
    if (workspace == nullptr) return fail(TS_ERR_WORKSPACE, "workspace is NULL");
    return hip_status(ts::launch_fill_zero(workspace, workspace_bytes, (hipStream_t)stream),
                      "workspace init");
}

ts_status ts_check(void* workspace, void* stream) {
    if (workspace == nullptr) return fail(TS_ERR_WORKSPACE, "workspace is NULL");
    uint32_t word = 0;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(&word, workspace, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_status(e, "ts_check");
    if (word == 0) return TS_OK;
    e = ts::launch_fill_zero(workspace, 4, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    std::string msg;
    if (word & ts::ERR_TILE_TOO_LONG) msg += "a tile was longer than the kernel capacity (skipped); ";
    if (word & ts::ERR_BAD_LABEL) msg += "label >= num_classes; ";
    if (word & ts::ERR_BAD_PERM) msg += "pi is not a permutation of its tile; ";
    if (word & ts::ERR_BAD_OFFSETS) msg += "a tile lies outside [0, total_len) (skipped); ";
    return fail(TS_ERR_INVALID, "device reported: %s", msg.c_str());
}

// Partition as the sorting of labels (the abstract's definition) with a sort schedule:
// Theorem 2 (THM2, tiles up to 16384) or the bitonic network (BITONIC, up to 4096).
// The composites carry the position, so the order inside a class is the input order,
// as for the split schedule.  Every payload channel is gathered in the sort kernel's
// store through the source positions, so no permutation is kept between launches and
// the call needs no workspace beyond the error word.
ts_status partition_by_sort(const uint32_t* labels_in, uint32_t* labels_out,
                            const uint32_t* payload_in, uint32_t* payload_out, uint32_t channels,
                            int64_t elem_stride, int64_t chan_stride, uint32_t num_classes,
                            int32_t* perm_out, const int64_t* tile_offsets, int64_t num_tiles,
                            int64_t max_tile_len, uint32_t flags, void* workspace, void* stream) {
    const int sched = sched_of(flags);
    if (max_tile_len > ts::sort_capacity(sched))
        return fail(TS_ERR_UNSUPPORTED, "tile_partition: max_tile_len %lld > %lld for this schedule",
                    (long long)max_tile_len, (long long)ts::sort_capacity(sched));
    if (num_tiles == 0) return TS_OK;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (flags & TS_FLAG_VALIDATE) {
        e = ts::launch_label_check(labels_in, tile_offsets, num_tiles, num_classes,
                                   (uint32_t*)workspace, s);
        if (e != hipSuccess) return hip_status(e, "tile_partition label check");
    }
    ts::SortArgs a{};
    a.keys_in = labels_in;
    a.keys_out = labels_out;
    a.pay = ts::PayloadRef{payload_in, payload_out, channels, elem_stride, chan_stride};
    a.perm_out = perm_out;
    a.offsets = tile_offsets;
    a.num_tiles = num_tiles;
    a.err = (uint32_t*)workspace;
    a.fuse_pay = channels > 0 ? 1u : 0u;
    e = ts::launch_sort(a, max_tile_len, sched, s);
    return hip_status(e, "tile_partition launch");
}

ts_status tile_partition(const uint32_t* labels_in, uint32_t* labels_out,
                         const uint32_t* payload_in, uint32_t* payload_out, uint32_t channels,
                         int64_t elem_stride, int64_t chan_stride, uint32_t num_classes,
                         int32_t* perm_out, const int64_t* tile_offsets, int64_t num_tiles,
                         int64_t max_tile_len, uint32_t flags, void* workspace,
                         size_t workspace_bytes, void* stream) {
    ts_status st = check_common(tile_offsets, num_tiles, max_tile_len, workspace, workspace_bytes);
    if (st != TS_OK) return st;
    if (num_classes < 1 || num_classes > 64)
        return fail(TS_ERR_INVALID, "num_classes must be in [1, 64] (got %u)", num_classes);
    if (num_tiles > 0 && labels_in == nullptr) return fail(TS_ERR_INVALID, "labels_in is NULL");
    if (labels_in != nullptr && labels_in == labels_out)
        return fail(TS_ERR_INVALID, "labels_in and labels_out alias");
    st = check_payload(payload_in, payload_out, channels, elem_stride, chan_stride, true);
    if (st != TS_OK) return st;
    const int sched = sched_of(flags);
    if (sched == TS_SCHED_THM2 || sched == TS_SCHED_BITONIC)
        return partition_by_sort(labels_in, labels_out, payload_in, payload_out, channels, elem_stride,
                                 chan_stride, num_classes, perm_out, tile_offsets, num_tiles,
                                 max_tile_len, flags, workspace, stream);
    if (sched == TS_SCHED_NAIVE && channels > 1)
        return fail(TS_ERR_UNSUPPORTED, "tile_partition: the naive schedule moves one payload channel (got %u)",
                    channels);
    if (max_tile_len > ts::partition_split_capacity())
        return fail(TS_ERR_UNSUPPORTED, "tile_partition: max_tile_len %lld > %lld",
                    (long long)max_tile_len, (long long)ts::partition_split_capacity());
    // the kernels address one tile of the payload through a 32-bit byte range
    if (channels > 0 && (uint64_t)max_tile_len * (uint64_t)elem_stride * 4u >= (1ull << 32))
        return fail(TS_ERR_UNSUPPORTED, "tile_partition: max_tile_len x elem_stride too large");
    ts::PartitionArgs a{};
    a.labels_in = labels_in;
    a.labels_out = labels_out;
    a.pay = ts::PayloadRef{payload_in, payload_out, channels, elem_stride, chan_stride};
    a.perm_out = perm_out;
    a.offsets = tile_offsets;
    a.num_tiles = num_tiles;
    a.num_classes = num_classes;
    a.nbits = bits_for(num_classes);
    a.validate = (flags & TS_FLAG_VALIDATE) ? 1u : 0u;
    a.err = (uint32_t*)workspace;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    switch (sched) {
        case TS_SCHED_AUTO:
        case TS_SCHED_SPLIT: e = ts::launch_partition_split(a, max_tile_len, s); break;
        case TS_SCHED_NAIVE:
            // the baseline kernel has no checks of its own
            e = a.validate ? ts::launch_label_check(labels_in, tile_offsets, num_tiles, num_classes,
                                                    a.err, s)
                           : hipSuccess;
            if (e == hipSuccess) e = ts::launch_partition_naive(a, max_tile_len, s);
            break;
        default: return fail(TS_ERR_UNSUPPORTED, "tile_partition: schedule %d not available", sched);
    }
    return hip_status(e, "tile_partition launch");
}

ts_status tile_permute(const uint32_t* in, uint32_t* out, uint32_t channels, int64_t elem_stride,
                       int64_t chan_stride, const uint32_t* aux_in, uint32_t* aux_out, const int32_t* pi,
                       uint32_t direction, int32_t* inv_out,
                       const int64_t* tile_offsets, int64_t num_tiles, int64_t max_tile_len,
                       uint32_t flags, void* workspace, size_t workspace_bytes, void* stream) {
    ts_status st = check_common(tile_offsets, num_tiles, max_tile_len, workspace, workspace_bytes);
    if (st != TS_OK) return st;
    if (direction != TS_SCATTER && direction != TS_GATHER)
        return fail(TS_ERR_INVALID, "tile_permute: direction must be TS_SCATTER or TS_GATHER");
    if (num_tiles > 0 && pi == nullptr) return fail(TS_ERR_INVALID, "tile_permute: pi is NULL");
    if ((aux_in == nullptr) != (aux_out == nullptr))
        return fail(TS_ERR_INVALID, "tile_permute: aux_in and aux_out must both be given");
    if (aux_in != nullptr && (const void*)aux_in == (const void*)aux_out)
        return fail(TS_ERR_INVALID, "tile_permute: aux_in and aux_out alias");
    if (aux_in != nullptr && sched_of(flags) == TS_SCHED_NAIVE)
        return fail(TS_ERR_UNSUPPORTED, "tile_permute: the naive schedule has no aux channel");
    if (channels == 0 && aux_in == nullptr && inv_out == nullptr) return TS_OK;
    if (channels > 0) {
        if (in == nullptr || out == nullptr) return fail(TS_ERR_INVALID, "tile_permute: in/out is NULL");
        st = check_payload(in, out, channels, elem_stride, chan_stride, true);
        if (st != TS_OK) return st;
    }
    if (inv_out != nullptr && ((const void*)inv_out == (const void*)pi ||
                               (const void*)inv_out == (const void*)in))
        return fail(TS_ERR_INVALID, "tile_permute: inv_out aliases pi or in");
    if (max_tile_len > ts::permute_split_capacity())
        return fail(TS_ERR_UNSUPPORTED, "tile_permute: max_tile_len %lld > %lld",
                    (long long)max_tile_len, (long long)ts::permute_split_capacity());
    // the kernels address one tile of a payload channel through a 32-bit byte range
    if (channels > 0 && (uint64_t)max_tile_len * (uint64_t)elem_stride * 4u >= (1ull << 32))
        return fail(TS_ERR_UNSUPPORTED, "tile_permute: max_tile_len x elem_stride too large");
    ts::PermuteArgs a{};
    a.pay = ts::PayloadRef{in, out, channels, elem_stride, chan_stride};
    a.aux = ts::PayloadRef{aux_in, aux_out, aux_in != nullptr ? 1u : 0u, 1, 0};
    a.pi = pi;
    a.direction = direction;
    a.inv_out = inv_out;
    a.offsets = tile_offsets;
    a.num_tiles = num_tiles;
    a.validate = (flags & TS_FLAG_VALIDATE) ? 1u : 0u;
    a.pi16 = (flags & TS_FLAG_PI_U16) ? 1u : 0u;
    a.inv16 = (flags & TS_FLAG_INV_U16) ? 1u : 0u;
    a.err = (uint32_t*)workspace;
    hipStream_t s = (hipStream_t)stream;
    const int sched = sched_of(flags);
    hipError_t e;
    switch (sched) {
        case TS_SCHED_AUTO:
        case TS_SCHED_SPLIT: e = ts::launch_permute_split(a, max_tile_len, s); break;
        case TS_SCHED_NAIVE: e = ts::launch_permute_naive(a, max_tile_len, s); break;
        default: return fail(TS_ERR_UNSUPPORTED, "tile_permute: schedule %d not available", sched);
    }
    return hip_status(e, "tile_permute launch");
}

ts_status tile_sort(const uint32_t* keys_in, uint32_t* keys_out, const uint32_t* payload_in,
                    uint32_t* payload_out, uint32_t channels, int64_t elem_stride,
                    int64_t chan_stride, int32_t* perm_out, const int64_t* tile_offsets,
                    int64_t num_tiles, int64_t total_len, int64_t max_tile_len, uint32_t flags,
                    void* workspace, size_t workspace_bytes, void* stream) {
    ts_status st = check_common(tile_offsets, num_tiles, max_tile_len, workspace, workspace_bytes);
    if (st != TS_OK) return st;
    if (total_len < 0) return fail(TS_ERR_INVALID, "tile_sort: total_len < 0");
    if (num_tiles > 0 && keys_in == nullptr) return fail(TS_ERR_INVALID, "tile_sort: keys_in is NULL");
    if (keys_in != nullptr && keys_in == keys_out)
        return fail(TS_ERR_INVALID, "tile_sort: keys_in and keys_out alias");
    st = check_payload(payload_in, payload_out, channels, elem_stride, chan_stride, true);
    if (st != TS_OK) return st;
    const int sched = resolve_sort_sched(flags, max_tile_len, num_tiles);
    if (sched != TS_SCHED_SPLIT && sched != TS_SCHED_THM2 && sched != TS_SCHED_BITONIC &&
        sched != TS_SCHED_MERGE && sched != TS_SCHED_NAIVE)
        return fail(TS_ERR_UNSUPPORTED, "tile_sort: schedule %d not available", sched);
    const int64_t cap = (sched == TS_SCHED_NAIVE)   ? 16384
                        : (sched == TS_SCHED_MERGE) ? ts::MERGE_MAX_TILE
                                                    : ts::sort_capacity(sched);
    if (max_tile_len > cap)
        return fail(TS_ERR_UNSUPPORTED, "tile_sort: max_tile_len %lld > %lld for this schedule",
                    (long long)max_tile_len, (long long)cap);
    if (num_tiles == 0) return TS_OK;
    ts::SortArgs a{};
    a.keys_in = keys_in;
    a.keys_out = keys_out;
    a.pay = ts::PayloadRef{payload_in, payload_out, channels, elem_stride, chan_stride};
    a.perm_out = perm_out;
    a.offsets = tile_offsets;
    a.num_tiles = num_tiles;
    a.f32 = (flags & TS_FLAG_F32_ORDERED) ? 1u : 0u;
    a.err = (uint32_t*)workspace;
    hipStream_t s = (hipStream_t)stream;
    if (sched == TS_SCHED_MERGE) {
        // pieces, merge rounds and the payload gather, all inside the workspace
        const size_t need = ts::merge_layout(num_tiles, total_len, max_tile_len).total;
        if (workspace_bytes < need)
            return fail(TS_ERR_WORKSPACE, "tile_sort: the merge schedule needs %zu workspace bytes (got %zu)",
                        need, workspace_bytes);
        return hip_status(ts::launch_sort_merge(a, total_len, max_tile_len, workspace, s),
                          "tile_sort launch");
    }
    // A small batch sorted by the split schedule gathers the payload in the sort
    // kernel's store (a global gather inside each tile), sparing the second launch.
    a.fuse_pay = (channels > 0 && sched == TS_SCHED_SPLIT && num_tiles <= g_sort_small_batch) ? 1u : 0u;
    // Otherwise the payload follows in a second launch: a gather by the permutation (a
    // conflict-free routing per tile; a direct LDS gather for the baseline), which keeps
    // the permutation in the workspace after its 256-byte header when perm_out is NULL.
    // (Writing the inverse from the sort's store and scattering by it routes once
    // instead of twice, but the scattered 4-byte stores of the inverse cost more than
    // the routing they save: measured on 4096 x 16384 keys with 8 channels.)
    const bool second = channels > 0 && !a.fuse_pay;
    if (second && a.perm_out == nullptr) {
        const size_t need = kWorkspaceBytes + (size_t)total_len * 4u;
        if (workspace_bytes < need)
            return fail(TS_ERR_WORKSPACE, "tile_sort: a payload without perm_out needs %zu workspace bytes", need);
        a.perm_out = (int32_t*)((char*)workspace + kWorkspaceBytes);
    }
    hipError_t e = (sched == TS_SCHED_NAIVE) ? ts::launch_sort_naive(a, max_tile_len, s)
                                             : ts::launch_sort(a, max_tile_len, sched, s);
    if (e != hipSuccess) return hip_status(e, "tile_sort launch");
    if (second) {
        ts::PermuteArgs p{};
        p.pay = a.pay;
        p.pi = a.perm_out;
        p.direction = TS_GATHER;
        p.offsets = tile_offsets;
        p.num_tiles = num_tiles;
        p.err = a.err;
        e = (sched == TS_SCHED_NAIVE) ? ts::launch_permute_naive(p, max_tile_len, s)
                                      : ts::launch_permute_split(p, max_tile_len < 4096 ? 4096 : max_tile_len, s);
        if (e != hipSuccess) return hip_status(e, "tile_sort payload gather launch");
    }
    return TS_OK;
}

ts_status ts_tune(const char* knob, int value) {
    if (knob == nullptr) return fail(TS_ERR_INVALID, "ts_tune: knob is NULL");
    if (std::strcmp(knob, "partition_waves_4096") == 0) {
        static const int ok[] = {1, 2, 4, 8, 16, 104, 106, 108, 164, 166, 168, 176};
        bool found = false;
        for (int v : ok) found |= (v == value);
        if (!found)
            return fail(TS_ERR_INVALID, "ts_tune: partition_waves_4096 must be one of 1, 2, 4, 8, 16, 104, 106, 108, 164, 166, 168, 176");
        ts::set_partition_waves(value);
        return TS_OK;
    }
    if (std::strcmp(knob, "oneshot") == 0) {
        if (value < 0 || value > 1) return fail(TS_ERR_INVALID, "ts_tune: oneshot must be 0 or 1");
        ts::set_oneshot(value);
        return TS_OK;
    }
    if (std::strcmp(knob, "naive_oneshot") == 0) {
        if (value < 0 || value > 1) return fail(TS_ERR_INVALID, "ts_tune: naive_oneshot must be 0 or 1");
        ts::set_naive_oneshot(value);
        return TS_OK;
    }
    if (std::strcmp(knob, "permute_variant") == 0) {
        if (!(value == 0 || value == 1 || value == 2 || (value >= 6 && value <= 13)))
            return fail(TS_ERR_INVALID, "ts_tune: permute_variant must be one of 0, 1, 2, 6 .. 13");
        ts::set_permute_variant(value);
        return TS_OK;
    }
    if (std::strcmp(knob, "sort_small_batch") == 0) {
        if (value < 0) return fail(TS_ERR_INVALID, "ts_tune: sort_small_batch must be >= 0");
        g_sort_small_batch = value;
        return TS_OK;
    }
    if (std::strcmp(knob, "merge_wide") == 0) {
        if (value != 4096 && value != 8192 && value != 16384 && value != 32768)
            return fail(TS_ERR_INVALID, "ts_tune: merge_wide must be 4096, 8192, 16384 or 32768");
        ts::set_merge_wide(value);
        return TS_OK;
    }
    if (std::strcmp(knob, "merge_pack") == 0) {
        if (value != 0 && value != 1) return fail(TS_ERR_INVALID, "ts_tune: merge_pack must be 0 or 1");
        ts::set_merge_pack(value);
        return TS_OK;
    }
    static const char* plans[3] = {"sort_plan_4096", "sort_plan_8192", "sort_plan_16384"};
    for (int i = 0; i < 3; ++i) {
        if (std::strcmp(knob, plans[i]) != 0) continue;
        const bool ok = value == TS_SCHED_SPLIT || value == TS_SCHED_MERGE || value == TS_SCHED_NAIVE ||
                        value == TS_SCHED_THM2 || value == TS_SCHED_BITONIC;
        if (!ok) return fail(TS_ERR_INVALID, "ts_tune: %s: schedule %d cannot sort such tiles", knob, value);
        g_sort_plan[i] = value;
        return TS_OK;
    }
    return fail(TS_ERR_INVALID, "ts_tune: unknown knob '%s'", knob);
}

ts_status ts_device_sort(const uint32_t* keys_in, uint32_t* keys_out, const uint32_t* payload_in,
                         uint32_t* payload_out, int32_t* perm_out, int64_t n, uint32_t flags,
                         void* workspace, size_t workspace_bytes, void* stream) {
    if (n < 0) return fail(TS_ERR_INVALID, "ts_device_sort: n < 0");
    if (n > INT32_MAX) return fail(TS_ERR_UNSUPPORTED, "ts_device_sort: n >= 2^31");
    if (workspace == nullptr) return fail(TS_ERR_WORKSPACE, "workspace is NULL");
    if (n == 0) return TS_OK;
    if (keys_in == nullptr || keys_out == nullptr) return fail(TS_ERR_INVALID, "ts_device_sort: keys are NULL");
    if (keys_in == keys_out) return fail(TS_ERR_INVALID, "ts_device_sort: keys_in and keys_out alias");
    if ((payload_in == nullptr) != (payload_out == nullptr))
        return fail(TS_ERR_INVALID, "ts_device_sort: payload_in and payload_out must both be given");
    if (payload_in != nullptr && payload_in == payload_out)
        return fail(TS_ERR_INVALID, "ts_device_sort: payload_in and payload_out alias");
    if (payload_in != nullptr && perm_out != nullptr)
        return fail(TS_ERR_UNSUPPORTED, "ts_device_sort: a payload and perm_out together");
    const bool carry = payload_in != nullptr || perm_out != nullptr;
    const size_t need = ts::device_sort_layout(n, ts::radix_tile(carry), carry).total;
    if (workspace_bytes < need)
        return fail(TS_ERR_WORKSPACE, "ts_device_sort needs %zu workspace bytes (got %zu)", need, workspace_bytes);
    ts::DeviceSortArgs d{};
    d.keys_in = keys_in;
    d.keys_out = keys_out;
    d.pay_in = payload_in;
    d.pay_out = payload_out;
    d.perm_out = perm_out;
    d.n = n;
    d.f32 = (flags & TS_FLAG_F32_ORDERED) ? 1u : 0u;
    d.err = (uint32_t*)workspace;
    return hip_status(ts::launch_device_sort(d, workspace, (hipStream_t)stream), "ts_device_sort launch");
}

ts_status ts_device_partition(const uint32_t* labels_in, uint32_t* labels_out,
                              const uint32_t* payload_in, uint32_t* payload_out, int32_t* perm_out,
                              int64_t n, uint32_t num_classes, uint32_t flags, void* workspace,
                              size_t workspace_bytes, void* stream) {
    if (n < 0) return fail(TS_ERR_INVALID, "ts_device_partition: n < 0");
    if (n > INT32_MAX) return fail(TS_ERR_UNSUPPORTED, "ts_device_partition: n >= 2^31");
    if (num_classes < 1 || num_classes > 64)
        return fail(TS_ERR_INVALID, "ts_device_partition: num_classes must be in [1, 64]");
    if (workspace == nullptr) return fail(TS_ERR_WORKSPACE, "workspace is NULL");
    if (n == 0) return TS_OK;
    if (labels_in == nullptr || labels_out == nullptr)
        return fail(TS_ERR_INVALID, "ts_device_partition: labels are NULL");
    if (labels_in == labels_out) return fail(TS_ERR_INVALID, "ts_device_partition: labels_in and labels_out alias");
    if ((payload_in == nullptr) != (payload_out == nullptr))
        return fail(TS_ERR_INVALID, "ts_device_partition: payload_in and payload_out must both be given");
    if (payload_in != nullptr && payload_in == payload_out)
        return fail(TS_ERR_INVALID, "ts_device_partition: payload_in and payload_out alias");
    if (payload_in != nullptr && perm_out != nullptr)
        return fail(TS_ERR_UNSUPPORTED, "ts_device_partition: a payload and perm_out together");
    const size_t need = ts::device_sort_layout(n, ts::RADIX_TILE_KEYS, false, false).total;
    if (workspace_bytes < need)
        return fail(TS_ERR_WORKSPACE, "ts_device_partition needs %zu workspace bytes (got %zu)", need,
                    workspace_bytes);
    int nbits = 0;
    while ((1u << nbits) < num_classes) ++nbits;
    ts::DeviceSortArgs d{};
    d.keys_in = labels_in;
    d.keys_out = labels_out;
    d.pay_in = payload_in;
    d.pay_out = payload_out;
    d.perm_out = perm_out;
    d.n = n;
    d.err = (uint32_t*)workspace;
    return hip_status(ts::launch_device_partition(d, nbits, num_classes, (flags & TS_FLAG_VALIDATE) != 0,
                                                  workspace, (hipStream_t)stream),
                      "ts_device_partition launch");
}

ts_status ts_copy(const void* src, void* dst, size_t bytes, void* stream) {
    if (bytes == 0) return TS_OK;
    if (src == nullptr || dst == nullptr) return fail(TS_ERR_INVALID, "ts_copy: NULL pointer");
    if (((uintptr_t)src | (uintptr_t)dst) & 15u)
        return fail(TS_ERR_INVALID, "ts_copy: src and dst must be 16-byte aligned");
    return hip_status(ts::launch_copy(src, dst, bytes, (hipStream_t)stream), "ts_copy launch");
}

ts_status ts_lds_probe(const uint32_t* lane_words, int op, int width, int iters, int waves,
                       int groups, uint64_t* cycles_out, uint32_t* sink, void* stream) {
    if (lane_words == nullptr || cycles_out == nullptr || sink == nullptr)
        return fail(TS_ERR_INVALID, "ts_lds_probe: NULL pointer");
    if (op < 0 || op > 2) return fail(TS_ERR_INVALID, "ts_lds_probe: op must be 0, 1 or 2");
    if (!(width == 1 || width == 2 || width == 4) || (op == 2 && width != 1))
        return fail(TS_ERR_INVALID, "ts_lds_probe: bad width");
    if (iters < 1 || waves < 1 || waves > 16 || groups < 1)
        return fail(TS_ERR_INVALID, "ts_lds_probe: bad iters/waves/groups");
    return hip_status(ts::launch_lds_probe(lane_words, op, width, iters, waves, groups, cycles_out,
                                           sink, (hipStream_t)stream),
                      "ts_lds_probe launch");
}

}  // extern "C"
