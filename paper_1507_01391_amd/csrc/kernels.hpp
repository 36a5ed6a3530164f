// Internal launch interface between the C ABI layer (api.cpp) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ts {

// Bits of the workspace error word (the TS_ERRBIT_* values of tilesort.h).
enum : uint32_t {
    ERR_TILE_TOO_LONG = 1u,   // a tile exceeded the kernel's capacity and was skipped
    ERR_BAD_LABEL = 2u,       // TS_FLAG_VALIDATE: label >= num_classes
    ERR_BAD_PERM = 4u,        // TS_FLAG_VALIDATE: pi is not a permutation of its tile
    ERR_BAD_OFFSETS = 8u,     // a tile outside [0, total_len) (skipped)
};


struct PayloadRef {
    const uint32_t* in;
    uint32_t* out;
    uint32_t channels;
    int64_t es;  // element stride (words)
    int64_t cs;  // channel stride (words)
};

struct PartitionArgs {
    const uint32_t* labels_in;
    uint32_t* labels_out;
    PayloadRef pay;
    int32_t* perm_out;
    const int64_t* offsets;
    int64_t num_tiles;
    uint32_t num_classes;
    int nbits;          // ceil(log2(num_classes))
    uint32_t validate;  // nonzero: check labels
    uint32_t* err;      // workspace error word
};

struct PermuteArgs {
    PayloadRef pay;     // in / out with channels and strides
    PayloadRef aux;     // optional extra channel (unit stride) moved first by the same routing
    const int32_t* pi;
    uint32_t direction;
    int32_t* inv_out;   // optional: receives pi^-1 (inv_out[pi[i]] = i)
    const int64_t* offsets;
    int64_t num_tiles;
    uint32_t validate;
    uint32_t pi16;      // pi holds uint16 values
    uint32_t inv16;     // inv_out receives uint16 values
    uint32_t* err;
};

struct SortArgs {
    const uint32_t* keys_in;
    uint32_t* keys_out;
    PayloadRef pay;
    int32_t* perm_out;
    const int64_t* offsets;
    int64_t num_tiles;
    uint32_t f32;       // nonzero: keys are binary32 patterns
    uint32_t* err;
    uint32_t fuse_pay;  // split schedule: gather the payload in the sort kernel's store
};

// One pass of the device-wide radix sort (device_sort.hip): tiles of 4096 items split
// on the digit bits shift .. shift + nbits - 1 and stored by digit block at goff.
struct RadixPass {
    const uint32_t* keys_in;
    uint32_t* keys_out;
    const uint32_t* pay_in;     // or NULL
    uint32_t* pay_out;          // or NULL
    const int64_t* offsets;     // num_tiles + 1 tile boundaries
    int64_t num_tiles;
    int shift, nbits;
    uint32_t f32_in, f32_out;   // map binary32 keys on load / back on store
    const uint32_t* hist;
    const uint32_t* goff;
    int64_t n_total;
    uint32_t* err;
    int tile;                   // RADIX_TILE_KEYS or RADIX_TILE_PAY
};
hipError_t launch_radix_pass(const RadixPass& r, hipStream_t s);
// Items per tile of a radix pass.  With a payload word (or the index) travelling, 8192:
// a digit's block of a tile holds 128 items on average and the scattered stores run
// faster (measured 7 % on the whole sort); keys alone keep 4096, where the pass is
// bound by its LDS splits and four resident tiles per CU beat two.
constexpr int RADIX_TILE_KEYS = 4096;
constexpr int RADIX_TILE_PAY = 8192;
constexpr int radix_tile(bool with_pay) { return with_pay ? RADIX_TILE_PAY : RADIX_TILE_KEYS; }
// Bits per pass (the last pass takes what is left): six passes sort 32-bit keys.  Six
// bits keep a digit's block of a 4096-item tile at 64 items on average; with 8-bit
// digits the 16-item blocks make the scattered stores 2.4x slower per pass.
constexpr int RADIX_BITS = 6;
constexpr int RADIX_DIGITS = 1 << RADIX_BITS;     // rows of the per-tile count tables
constexpr int RADIX_PASSES = (32 + RADIX_BITS - 1) / RADIX_BITS;

struct DeviceSortArgs {
    const uint32_t* keys_in;
    uint32_t* keys_out;
    const uint32_t* pay_in;     // one payload word per key, or NULL
    uint32_t* pay_out;
    int32_t* perm_out;          // or NULL; not together with a payload
    int64_t n;
    uint32_t f32;
    uint32_t* err;
};
struct DeviceSortLayout {
    size_t offsets, hist, goff, bsum, keys, pay, total;
};
// with_pay: a payload word travels; pingpong: room for a second copy of the data (the
// sort's passes alternate between it and the output; a single partition pass needs none)
// tile: items per tile of the passes (radix_tile)
DeviceSortLayout device_sort_layout(int64_t n, int tile, bool with_pay, bool pingpong = true);
hipError_t launch_device_sort(const DeviceSortArgs& d, void* ws, hipStream_t s);
// One pass on the low `nbits` bits of the labels; with `validate`, labels >= num_classes
// set ERR_BAD_LABEL.
hipError_t launch_device_partition(const DeviceSortArgs& d, int nbits, uint32_t num_classes,
                                   bool validate, void* ws, hipStream_t s);

// Sorting tiles of uneven length by pieces and merges (merge.hip).
constexpr int MERGE_PIECE = 4096;          // keys per wavefront work item
constexpr int MERGE_POS_BITS = 28;         // tile positions fit in 28 bits
constexpr int64_t MERGE_MAX_TILE = int64_t(1) << MERGE_POS_BITS;
constexpr int MERGE_MAX_ROUNDS = 16;       // log2(MERGE_MAX_TILE / MERGE_PIECE)
constexpr int MERGE_COUNTER_WORD = 16;     // first counter word in the workspace header
constexpr int MERGE_COUNTER_BYTES = 96;    // words 16 .. 39: bins 0 .. 3, pieces, bins 4 .. 6,
                                           // rounds 0 .. 15 at 8 + r

// Byte offsets of the regions a merge-schedule sort carves out of the workspace.
struct MergeLayout {
    int64_t cap;       // entries per piece list and per round list
    int rounds;        // merge rounds provisioned (0 when max_len <= MERGE_PIECE)
    size_t bins, pieces, round_lists, coranks, run0, run1, total;
};
MergeLayout merge_layout(int64_t num_tiles, int64_t total_len, int64_t max_len);

struct MergeArgs {
    SortArgs s;
    uint32_t* counters;      // MERGE_COUNTER_BYTES, zeroed by the launcher
    uint64_t* bins;          // 7 lists of num_tiles entries (tile << 16)
    uint64_t* pieces;        // cap entries (tile << 16 | piece)
    uint64_t* round_lists;   // rounds x cap entries (tile << 16 | output piece)
    int32_t* coranks;        // rounds x cap x 2
    uint64_t* run0;          // total_len composites
    uint64_t* run1;          // total_len composites (only when rounds >= 2)
    int64_t cap;
    int rounds;
    int pack;                // nonzero: up to 8 short tiles share one wavefront
    int64_t wide_max;        // tiles of up to this many keys are sorted whole by one workgroup
    int64_t max_len;
    int64_t total_len;       // keys of all tiles; every tile must lie in [0, total_len)
};
hipError_t launch_sort_merge(const SortArgs& s, int64_t total_len, int64_t max_len, void* ws,
                             hipStream_t st);
void set_merge_pack(int v);
void set_merge_wide(int v);

// Device properties cached by the API layer.
int num_cus();
// Record `msg` as the thread's last error message and return st (a ts_status).
int set_error(int st, const char* msg);

// Each returns hipSuccess or the launch error.  `cap` is the kernel's tile capacity.
hipError_t launch_partition_split(const PartitionArgs& a, int64_t max_len, hipStream_t s);
hipError_t launch_partition_naive(const PartitionArgs& a, int64_t max_len, hipStream_t s);
// Flags labels >= num_classes (partition through the sort schedules).
hipError_t launch_label_check(const uint32_t* labels, const int64_t* offsets, int64_t num_tiles,
                              uint32_t num_classes, uint32_t* err, hipStream_t s);
hipError_t launch_permute_split(const PermuteArgs& a, int64_t max_len, hipStream_t s);
hipError_t launch_permute_naive(const PermuteArgs& a, int64_t max_len, hipStream_t s);
hipError_t launch_sort(const SortArgs& a, int64_t max_len, int sched, hipStream_t s);
hipError_t launch_sort_split(const SortArgs& a, int64_t max_len, hipStream_t s);
hipError_t launch_sort_naive(const SortArgs& a, int64_t max_len, hipStream_t s);

int64_t partition_split_capacity();
void set_partition_waves(int nw);
void set_permute_variant(int v);
int64_t permute_split_capacity();
int64_t sort_capacity(int sched);

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s);
hipError_t launch_lds_probe(const uint32_t* lane_words, int op, int width, int iters, int waves,
                            int groups, uint64_t* cycles_out, uint32_t* sink, hipStream_t s);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);

// Grid size for a persistent kernel: min(work items, resident blocks on the device).
int persistent_grid(const void* kernel, int block_threads, size_t dyn_lds, int64_t work);
void set_naive_oneshot(int v);
void set_oneshot(int v);
bool tile_oneshot();

}  // namespace ts
