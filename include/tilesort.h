/*
 * tilesort.h -- C interface of libtilesort.so: sorting, w-way partitioning
 * and permuting tiles of 32-bit items in one workgroup's LDS on MI355X
 * (gfx950) without LDS bank conflicts.
 *
 * The three problems are those of Afshani & Sitchinava, "Sorting and
 * Permuting without Bank Conflicts on GPUs", Sec. 1 ("Problems of interest"):
 * sorting, w-way partition (the abstract defines it as sorting an input with
 * n/w copies of every label) and permutation.  Shared memory is the paper's
 * w x m matrix with one row per bank (Sec. 1, "Model of Computation"); here
 * w = 64 lanes of a wavefront and the LDS banks of one CU.
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - All array pointers are DEVICE pointers (hipMalloc / torch allocations);
 *    the caller owns every buffer.  The library allocates nothing on these
 *    calls; the only scratch it uses is the caller's `workspace`.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Every call only enqueues work on that stream and returns; results are
 *    ready when the stream is.
 *  - Tiles: tile t is the item range [tile_offsets[t], tile_offsets[t+1]) of
 *    the flat arrays.  `tile_offsets` is a device int64 array of num_tiles+1
 *    non-decreasing entries, tile_offsets[0] >= 0.  `max_tile_len` is a host
 *    upper bound on every tile's length (used to pick kernels); a longer tile
 *    is skipped and flagged in the workspace error word (see ts_check).
 *  - Keys / labels / permutation entries are contiguous 32-bit arrays indexed
 *    by the global item index g.
 *  - Payload: `channels` 32-bit words per item; word (g, c) lives at
 *    payload[g * elem_stride + c * chan_stride] (units of 32-bit words).
 *    Array-of-structs is elem_stride = channels, chan_stride = 1;
 *    channel-planar is elem_stride = 1, chan_stride = total item count.
 *    Any 32-bit type (fp32, int32, uint32) is moved bit-exactly.
 *  - perm_out / pi are tile-local int32 indices.
 *  - Input and output arrays must not overlap.
 *  - Workspace: at least ts_workspace_bytes(...) bytes of device memory,
 *    prepared once with ts_workspace_init.  It holds the error word and,
 *    for some schedules, work-queue counters.  Calls that share a workspace
 *    must be ordered on one stream.
 *
 * Errors: host-detectable argument problems return TS_ERR_INVALID (or
 * TS_ERR_UNSUPPORTED for combinations not implemented) and set the message
 * returned by ts_last_error() (thread-local).  A failed kernel launch returns
 * TS_ERR_HIP.  Inputs that break the data contract (label >= num_classes,
 * pi not a permutation of its tile) never cause out-of-bounds accesses --
 * indices are masked to the tile -- but the output is unspecified; with
 * TS_FLAG_VALIDATE the kernels record such inputs in the workspace error word
 * and ts_check reports them.
 */
#ifndef TILESORT_H
#define TILESORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ts_status {
    TS_OK = 0,
    TS_ERR_INVALID = 1,
    TS_ERR_UNSUPPORTED = 2,
    TS_ERR_HIP = 3,
    TS_ERR_WORKSPACE = 4
} ts_status;

/* tile_permute directions */
enum { TS_SCATTER = 0, /* out[pi[i]] = in[i] */
       TS_GATHER = 1   /* out[i] = in[pi[i]] */ };

/* flags */
enum {
    /* keys are IEEE binary32 bit patterns: compared through the order-preserving
       map (negatives: all bits flipped; non-negatives: sign bit set), so -0 < +0;
       the original bits are written to keys_out */
    TS_FLAG_F32_ORDERED = 1u,
    /* kernels check labels / pi against the data contract and record violations
       (labels: every partition schedule; pi: the SPLIT permute schedule) */
    TS_FLAG_VALIDATE = 2u,
    /* tile_permute: pi points to uint16 values (tile-local indices fit in 16 bits
       for every supported tile length); halves the index bytes read */
    TS_FLAG_PI_U16 = 4u,
    /* tile_permute: inv_out receives uint16 values */
    TS_FLAG_INV_U16 = 8u
};

/* Schedule selection, stored in flags bits 8..11 (TS_SCHED(x) = x << 8). */
#define TS_SCHED(x) ((uint32_t)(x) << 8)
enum {
    TS_SCHED_AUTO = 0,    /* the plan chosen by the autotuner's table (default) */
    TS_SCHED_SPLIT = 1,   /* alternating-direction binary splits (partition, permute, sort) */
    TS_SCHED_THM2 = 2,    /* the paper's Theorem 2 schedule: Lemma 1 on super-rows of 8
                             rows, column sorts, row sorts (sort and partition); a 64 x m
                             tile, m = 64 in one wavefront, m = 128 / 256 spread over 2 / 4 */
    TS_SCHED_BITONIC = 3, /* Batcher's network: register stages + conflict-free transposes,
                             tiles of 8192 / 16384 over 2 / 4 wavefronts (sort, partition) */
    TS_SCHED_MERGE = 4,   /* sort of uneven tiles up to 2^28 keys: short tiles packed up to
                             eight per wavefront, tiles up to 32768 keys sorted whole by one
                             workgroup of up to 8 wavefronts, longer tiles cut into 4096-key
                             pieces sorted like BITONIC, then rounds of pairwise bitonic
                             merges (sort) */
    TS_SCHED_NAIVE = 15   /* baseline: plain LDS counting / direct scatter, with bank
                             conflicts (all three ops) */
};

/* Operation ids for ts_workspace_bytes */
enum { TS_OP_SORT = 0, TS_OP_PARTITION = 1, TS_OP_PERMUTE = 2, TS_OP_DEVICE_SORT = 3,
       TS_OP_DEVICE_PARTITION = 4 };

/*
 * tile_sort -- sorting (Sec. 1, "Problems of interest": sorting; Sec. 2, Lemma 1
 * and Theorem 2).  Every tile is sorted ascending by its uint32 key; equal keys
 * keep input order (stable), so the result is unique.
 *   keys_in / keys_out  : uint32 [N]; keys_out receives the sorted original bits.
 *   payload_in / out    : optional (channels may be 0; pointers may then be NULL);
 *                         payload_out[k] = payload_in[source of k].
 *   perm_out            : optional int32 [N]: tile-local source index of slot k.
 *   total_len           : N = tile_offsets[num_tiles], the length of the flat arrays;
 *                         every tile must lie in [0, N).  The merge schedule places its
 *                         runs in the workspace by it and skips (and flags) a tile
 *                         outside [0, N); the other schedules keep the permutation of a
 *                         payload without perm_out at workspace index = item index.
 * Supported tile length: 16384 for BITONIC, THM2, SPLIT and NAIVE, 2^28 for MERGE; a
 * longer max_tile_len returns TS_ERR_UNSUPPORTED.  AUTO takes the autotuned plan for
 * max_tile_len up to 4096 / 8192 / 16384 and MERGE beyond.
 * The workspace must hold ts_workspace_bytes(TS_OP_SORT, flags, ...) bytes: the
 * merge schedule needs about 16 bytes per key for its runs and work lists, a payload
 * without perm_out (outside the merge schedule) 4 bytes per key for the permutation.
 */
ts_status tile_sort(const uint32_t* keys_in, uint32_t* keys_out,
                    const uint32_t* payload_in, uint32_t* payload_out, uint32_t channels,
                    int64_t elem_stride, int64_t chan_stride, int32_t* perm_out,
                    const int64_t* tile_offsets, int64_t num_tiles, int64_t total_len,
                    int64_t max_tile_len, uint32_t flags, void* workspace,
                    size_t workspace_bytes, void* stream);

/*
 * tile_partition -- w-way partition (Sec. 1: an item with label i is sent to row i;
 * abstract: partitioning = sorting an input with n/w copies of each label;
 * Corollary 1 and Theorem 2 solve it in O(m) steps).  Labels are uint32 in
 * [0, num_classes), 1 <= num_classes <= 64.  Output: items grouped by label in
 * ascending label order, input order kept within a label (stable); labels_out,
 * payload_out and perm_out (optional) follow that order.
 * Schedules: SPLIT (default; tiles up to 16384), NAIVE (up to 16384, one payload
 * channel), and THM2 / BITONIC (up to 16384), which partition by sorting the labels
 * with those sort schedules.  Payload: any number of channels (SPLIT moves
 * the first with the label through LDS and gathers the others through the source
 * positions at the store; THM2 / BITONIC gather every channel that way); NAIVE with
 * channels > 1 returns TS_ERR_UNSUPPORTED.  No workspace beyond the error word
 * (ts_workspace_bytes(TS_OP_PARTITION, ...) is 256 bytes).
 */
ts_status tile_partition(const uint32_t* labels_in, uint32_t* labels_out,
                         const uint32_t* payload_in, uint32_t* payload_out, uint32_t channels,
                         int64_t elem_stride, int64_t chan_stride, uint32_t num_classes,
                         int32_t* perm_out,
                         const int64_t* tile_offsets, int64_t num_tiles, int64_t max_tile_len,
                         uint32_t flags, void* workspace, size_t workspace_bytes, void* stream);

/*
 * tile_permute -- permutation (Sec. 1: an item labelled (i, j) goes to slot j of
 * row i; here the label is the tile-local linear destination).  pi is int32 [N],
 * a permutation of [0, len) inside every tile.
 *   TS_SCATTER: out[pi[i]] = in[i];   TS_GATHER: out[i] = in[pi[i]].
 * in / out use the payload addressing above with `channels` words per item
 * (channels may be 0 when only inv_out is wanted).
 *   aux_in / aux_out : optional extra channel (uint32 [N] each, unit stride, both or
 *             neither), moved by the same routing as the payload: e.g. the gradient
 *             of the keys beside the gradients of a multi-channel payload.  Not with
 *             TS_SCHED_NAIVE (TS_ERR_UNSUPPORTED).
 *   inv_out : optional int32 [N]: receives the tile-local inverse permutation,
 *             inv_out[pi[i]] = i, computed by the same routing (no extra pass);
 *             a later GATHER by pi equals a SCATTER by inv_out, which routes once
 *             instead of twice.  Must not alias pi or in.
 * With TS_FLAG_PI_U16 pi is read as uint16 [N], with TS_FLAG_INV_U16 inv_out is
 * written as uint16 [N] (the pointers keep their declared types; cast them).
 * Supported tile length: max_tile_len <= 16384.
 */
ts_status tile_permute(const uint32_t* in, uint32_t* out, uint32_t channels,
                       int64_t elem_stride, int64_t chan_stride,
                       const uint32_t* aux_in, uint32_t* aux_out,
                       const int32_t* pi, uint32_t direction, int32_t* inv_out,
                       const int64_t* tile_offsets, int64_t num_tiles, int64_t max_tile_len,
                       uint32_t flags, void* workspace, size_t workspace_bytes, void* stream);

/*
 * ts_device_sort -- stable ascending sort of one array of n uint32 keys (the whole
 * array, not tiles), built on the conflict-free 64-way partition: an LSD radix sort
 * whose every pass partitions each tile on a 6-bit digit with the split schedule and
 * stores each digit block at its place in the array (Sec. 1: the partition step of a
 * quicksort with pivots, here with digit buckets).  Six passes.  Tiles hold 4096 keys
 * when the keys travel alone and 8192 items when a payload word or the permutation
 * travels with them.
 *   keys_in / keys_out  : uint32 [n] (device, must not alias); with
 *                         TS_FLAG_F32_ORDERED binary32 bit patterns, -0 < +0.
 *   payload_in / out    : optional uint32 [n] moved with the keys (one word per key).
 *   perm_out            : optional int32 [n]: source index of every output slot; not
 *                         together with a payload (TS_ERR_UNSUPPORTED).
 *   n                   : 0 <= n < 2^31.
 *   workspace           : ts_workspace_bytes(TS_OP_DEVICE_SORT, flags, 1, n, n, c) bytes
 *                         with c = 1 when a payload or perm_out is given, else 0; holds
 *                         one ping-pong copy of the keys (and payload words) plus the
 *                         tile histograms.
 * Returns TS_ERR_INVALID for NULL or aliasing arrays, TS_ERR_WORKSPACE for a short
 * workspace; the work is enqueued on `stream` (no host synchronisation).
 */
ts_status ts_device_sort(const uint32_t* keys_in, uint32_t* keys_out, const uint32_t* payload_in,
                         uint32_t* payload_out, int32_t* perm_out, int64_t n, uint32_t flags,
                         void* workspace, size_t workspace_bytes, void* stream);

/*
 * ts_device_partition -- stable w-way partition of one array of n labels (the whole
 * array, not tiles): items grouped by label in ascending label order, input order kept
 * within a label (Sec. 1: partitioning, and its use as the step of a quicksort with
 * pivots).  One pass of ts_device_sort with the label as the digit: per-tile label
 * counts, their prefix in label-major order, and the conflict-free split partition of
 * every tile (4096 labels alone, 8192 with a payload word or the permutation) storing
 * each label block at its place in the array.
 *   labels_in / out     : uint32 [n] (device, must not alias); labels in
 *                         [0, num_classes), 1 <= num_classes <= 64.
 *   payload_in / out    : optional uint32 [n] moved with the labels (one word each).
 *   perm_out            : optional int32 [n]: source index of every output slot; not
 *                         together with a payload (TS_ERR_UNSUPPORTED).
 *   n                   : 0 <= n < 2^31.
 *   flags               : TS_FLAG_VALIDATE: a label >= num_classes sets the workspace
 *                         error word (ts_check).  Unchecked, such a label is split on
 *                         its low ceil(log2(num_classes)) bits; no access leaves the
 *                         arrays either way.
 *   workspace           : ts_workspace_bytes(TS_OP_DEVICE_PARTITION, flags, 1, n, n, 0)
 *                         bytes (the tile count tables; no second copy of the data).
 * Returns TS_ERR_INVALID for NULL or aliasing arrays or a bad num_classes,
 * TS_ERR_WORKSPACE for a short workspace; the work is enqueued on `stream`.
 */
ts_status ts_device_partition(const uint32_t* labels_in, uint32_t* labels_out,
                              const uint32_t* payload_in, uint32_t* payload_out, int32_t* perm_out,
                              int64_t n, uint32_t num_classes, uint32_t flags, void* workspace,
                              size_t workspace_bytes, void* stream);

/* Bits of the device error word: ts_check reports them, tile_sort_noalloc ORs them
   into its err_out word. */
enum {
    TS_ERRBIT_TILE_TOO_LONG = 1u, /* a tile was longer than max_tile_len (skipped) */
    TS_ERRBIT_BAD_LABEL = 2u,     /* TS_FLAG_VALIDATE: a label >= num_classes */
    TS_ERRBIT_BAD_PERM = 4u,      /* TS_FLAG_VALIDATE: pi is not a permutation of its tile */
    TS_ERRBIT_BAD_OFFSETS = 8u    /* a tile outside [0, total_len) (skipped) */
};

/*
 * tile_sort_noalloc -- tile_sort for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, results and schedules as tile_sort, but no workspace.  Its scratch
 * (error word, work counters and lists, the permutation of a payload without perm_out)
 * is a static 32 MiB device array in the library, one per GPU, kept until the process
 * ends.  The call allocates nothing and enqueues only kernels (capturable).
 *   err_out : optional device uint32; the call ORs the TS_ERRBIT_* bits of the
 *             contract violations it met into it (the caller clears it).
 * Returns TS_ERR_WORKSPACE when ts_workspace_bytes(TS_OP_SORT, flags, ...) for these
 * sizes exceeds 32 MiB (e.g. the merge schedule with tiles above 32768 keys, whose runs
 * take 16 bytes per key), else what tile_sort returns.  Every call on one GPU shares
 * the array: calls that overlap in time on one GPU (two streams, two threads) race and
 * must be ordered by the caller.
 */
ts_status tile_sort_noalloc(const uint32_t* keys_in, uint32_t* keys_out,
                            const uint32_t* payload_in, uint32_t* payload_out, uint32_t channels,
                            int64_t elem_stride, int64_t chan_stride, int32_t* perm_out,
                            const int64_t* tile_offsets, int64_t num_tiles, int64_t total_len,
                            int64_t max_tile_len, uint32_t flags, uint32_t* err_out, void* stream);

/* Bytes of workspace a call of operation `op` (TS_OP_*) with these flags and sizes
   needs (never 0).  total_len is the number of items (tile_offsets[num_tiles]). */
size_t ts_workspace_bytes(int op, uint32_t flags, int64_t num_tiles, int64_t total_len,
                          int64_t max_tile_len, uint32_t channels);

/* Zero a workspace (its error word and counters) on `stream`.  Call once after
   allocating it. */
ts_status ts_workspace_init(void* workspace, size_t workspace_bytes, void* stream);

/* Synchronise `stream`, read and clear the workspace error word.  Returns TS_OK,
   or TS_ERR_INVALID with ts_last_error() describing the recorded violation. */
ts_status ts_check(void* workspace, void* stream);

/* Message for the last non-OK status returned on this thread. */
const char* ts_last_error(void);

/* Library version string. */
const char* ts_version(void);

/* ------------------------------------------------------------------------------
 * Measurement helpers (not part of the hot path).
 * ------------------------------------------------------------------------------ */

/* Plain device-to-device copy of `bytes` bytes (src, dst: device, 16-byte aligned,
   not overlapping) with streaming 16-byte vector loads and stores, one contiguous
   32 KiB chunk per workgroup: the HBM bandwidth reference kernel.  TS_ERR_INVALID for
   NULL or misaligned pointers. */
ts_status ts_copy(const void* src, void* dst, size_t bytes, void* stream);

/*
 * LDS access probe.  One kernel launch = `waves` wavefronts per workgroup x
 * `groups` workgroups; every wave repeats `iters` times one LDS instruction whose
 * 64 per-lane addresses come from lane_words[64] (32-bit word index into a 64 KiB
 * LDS array, taken modulo 16384 and rounded down to the access width).
 *   op 0 = ds_read, 1 = ds_write, 2 = ds_bpermute (lane_words = source lane);
 *   width = 1, 2 or 4 words (b32 / b64 / b128; bpermute: 1).
 * cycles_out (device, one uint64 per wave) receives the s_memtime ticks of the
 * timed loop; sink (device, 64 words per wave) receives data so the loop is kept.
 */
ts_status ts_lds_probe(const uint32_t* lane_words, int op, int width, int iters, int waves,
                       int groups, uint64_t* cycles_out, uint32_t* sink, void* stream);

/* Override a tuning knob of the kernel-selection table (used by the autotuner).
   Knobs:
   "partition_waves_4096" -- split partition kernel for tiles of up to 4096 items:
      1, 2, 4, 8 or 16 waves per workgroup on a persistent grid; 104 / 108: 4 / 8
      waves with registers capped so four workgroups fit on a CU; 106: 8 waves, three
      workgroups per CU, loading the next tile during the current one; 164 / 166 / 168:
      4 / 8 / 8 waves, one workgroup per tile with streaming global accesses, registers
      capped for 4 / 3 / 4 workgroups per CU (168 is the default); 176: as 166 with
      plain accesses.
   "permute_variant" -- router permute kernel for tiles of 4097..8192 items: 0: 16
      waves, persistent grid; 1: the same with registers capped for two workgroups per
      CU; 2: 8 waves; 6 (default) / 7: 16 capped waves, one workgroup per tile, with /
      without streaming accesses; 8: 6 on a persistent grid; 9 / 10 / 11 / 12 / 13:
      8 / 4 / 8 / 8 / 8 waves, one workgroup per tile, streaming accesses, registers
      for 4 / 2 / 3 / 2 waves per SIMD / no register cap.
   "oneshot" -- launch shape of every other split-partition, split-sort and permute
      kernel: 1 (default) one workgroup per tile with streaming accesses, 0 a
      persistent grid.
   "naive_oneshot" -- the same choice for the naive-LDS kernels (default 0).
   "merge_pack" -- 1: tiles of up to 2048 keys share a wavefront in the merge
      schedule, 0: one tile per wavefront.
   "merge_wide" -- longest tile the merge schedule sorts whole in one workgroup of
      2 / 4 / 8 wavefronts: 8192, 16384 or 32768 (default); 4096: none, longer tiles
      go through 4096-key pieces and merge rounds.
   "sort_plan_4096", "sort_plan_8192", "sort_plan_16384" -- the TS_SCHED_* value that
      tile_sort's AUTO uses for max_tile_len up to that length.
   "sort_small_batch" -- AUTO sorts batches of at most this many tiles of up to 4096
      keys with TS_SCHED_SPLIT (lower latency per tile); default 1024, 0 disables.
   Returns TS_ERR_INVALID for an unknown knob or value. */
ts_status ts_tune(const char* knob, int value);

#ifdef __cplusplus
}
#endif

#endif /* TILESORT_H */
