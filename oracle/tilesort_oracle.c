/*
 * CPU oracle for tile sort / partition / permute.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the HIP library.
 *
 * Every routine is the plain definition of the problem, written for
 * readability, not speed:
 *
 *  - Sorting (Afshani & Sitchinava, Sec. 1, "Problems of interest", sorting):
 *    the items of a tile are put in ascending order.  Ties are broken by the
 *    item's position inside the tile, i.e. the sort is stable, which makes the
 *    output (keys, payload, source index) unique.
 *  - w-way partition (abstract; Sec. 1 "Problems of interest", partition):
 *    items carry a label in [0, w); the result is every item grouped by label,
 *    in ascending label order, keeping input order inside a label (a stable
 *    counting sort; the abstract defines partitioning as sorting an input that
 *    holds n/w copies of each label).
 *  - Permutation (Sec. 1 "Problems of interest", permutation): every item has
 *    a distinct destination.  SCATTER writes out[pi[i]] = in[i]; GATHER writes
 *    out[i] = in[pi[i]].
 *
 * Layout conventions shared with the public C interface:
 *  - keys / labels are contiguous uint32 arrays over all tiles;
 *  - tile t is the half-open range [offsets[t], offsets[t+1]);
 *  - payload word (g, c) of global item g lives at
 *    payload[g * elem_stride + c * chan_stride] (32-bit words);
 *  - pi and perm are tile-local int32 indices.
 *
 * Return codes: 0 = ok, -1 = invalid arguments, -2 = input breaks the data
 * contract (label out of range, pi not a permutation).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_SCATTER 0
#define ORACLE_GATHER 1
#define ORACLE_FLAG_F32_ORDERED 1u

/* Order-preserving map from an IEEE-754 binary32 bit pattern to uint32:
 * negative numbers have all bits flipped, non-negative ones get the sign bit
 * set.  For any two non-NaN floats a < b  <=>  map(a) < map(b) as unsigned;
 * -0.0 maps below +0.0. */
uint32_t oracle_f32_order(uint32_t b) {
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

uint32_t oracle_f32_order_inv(uint32_t u) {
    return (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
}

static int offsets_ok(const int64_t* offsets, int64_t num_tiles) {
    if (num_tiles < 0 || (num_tiles > 0 && offsets == NULL)) return 0;
    if (num_tiles > 0 && offsets[0] < 0) return 0;
    for (int64_t t = 0; t < num_tiles; ++t)
        if (offsets[t + 1] < offsets[t]) return 0;
    return 1;
}

/* ---------------------------------------------------------------- sorting */

/* Top-down merge sort of idx[0..n) by key[idx], stable: on equal keys the
 * element from the left half (smaller original position) goes first. */
static void merge_sort_idx(int32_t* idx, int32_t* tmp, int64_t n, const uint32_t* key) {
    if (n < 2) return;
    int64_t h = n / 2;
    merge_sort_idx(idx, tmp, h, key);
    merge_sort_idx(idx + h, tmp, n - h, key);
    int64_t a = 0, b = h, o = 0;
    while (a < h && b < n) {
        if (key[idx[b]] < key[idx[a]]) tmp[o++] = idx[b++];
        else tmp[o++] = idx[a++];
    }
    while (a < h) tmp[o++] = idx[a++];
    while (b < n) tmp[o++] = idx[b++];
    memcpy(idx, tmp, (size_t)n * sizeof(int32_t));
}

static void sort_one_tile(const uint32_t* keys, uint32_t* keys_out,
                          const uint32_t* payload, uint32_t* payload_out, uint32_t channels,
                          int64_t es, int64_t cs, int32_t* perm_out,
                          int64_t o, int64_t n, uint32_t flags) {
    if (n == 0) return;
    uint32_t* k = (uint32_t*)malloc((size_t)n * sizeof(uint32_t));
    int32_t* idx = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t* tmp = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    for (int64_t i = 0; i < n; ++i) {
        k[i] = (flags & ORACLE_FLAG_F32_ORDERED) ? oracle_f32_order(keys[o + i]) : keys[o + i];
        idx[i] = (int32_t)i;
    }
    merge_sort_idx(idx, tmp, n, k);
    for (int64_t r = 0; r < n; ++r) {
        int64_t src = idx[r];
        if (keys_out) keys_out[o + r] = keys[o + src];   /* original bits, not the mapped key */
        if (perm_out) perm_out[o + r] = (int32_t)src;
        if (payload && payload_out)
            for (uint32_t c = 0; c < channels; ++c)
                payload_out[(o + r) * es + (int64_t)c * cs] = payload[(o + src) * es + (int64_t)c * cs];
    }
    free(k);
    free(idx);
    free(tmp);
}

int oracle_tile_sort(const uint32_t* keys, uint32_t* keys_out,
                     const uint32_t* payload, uint32_t* payload_out, uint32_t channels,
                     int64_t elem_stride, int64_t chan_stride, int32_t* perm_out,
                     const int64_t* offsets, int64_t num_tiles, uint32_t flags, int nthreads) {
    if (!offsets_ok(offsets, num_tiles) || (num_tiles > 0 && keys == NULL)) return -1;
    if (channels > 0 && (payload == NULL || payload_out == NULL)) return -1;
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
    for (int64_t t = 0; t < num_tiles; ++t)
        sort_one_tile(keys, keys_out, payload, payload_out, channels, elem_stride, chan_stride,
                      perm_out, offsets[t], offsets[t + 1] - offsets[t], flags);
    return 0;
}

/* -------------------------------------------------------------- partition */

static int partition_one_tile(const uint32_t* labels, uint32_t* labels_out,
                              const uint32_t* payload, uint32_t* payload_out, uint32_t channels,
                              int64_t es, int64_t cs, uint32_t num_classes, int32_t* perm_out,
                              int64_t o, int64_t n) {
    int64_t* start = (int64_t*)calloc(num_classes, sizeof(int64_t));
    int bad = 0;
    /* count the copies of every label */
    for (int64_t i = 0; i < n; ++i) {
        uint32_t l = labels[o + i];
        if (l >= num_classes) { bad = 1; break; }
        start[l] += 1;
    }
    if (!bad) {
        /* exclusive prefix sum: first output slot of every label */
        int64_t run = 0;
        for (uint32_t c = 0; c < num_classes; ++c) {
            int64_t cnt = start[c];
            start[c] = run;
            run += cnt;
        }
        /* walk the input in order; each item takes the next free slot of its label */
        for (int64_t i = 0; i < n; ++i) {
            uint32_t l = labels[o + i];
            int64_t d = start[l]++;
            if (labels_out) labels_out[o + d] = l;
            if (perm_out) perm_out[o + d] = (int32_t)i;
            if (payload && payload_out)
                for (uint32_t c = 0; c < channels; ++c)
                    payload_out[(o + d) * es + (int64_t)c * cs] = payload[(o + i) * es + (int64_t)c * cs];
        }
    }
    free(start);
    return bad;
}

int oracle_tile_partition(const uint32_t* labels, uint32_t* labels_out,
                          const uint32_t* payload, uint32_t* payload_out, uint32_t channels,
                          int64_t elem_stride, int64_t chan_stride, uint32_t num_classes,
                          int32_t* perm_out, const int64_t* offsets, int64_t num_tiles,
                          int nthreads) {
    if (!offsets_ok(offsets, num_tiles) || (num_tiles > 0 && labels == NULL)) return -1;
    if (num_classes == 0) return -1;
    if (channels > 0 && (payload == NULL || payload_out == NULL)) return -1;
    if (nthreads < 1) nthreads = 1;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads) reduction(| : bad)
    for (int64_t t = 0; t < num_tiles; ++t)
        bad |= partition_one_tile(labels, labels_out, payload, payload_out, channels, elem_stride,
                                  chan_stride, num_classes, perm_out, offsets[t],
                                  offsets[t + 1] - offsets[t]);
    return bad ? -2 : 0;
}

/* ------------------------------------------------------------ permutation */

static int permute_one_tile(const uint32_t* in, uint32_t* out, uint32_t channels, int64_t es,
                            int64_t cs, const int32_t* pi, uint32_t direction, int64_t o,
                            int64_t n) {
    /* pi must be a permutation of [0, n) */
    unsigned char* seen = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
    int bad = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t p = pi[o + i];
        if (p < 0 || p >= n || seen[p]) { bad = 1; break; }
        seen[p] = 1;
    }
    free(seen);
    if (bad) return 1;
    for (int64_t i = 0; i < n; ++i) {
        int64_t p = pi[o + i];
        int64_t dst = (direction == ORACLE_SCATTER) ? p : i;
        int64_t src = (direction == ORACLE_SCATTER) ? i : p;
        for (uint32_t c = 0; c < channels; ++c)
            out[(o + dst) * es + (int64_t)c * cs] = in[(o + src) * es + (int64_t)c * cs];
    }
    return 0;
}

int oracle_tile_permute(const uint32_t* in, uint32_t* out, uint32_t channels, int64_t elem_stride,
                        int64_t chan_stride, const int32_t* pi, uint32_t direction,
                        const int64_t* offsets, int64_t num_tiles, int nthreads) {
    if (!offsets_ok(offsets, num_tiles)) return -1;
    if (num_tiles > 0 && (in == NULL || out == NULL || pi == NULL)) return -1;
    if (direction != ORACLE_SCATTER && direction != ORACLE_GATHER) return -1;
    if (nthreads < 1) nthreads = 1;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads) reduction(| : bad)
    for (int64_t t = 0; t < num_tiles; ++t)
        bad |= permute_one_tile(in, out, channels, elem_stride, chan_stride, pi, direction,
                                offsets[t], offsets[t + 1] - offsets[t]);
    return bad ? -2 : 0;
}
