// Launchers of ko_select.hip (internal to libko).  Each returns a hipError_t
// value as int.
#pragma once

#include <stdint.h>

#include "ko_device.h"

namespace ko {

int launch_sample_orders(uint32_t n, uint32_t set, uint64_t seed, uint64_t first,
                         const uint64_t *indices, uint64_t count, uint8_t *orders, uint8_t *positions,
                         void *stream);
int launch_radix_hist_f32(const float *src, uint64_t count, uint32_t shift, uint64_t mask,
                          uint64_t prefix, unsigned long long *bins, int grid_cap, void *stream);
int launch_radix_hist_i64(const int64_t *src, uint64_t count, uint32_t shift, uint64_t mask,
                          uint64_t prefix, unsigned long long *bins, int grid_cap, void *stream);
int launch_gather_f32(const float *src, uint64_t count, uint32_t kth_key, uint64_t *out, uint64_t cap,
                      unsigned long long *cursor, int grid_cap, void *stream);
int launch_bitonic_sort_u64(uint64_t *keys, uint64_t used, uint64_t n_pow2, void *stream);
int launch_minmax_i64(const int64_t *v, uint64_t count, unsigned long long *mm, int grid_cap, void *stream);
// Tiles of the radix sort (counts needs 256 * tiles words).
uint64_t sort_tiles(uint64_t count);
// Stable sort of v[0, count) (count < 2^32) by value: `passes` 8-bit digits of
// v - vmin, ping-ponging between the (keys, idx) buffers a and b; sorted values
// and their indices in v to `sorted` and `index` (either may be null).
int launch_sort_i64(const int64_t *v, uint64_t count, int64_t vmin, uint32_t passes, uint64_t *keys_a,
                    uint32_t *idx_a, uint64_t *keys_b, uint32_t *idx_b, uint32_t *counts, int64_t *sorted,
                    uint64_t *index, void *stream);
int launch_unpack_topk(const uint64_t *keys, uint32_t k, int64_t *idx, float *val, void *stream);
// Statistics of v[0, count) (min/max with the smallest index on ties, counts
// against *ref if ref is not null) into `stats` (one ko_set_stats): n_parts
// workgroups write Partials to `parts`, one more workgroup combines them.
int launch_stats_i64(const int64_t *v, uint64_t count, const int64_t *ref, Partial *parts, uint32_t n_parts,
                     void *stats, void *stream);

}  // namespace ko
