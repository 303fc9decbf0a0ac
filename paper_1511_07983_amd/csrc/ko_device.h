// Records shared by the host side of libko and its gfx950 kernels.
// Internal to the library: none of these types cross the C ABI.
#pragma once

#include <stdint.h>

namespace ko {

// Largest kernel set the device path handles.  Live block groups never
// exceed the set size (see ko_wave.h), so the wave engine's per-wave group
// ring has at most kMaxSet slots.
constexpr int kMaxSet = 20;
constexpr int kWave = 64;

// One kernel of a set, derived on the host from ko_kernel and the GPU model.
// 32 bytes, read with scalar loads.
struct KernelRec {
    uint32_t u_reg;     // lane registers per block
    uint32_t u_lds;     // LDS bytes per block (0 = none)
    uint32_t u_wave;    // waves per block
    uint32_t tblk;      // blocks in the grid
    float inv_reg;      // reciprocals of u_*, rounded up by 3 ulps (see cap_of)
    float inv_lds;
    float inv_wave;
    uint32_t dur;       // cycles per block, < 2^31
};

// One set of a batch.  48 bytes.
struct SetRec {
    uint32_t n;          // kernels in the set
    uint32_t kbase;      // index of its first KernelRec
    uint64_t n_orders;   // orders evaluated for this set
    uint64_t out_base;   // index of its first makespan in the output array
    uint64_t rank_lo;    // ALL / RANK_RANGE: rank of its first order
    uint64_t item_base;  // its first work item
    uint64_t list_base;  // EXPLICIT: byte offset of its first order
};

// Per-work-item partial statistics, reduced per set by ko_reduce_sets.  64 bytes.
struct Partial {
    int64_t min_ms;
    int64_t max_ms;
    uint64_t argmin;
    uint64_t argmax;
    uint64_t n_less;
    uint64_t n_equal;
    uint64_t n_greater;
    uint64_t count;
};

enum : int32_t { kModeAll = 0, kModeRange = 1, kModeExplicit = 2, kModeSampled = 3 };

// One order a lane of the lane kernel gave up on (it outgrew the lane's
// capacities).  spill_kernel evaluates it with the wave engine and
// reduce_kernel folds it into its set's statistics.  32 bytes.
struct SpillRec {
    uint32_t set;       // batch index of its set
    uint32_t item;      // its work item
    uint64_t sample;    // index of the order among its set's orders
    uint64_t pos;       // its slot in the makespan array
    int64_t makespan;   // written by spill_kernel
};

// Device status bits (OR-ed into the workspace status word).
enum : uint32_t { kStatusGroupOverflow = 1u, kStatusBadOrder = 2u };

struct SimArgs {
    const KernelRec *krec;
    const SetRec *sets;
    int32_t n_sets;
    int32_t mode;
    uint64_t n_items;
    uint64_t chunk;          // orders per work item
    uint64_t seed;           // SAMPLED
    const uint8_t *orders;   // EXPLICIT
    const int64_t *ref;      // per set, or null
    int64_t *makespans;      // or null
    Partial *partials;       // per item
    unsigned long long *item_counter;
    uint32_t *status;
    // simulate_kernel only: take items from this list (item_list_count
    // entries, a device word) instead of 0..n_items-1; null = no list
    const uint32_t *item_list;
    const unsigned long long *item_list_count;
    // simulate_lanes_kernel only: orders that exceeded a lane's capacities
    // are recorded in spill (count in spill_count, at most spill_cap); the
    // work items of orders that found the record list full are appended to
    // ovf_list (count in ovf_count) and marked in handed_bits, and then re-run
    // whole by simulate_kernel.  spill_kernel reads the records and the bits.
    uint32_t *ovf_list;
    unsigned long long *ovf_count;
    SpillRec *spill;
    unsigned long long *spill_count;
    uint64_t spill_cap;
    uint32_t *handed_bits;
    // GPU model
    uint32_t n_cu;
    uint32_t cap_reg, cap_lds, cap_wave, cap_blk;
    // memory contention (simulate_kernel only): per KernelRec, the memory
    // share of one block in 1/1024 units, and 1024 times the memory-bound
    // blocks served at full speed; share = null for the model without it
    const uint32_t *share;
    uint64_t mem_cap;
};

struct ReduceArgs {
    const SetRec *sets;
    int32_t n_sets;
    int32_t mode;
    uint64_t chunk;
    const Partial *partials;
    void *stats;             // ko_set_stats[n_sets] (layout-compatible with Partial)
    const int64_t *ref;      // per set, or null
    // orders the lane kernel spilled (null when the wave engine ran alone)
    const SpillRec *spill;
    const unsigned long long *spill_count;
    uint64_t spill_cap;
    const uint32_t *handed_bits;
};

struct HistArgs {
    const SetRec *sets;
    int32_t n_sets;
    const int64_t *makespans;
    const void *stats;       // ko_set_stats[n_sets]
    uint64_t *hist;
    int32_t n_bins;
    uint64_t per_block;      // orders per workgroup
    const uint64_t *block_base;  // per set: first workgroup (n_sets+1 entries)
};

// Launchers (ko_sim.hip).  Each returns a hipError_t value as int.
int launch_simulate(const SimArgs &a, int slots_per_lane, uint32_t group_slots, int grid,
                    void *stream);
int launch_reduce(const ReduceArgs &a, void *stream);
// Spilled orders of the lane kernel, one wavefront per order (ko_sim.hip).
int launch_spill(const SimArgs &a, int slots_per_lane, uint32_t group_slots, int grid, void *stream);

// Lane kernels (ko_lanes.hip): one order per lane, CU states as runs.  A set
// class is the largest set size a variant takes (8, 10, 12 or 16); each holds
// lane_entry_cap(class) group entries per lane in LDS.
constexpr uint32_t lane_entry_cap(int set_class)
{
    return set_class <= 10 ? 32u : (set_class <= 12 ? 48u : 64u);
}
// Most entries per lane a class takes (its entry masks are 32 or 64 bits).
constexpr uint32_t lane_entry_max(int set_class) { return set_class <= 10 ? 32u : 64u; }
int launch_simulate_lanes(const SimArgs &a, int set_class, uint32_t entries, int grid, void *stream);
int launch_hist(const HistArgs &a, uint64_t n_blocks, void *stream);
int launch_zero_u64(uint64_t *p, uint64_t count, void *stream);
int device_cu_count(int *out);

}  // namespace ko
