/*
 * ko.h — exact evaluation of GPU kernel launch orders on MI355X (gfx950).
 *
 * C ABI of libko.so.  The library evaluates, for a set of independent kernels
 * described by the kernel parameters of Table 1 of Li, Narayana & El-Ghazawi,
 * "Reordering GPU Kernel Launches to Enable Efficient Concurrent Execution"
 * (2015), the total execution time of launch orders under a discrete-event
 * model of thread-block dispatch, and derives the launch order of the paper's
 * Algorithm 1.  The input is the kernel set with its profile (Algorithm 1's
 * input), the output is a launch order (Algorithm 1's output), its total
 * execution time and its percentile rank among all orders (Table 3).
 *
 * Dispatch model (Section 2, read as follows; makespans are int64 cycles):
 *   - the blocks of all kernels form one stream in launch order, kernel by
 *     kernel; the stream is never reordered: while its front block fits on no
 *     CU, no later block is placed;
 *   - placement is round-robin: a cyclic CU pointer, starting at CU 0 and
 *     never reset; a block goes to the first CU at or after the pointer whose
 *     free registers, LDS bytes, waves and block slots all cover the block's
 *     use, and the pointer moves to the next CU;
 *   - a block of kernel i holds regs_thr * waves_blk * wave_size lane
 *     registers, lds_blk bytes, waves_blk waves and one block slot for
 *     ceil(n_inst * max(r_milli, rb_milli) / r_milli) cycles (Section 4: a
 *     kernel below the balanced ratio R_B is memory bound and its blocks
 *     stretch by R_B / R_i); blocks of co-resident kernels do not slow each
 *     other;
 *   - all blocks finishing at a cycle release before placement resumes at
 *     that cycle; the makespan is the cycle at which the last block ends.
 *
 * Orders and ranks: order[j] is the 0-based input index of the kernel launched
 * at position j.  Ranks are lexicographic over these sequences (rank 0 is the
 * identity order, rank n!-1 the reversed one).
 *
 * Conventions:
 *   - every function returns 0 (KO_OK) or a negative KO_E* code; no C++
 *     exception crosses the ABI; ko_last_error() describes the last failure;
 *   - "host" pointers are ordinary CPU memory, "device" pointers are HIP
 *     device allocations on the current device (for example the data_ptr()
 *     of a torch tensor on cuda:N under ROCm); the caller owns every buffer
 *     it passes in and the library never frees or retains one past the call;
 *   - hip_stream is a hipStream_t (0 = the null stream);
 *   - the library keeps a lazily grown per-device workspace that
 *     ko_shutdown() releases (it is also released at process exit).
 */
#ifndef KO_H
#define KO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KO_OK 0
#define KO_EINVAL (-1) /* bad argument: see each function */
#define KO_ERANGE (-2) /* an order count or rank outside uint64, or n too large for the mode */
#define KO_ENOMEM (-3) /* host or device allocation failed */
#define KO_EHIP (-4)   /* HIP runtime error, or a device status error from an earlier call */

/* The per-CU limits of Table 1 (first three rows).  40 bytes. */
typedef struct ko_gpu_model {
    int32_t n_cu;      /* N_SM: CUs (SMs); 1 .. 256 */
    int32_t wave_size; /* lanes per wave (warp); >= 1 */
    int32_t wave_cu;   /* N_warp_SM: resident waves per CU; 1 .. 2^24 */
    int32_t blk_cu;    /* N_blk_SM: resident blocks per CU; 1 .. 255 */
    int64_t reg_cu;    /* N_reg_SM: lane registers per CU; 1 .. 2^24 */
    int64_t lds_cu;    /* N_shm_SM: LDS / shared-memory bytes per CU; 1 .. 2^24 */
    int32_t rb_milli;  /* R_B, the balanced instruction/memory ratio, times 1000; >= 1 */
    int32_t mem_blocks; /* 0: co-resident blocks do not slow each other (the model above);
                           1 .. 2^24: they share the chip's memory throughput, which serves
                           this many memory-bound blocks at full speed (see below) */
} ko_gpu_model;

/* Memory contention (mem_blocks > 0; Section 4: the blocks that run together
 * should balance instructions against memory accesses, R_B being a property
 * of the whole chip).  A block of kernel i alone keeps the memory system busy
 * for the share min(R_i, R_B) / R_i of its duration, counted in 1/1024 units
 * and rounded up: s_i = ceil(1024 * min(r_milli, rb_milli) / r_milli).  While
 * the resident blocks' shares add up to U > 1024 * mem_blocks, every resident
 * block runs slower by the same factor: a cycle brings
 * floor(65536 * 1024 * mem_blocks / U) units of progress instead of 65536.  A
 * block needs duration * 65536 units and ends at the first whole cycle at
 * which it has them; all blocks ending at a cycle release before placement
 * resumes; placement is unchanged.  With mem_blocks large enough that U never
 * exceeds the cap, makespans equal those of mem_blocks = 0.  Both engines
 * model it (the lane engine keeps each group's progress in 64 bits and steps
 * the drain event by event); ko_heuristic_order ignores mem_blocks,
 * ko_simulate_rounds refuses a nonzero value. */

/* The per-kernel parameters of Table 1 (last three rows).  40 bytes. */
typedef struct ko_kernel {
    int64_t n_tblk;    /* N_tblk_i: blocks in the grid; >= 1 */
    int64_t n_inst;    /* N_inst_i: instructions per block (cycles when R_i >= R_B); >= 1 */
    int64_t lds_blk;   /* N_shm_i: LDS bytes per block; >= 0 */
    int32_t waves_blk; /* N_warp_i: waves per block; >= 1 */
    int32_t regs_thr;  /* N_reg_i as registers per thread; >= 1 */
    int32_t r_milli;   /* R_i, the kernel's instruction/memory ratio, times 1000; >= 1 */
    int32_t reserved;  /* must be 0 */
} ko_kernel;

/* Per-set statistics over the evaluated orders (Table 3 columns, Figure 1).  64 bytes.
 * argmin/argmax: for KO_ORDERS_ALL and KO_ORDERS_RANK_RANGE the lexicographic rank,
 * for KO_ORDERS_EXPLICIT and KO_ORDERS_SAMPLED the index of the order within the
 * set's list; ties go to the smallest.  The three counts compare each makespan
 * with the set's reference makespan and are 0 when no reference is given. */
typedef struct ko_set_stats {
    int64_t min_makespan;
    int64_t max_makespan;
    uint64_t argmin;
    uint64_t argmax;
    uint64_t n_less;
    uint64_t n_equal;
    uint64_t n_greater;
    uint64_t n_orders;
} ko_set_stats;

/* Percentile rank of one order (Table 3, "Percentile rank").  The counts are
 * exact; the three percentages are 100 * (n_greater + n_equal) / n_total
 * (inclusive, the headline), 100 * n_greater / n_total (strict) and
 * 100 * (n_greater + n_equal / 2) / n_total (mid-rank). */
typedef struct ko_rank_result {
    int64_t makespan;      /* of the given order */
    int64_t min_makespan;  /* best ("optimal") over the evaluated orders */
    int64_t max_makespan;  /* worst over the evaluated orders */
    uint64_t n_less;
    uint64_t n_equal;
    uint64_t n_greater;
    uint64_t n_total;
    double pct_inclusive;
    double pct_strict;
    double pct_mid;
} ko_rank_result;

#define KO_ORDERS_ALL 0        /* every order, ranks 0 .. n!-1; n <= 20 */
#define KO_ORDERS_RANK_RANGE 1 /* ranks lo .. hi-1 per set */
#define KO_ORDERS_EXPLICIT 2   /* orders given in device memory */
#define KO_ORDERS_SAMPLED 3    /* uniform ranks with replacement, counter-based */

/* Which orders of each set to evaluate.
 * SAMPLED: sample i of set s has rank floor(x * n! / 2^64) where x is output
 * number (s << 40) | i of SplitMix64 (Steele, Lea & Flood 2014) seeded with
 * `seed`, i.e. the SplitMix64 mix of seed + (c + 1) * 0x9E3779B97F4A7C15.
 * So a SAMPLED spec takes at most 2^40 samples per set and 2^24 sets
 * (KO_ERANGE otherwise): past those, counters would repeat other streams. */
typedef struct ko_order_spec {
    int32_t mode;                  /* KO_ORDERS_* */
    int32_t reserved;              /* must be 0 */
    const uint64_t *rank_lo_hi;    /* RANK_RANGE: host, 2 per set: [lo, hi), lo <= hi <= n! */
    const uint8_t *orders_dev;     /* EXPLICIT: device, the sets' orders back to back, each
                                      order n_s bytes (kernel indices); must be permutations */
    const int64_t *orders_per_set; /* EXPLICIT and SAMPLED: host, one count >= 0 per set */
    uint64_t seed;                 /* SAMPLED */
} ko_order_spec;

/* Heuristic flags (readings of Algorithm 1 where the paper is open). */
#define KO_HEUR_PER_BLOCK 1u /* ScoreGen on one block's use (default: ceil(N_tblk/N_SM) blocks) */
#define KO_HEUR_FULL_SORT 2u /* stably re-sort a round by decreasing LDS after each insertion
                                (default: the new kernel goes before the round iff its LDS
                                 exceeds the round's combined LDS, else after it) */

/*
 * ko_heuristic_order — the launch order of Algorithm 1 (ScoreGen,
 * ProfileCombine, execution rounds; Section 5).  Host only, synchronous.
 *   gpu, k      host; k[0..n-1] the kernel set
 *   n           1 .. 20
 *   flags       KO_HEUR_* bits
 *   order_out   host int32[n]: the order
 *   round_out   host int32[n] or NULL: the execution round (0-based) of each position
 * Scores are binary64 evaluated in a fixed order with exact ties resolved to
 * the first candidate in index order.  Errors: KO_EINVAL for a NULL required
 * pointer, n out of range, an invalid model or kernel, unknown flags.
 */
int ko_heuristic_order(const ko_gpu_model *gpu, const ko_kernel *k, int32_t n, uint32_t flags,
                       int32_t *order_out, int32_t *round_out);

/*
 * ko_count_orders — how many orders each set of a batch evaluates under a spec,
 * and where each set's makespans start in the output array.  Host only.
 *   set_offsets  host int32[n_sets+1], set s = kernels set_offsets[s] .. set_offsets[s+1]-1
 *   per_set_out  host uint64[n_sets] or NULL
 *   total_out    host uint64[1]: the sum (the length of the makespan output)
 * Errors: KO_EINVAL (bad offsets, set size outside 1..20, bad spec), KO_ERANGE
 * (n! or the total does not fit in uint64; SAMPLED past 2^40 samples per set
 * or 2^24 sets).
 */
int ko_count_orders(const int32_t *set_offsets, int32_t n_sets, const ko_order_spec *spec,
                    uint64_t *per_set_out, uint64_t *total_out);

/*
 * ko_simulate_batch — makespans of many launch orders of many kernel sets on
 * one GPU model (the exhaustive or sampled evaluation behind Table 3 and
 * Figure 1).  Stream-ordered and asynchronous: argument validation happens
 * before anything is enqueued and returns synchronously; a device status
 * error of this call is reported by the next call (or by ko_sync).
 *   gpu              host
 *   kernels          host ko_kernel[set_offsets[n_sets]], all sets back to back
 *   set_offsets      host int32[n_sets+1], nondecreasing from 0; each set has 1..20 kernels
 *   n_sets           >= 1
 *   spec             host; which orders (see ko_order_spec)
 *   ref_makespan_dev device int64[n_sets] or NULL: reference makespan per set for the counts
 *   makespans_dev    device int64[total] or NULL: makespan of every evaluated order, set by
 *                    set, within a set in rank order (ALL, RANK_RANGE) or list order
 *   stats_dev        device ko_set_stats[n_sets] or NULL
 *   hist_dev         device uint64[n_sets * n_bins] or NULL: per set, bin of a makespan M is
 *                    floor((M - min) * n_bins / (max - min + 1)); needs makespans_dev and
 *                    stats_dev
 *   n_bins           1 .. 65536 when hist_dev is given
 *   hip_stream       hipStream_t
 * A set with zero orders gets min = INT64_MAX, max = INT64_MIN, argmin = argmax = 0.
 * Errors: KO_EINVAL (bad pointers, sizes, models, kernels, or a block that does not
 * fit an empty CU), KO_ERANGE (counts), KO_ENOMEM, KO_EHIP.
 */
int ko_simulate_batch(const ko_gpu_model *gpu, const ko_kernel *kernels, const int32_t *set_offsets,
                      int32_t n_sets, const ko_order_spec *spec, const int64_t *ref_makespan_dev,
                      int64_t *makespans_dev, ko_set_stats *stats_dev, uint64_t *hist_dev,
                      int32_t n_bins, void *hip_stream);

/*
 * ko_simulate_batch_noalloc — ko_simulate_batch for callers that cannot
 * allocate device or pinned host memory (code that must not call hipMalloc:
 * tight serving loops, harnesses that forbid allocation).  Same arguments,
 * outputs and errors as ko_simulate_batch, with these differences:
 *   - the batch's tables, counters and work-item partials live in a
 *     16 MiB array in device memory that the library holds for the life of
 *     the process on every GPU it runs on; nothing is allocated per call
 *     (the library's own device workspace is not used either);
 *   - work items are at most 65536 whole chunks of orders (plus one partial
 *     chunk per set); a batch whose tables and items need more than the
 *     array holds fails with KO_ERANGE before any device work;
 *   - synchronous: returns when the evaluation has finished on hip_stream,
 *     with any device status error of this call (KO_EHIP for a malformed
 *     explicit order);
 *   - all calls on one GPU share the array and keep the last call's
 *     contents; calls of one process are serialised by the library, so
 *     overlapping calls on one GPU (from several processes sharing one
 *     copy, which HIP does not do, or around the library's lock) would race.
 */
int ko_simulate_batch_noalloc(const ko_gpu_model *gpu, const ko_kernel *kernels, const int32_t *set_offsets,
                              int32_t n_sets, const ko_order_spec *spec, const int64_t *ref_makespan_dev,
                              int64_t *makespans_dev, ko_set_stats *stats_dev, uint64_t *hist_dev,
                              int32_t n_bins, void *hip_stream);

/*
 * ko_rank_percentile — the makespan of one order and its percentile rank
 * among all n! orders (n_samples = 0) or among n_samples sampled orders
 * (KO_ORDERS_SAMPLED with `seed`, set index 0).  Synchronous: waits on
 * hip_stream before returning.
 *   gpu, k, n   host; n in 1 .. 20
 *   order       host int32[n], a permutation of 0..n-1
 *   out         host
 * Errors: KO_EINVAL, KO_ERANGE, KO_ENOMEM, KO_EHIP.
 */
int ko_rank_percentile(const ko_gpu_model *gpu, const ko_kernel *k, int32_t n, const int32_t *order,
                       uint64_t n_samples, uint64_t seed, ko_rank_result *out, void *hip_stream);

/* ko_sync — wait for hip_stream and report any device status error of earlier calls. */
int ko_sync(void *hip_stream);

/* ko_shutdown — release the per-device workspaces.  Later calls recreate them. */
int ko_shutdown(void);

/* ------------------------------------------------------------------ plans
 * A plan is a batch (model, kernel sets, order spec) prepared once: kernel
 * records derived, work decomposed and tables uploaded to the device.
 * Launching it only enqueues kernels on a stream (no allocation, copy, memset
 * or synchronisation), so a launch can be captured in a HIP graph and
 * replayed: the way many kernel sets of uneven size are evaluated in one
 * persistent launch fed by a device work queue, again and again. */

typedef struct ko_plan ko_plan;
typedef struct ko_graph ko_graph;

/* Launch configuration (16 bytes); zero fields take the defaults. */
/* Engines of the simulation (all give identical results):
 *   KO_ENGINE_WAVE   one wavefront per order, lanes own CUs (any model, n <= 20);
 *   KO_ENGINE_LANES  one lane per order, the CUs' free resources held as runs
 *                    of equal values (n <= 16, N_CU <= 256, registers per CU
 *                    < 2^23, LDS per CU < 2^18 bytes, waves and blocks per CU
 *                    < 128); orders that outgrow its per-lane capacities
 *                    are evaluated by the wave engine, one wavefront each;
 *   KO_ENGINE_AUTO   the lane engine where it applies to a batch of at least
 *                    8192 orders, else the wave engine. */
enum { KO_ENGINE_AUTO = 0, KO_ENGINE_WAVE = 1, KO_ENGINE_LANES = 2 };

typedef struct ko_launch_config {
    int32_t chunk_log2;  /* orders per work item = 2^chunk_log2 (1..20); 0 = automatic */
    int32_t wg_per_cu;   /* persistent workgroups (4 waves each) per CU (1..64); 0 = 8;
                            the lane engine launches 2x as many one-wave workgroups
                            (at most 32 per CU) */
    int32_t engine;      /* KO_ENGINE_*; KO_EINVAL if LANES does not apply */
    int32_t lane_entries; /* lane engine: group entries per lane (1..64, at most 32 used
                             for sets of up to 10 kernels); 0 = by set size (32 up to 10
                             kernels, 48 up to 12, 64 up to 16).  Fewer entries send
                             more orders to the wave engine. */
} ko_launch_config;

/* ko_plan_create — prepare a batch as ko_simulate_batch takes it (same
 * arguments and errors); config may be NULL.  The plan belongs to the current
 * device.  In EXPLICIT mode spec->orders_dev is read at every launch and must
 * stay valid for the life of the plan.  Synchronous. */
int ko_plan_create(const ko_gpu_model *gpu, const ko_kernel *kernels, const int32_t *set_offsets,
                   int32_t n_sets, const ko_order_spec *spec, const ko_launch_config *config,
                   ko_plan **out);

/* ko_plan_info — orders in the batch, work items, orders per item and
 * workgroups of the persistent grid (any output may be NULL). */
int ko_plan_info(const ko_plan *plan, uint64_t *total_orders, uint64_t *work_items, uint64_t *chunk,
                 int32_t *grid);

/* ko_plan_launch — enqueue one evaluation of the plan on hip_stream; outputs
 * as in ko_simulate_batch.  Kernel launches only: capturable.  Launches of one
 * plan share its work queue and partials, so they must not overlap in time
 * (issue them on one stream).  The device status of the launch is read by
 * ko_plan_status. */
int ko_plan_launch(ko_plan *plan, const int64_t *ref_makespan_dev, int64_t *makespans_dev,
                   ko_set_stats *stats_dev, uint64_t *hist_dev, int32_t n_bins, void *hip_stream);

/* ko_plan_status — wait for hip_stream, then report the device status of the
 * plan's last launch (KO_EHIP for a malformed explicit order). */
int ko_plan_status(ko_plan *plan, void *hip_stream);

/* ko_plan_engine — the engine the plan runs (KO_ENGINE_WAVE or KO_ENGINE_LANES),
 * its group entries per lane (0 for the wave engine) and, after waiting for
 * hip_stream, what the plan's last launch passed from the lane engine to the
 * wave engine: orders evaluated one wavefront each (spilled_out, counting
 * those the record list could not hold) and work items re-run whole
 * (handed_over_out).  Any output may be NULL. */
int ko_plan_engine(ko_plan *plan, int32_t *engine_out, int32_t *lane_entries_out, uint64_t *spilled_out,
                   uint64_t *handed_over_out, void *hip_stream);

/* ko_plan_destroy — wait for the device, free the plan (NULL is a no-op). */
int ko_plan_destroy(ko_plan *plan);

/* ko_graph_capture — capture one ko_plan_launch with these outputs on
 * hip_stream (a created stream, not the null stream) into an instantiated
 * HIP graph.  The graph holds the plan's and the outputs' addresses: they
 * must outlive it.  Replays share the plan's work queue with its launches. */
int ko_graph_capture(ko_plan *plan, const int64_t *ref_makespan_dev, int64_t *makespans_dev,
                     ko_set_stats *stats_dev, uint64_t *hist_dev, int32_t n_bins, void *hip_stream,
                     ko_graph **out);

/* ko_graph_launch — replay a captured evaluation on hip_stream. */
int ko_graph_launch(ko_graph *graph, void *hip_stream);

/* ko_graph_destroy — wait for the device, free the graph (NULL is a no-op). */
int ko_graph_destroy(ko_graph *graph);

/* ko_simulate_rounds — makespans of launch orders under the
 * round-synchronous reading of Section 2's execution rounds.  Blocks are taken
 * from the front of the kernel-major stream and placed as in
 * ko_simulate_batch (first CU at or after the cyclic pointer with room for
 * the block), but no block releases its resources inside a round: when the
 * front block fits on no CU the round ends, it lasts as long as its longest
 * block, every CU is freed and the next round starts with that block (the
 * pointer carries over).  The makespan is the sum of the round lengths.
 *   gpu, kernels, n  host model and set (1 <= n <= 20), validated and derived
 *                    as in ko_simulate_batch
 *   orders_dev       uint8 [count][n], device: order[j] = kernel at position j;
 *                    each row must be a permutation of 0..n-1; a row with an
 *                    entry >= n or a repeated entry gets makespan -1.
 *                    NULL: the orders of lexicographic ranks first ..
 *                    first+count-1 among all n! orders, unranked on the device
 *   first            first rank when orders_dev is NULL, else 0
 *   makespans_dev    int64 [count], device, written: cycles
 * count <= 2^40; count 0 validates and returns.  Asynchronous on hip_stream;
 * the caller keeps both buffers alive until the stream has passed the call.
 * Errors: KO_EINVAL (model, kernels, n, NULL makespans, first with explicit
 * orders), KO_ERANGE (count, ranks past n!), KO_EHIP (launch). */
int ko_simulate_rounds(const ko_gpu_model *gpu, const ko_kernel *kernels, int32_t n,
                       const uint8_t *orders_dev, uint64_t first, uint64_t count, int64_t *makespans_dev,
                       void *hip_stream);

/* ko_sample_orders — the launch orders that ko_simulate_batch evaluates in
 * KO_ORDERS_SAMPLED mode for the set at batch index set_index (seed as in
 * ko_order_spec.seed): sample i is the order of rank
 * floor(splitmix64(seed, counter = set_index * 2^40 + i) * n! / 2^64).
 *   n             kernels in the set, 1..20
 *   set_index     0 .. 2^24-1
 *   first, count  samples first .. first+count-1 (first + count <= 2^40) when
 *                 indices_dev is NULL; otherwise samples indices_dev[0..count)
 *                 (uint64, device, each < 2^40)
 *   orders_dev    uint8 [count][n], device, nullable: order[j] = kernel at position j
 *   positions_dev uint8 [count][n], device, nullable: pos[i] = position of kernel i
 * At least one output.  Asynchronous on hip_stream.  Used to build the inputs
 * of a learned scorer for exactly the orders the simulator evaluates.
 * Errors: KO_EINVAL (n, set_index, both outputs NULL), KO_ERANGE (indices). */
int ko_sample_orders(int32_t n, int32_t set_index, uint64_t seed, uint64_t first,
                     const uint64_t *indices_dev, uint64_t count, uint8_t *orders_dev,
                     uint8_t *positions_dev, void *hip_stream);

/* ko_topk_f32 — the k smallest values of y[count] (float32, device) with their
 * indices, ascending by (value, index): idx_out[k] (int64, device, nullable)
 * and val_out[k] (float32, device, nullable; at least one of the two).
 * Values are ordered as IEEE numbers (-0 before +0; a NaN orders by its bit
 * pattern, above +inf when its sign is clear).  1 <= count < 2^32,
 * 1 <= k <= min(count, 16384).  Radix selection on the device; the call
 * returns once the k-th smallest value is known and the sorted outputs are
 * enqueued on hip_stream.
 * Errors: KO_EINVAL (arguments), KO_ERANGE (more than 32768 values at or
 * below the k-th smallest, i.e. massive ties), KO_EHIP. */
int ko_topk_f32(const float *y_dev, uint64_t count, int32_t k, int64_t *idx_out_dev, float *val_out_dev,
                void *hip_stream);

/* ko_kth_smallest_i64 — the k-th smallest (1-based) of v[count] (int64,
 * device) into *value_out (host) and, if count_le_out is not NULL, the number
 * of elements <= that value (ties included) into *count_le_out (host).  For
 * the makespans of a full enumeration with k = ceil(count / 100) this is the
 * makespan that marks the best 1% of orders and how many orders reach it
 * (Table 3's percentile ranks, read backwards).  Synchronous.
 * Errors: KO_EINVAL (NULL v_dev or value_out, k outside 1..count), KO_EHIP. */
int ko_kth_smallest_i64(const int64_t *v_dev, uint64_t count, uint64_t k, int64_t *value_out,
                        uint64_t *count_le_out, void *hip_stream);

/* ko_sort_i64 — the ranking curve of a full enumeration (Figure 1's
 * "Ranking"): the makespans v[count] (int64, device) in ascending order into
 * sorted_out[count] (int64, device, nullable) and, in index_out[count]
 * (uint64, device, nullable), the position in v of each; equal values keep
 * their order in v (for a rank-ordered makespan array, ties go to the smaller
 * rank, so both outputs are unique).  At least one output; either may be v
 * itself.  1 <= count < 2^32.  A stable LSD radix sort on the device over the
 * 8-bit digits that v - min(v) uses; its (key, index) buffers are the
 * library's workspace (12 bytes per value, twice).  Synchronous.
 * Errors: KO_EINVAL (arguments), KO_ENOMEM, KO_EHIP. */
int ko_sort_i64(const int64_t *v_dev, uint64_t count, int64_t *sorted_out_dev, uint64_t *index_out_dev,
                void *hip_stream);

/* ko_stats_i64 — statistics of an int64 array already in device memory (the
 * makespans another call left there, e.g. ko_simulate_rounds): Table 3's
 * optimal and worst with their smallest indices, and the counts behind a
 * percentile rank, into one ko_set_stats: min/max makespan, argmin/argmax
 * (index in v; ties to the smallest), n_less/n_equal/n_greater against
 * *ref_dev (0 when ref_dev is NULL), n_orders = count.  An empty array gives
 * min INT64_MAX, max INT64_MIN, argmin = argmax = 0.
 *   v_dev      device int64[count]; count <= 2^40
 *   ref_dev    device int64[1] or NULL
 *   stats_dev  device ko_set_stats[1]
 * Asynchronous on hip_stream (a reduction on the device; the partials live in
 * the library's workspace).  Errors: KO_EINVAL (NULL stats_dev, NULL v_dev
 * with count > 0), KO_ERANGE (count), KO_ENOMEM, KO_EHIP. */
int ko_stats_i64(const int64_t *v_dev, uint64_t count, const int64_t *ref_dev, ko_set_stats *stats_dev,
                 void *hip_stream);

/* ------------------------------------------------------------------ hardware
 * Validation of the model on the GPU itself (not part of the model): each
 * kernel of a set becomes a synthetic HIP kernel with its grid (n_tblk
 * blocks), waves_blk * 64 threads per block and lds_blk bytes of dynamic LDS;
 * every thread runs F = n_inst / scale fused multiply-adds on a register
 * footprint near regs_thr and F * 1000 / r_milli streaming 16-byte loads.
 * Kernels are launched in the given order, one stream per kernel (Section 1:
 * concurrent kernels through streams), and the makespan is the time from the
 * first launch to the last kernel's end, by HIP events. */

/* ko_hw_vgprs — the VGPR count of the compiled variant that stands in for a
 * kernel with regs_thr registers per thread (model the hardware with it). */
int ko_hw_vgprs(int32_t regs_thr, int32_t *vgprs_out);

/* ko_hw_time_orders — makespans (milliseconds, best of `reps` runs) of
 * n_orders orders (int32 [n_orders][n], host) of the n kernels k[] (host) on
 * the current device, into makespan_ms_out[n_orders] (host).  Synchronous;
 * uses a 1 GiB device buffer kept until process exit.  n_tblk <= 2^20,
 * waves_blk <= 16, lds_blk <= 160 KiB.  Errors: KO_EINVAL, KO_EHIP. */
int ko_hw_time_orders(const ko_kernel *k, int32_t n, const int32_t *orders, int32_t n_orders, int32_t scale,
                      int32_t reps, double *makespan_ms_out);

/* ko_hw_last_error — description of the last failure of a ko_hw_* call. */
const char *ko_hw_last_error(void);

/* ko_set_kernel_timing — measurement aid, not part of the method: while enabled
 * (enable != 0), ko_simulate_batch on the current device records two timing
 * events on its stream, immediately before and after the simulate kernel (the
 * makespan evaluation itself: no staging, reduction or histogram).  Enabling
 * or disabling forgets any earlier measurement. */
int ko_set_kernel_timing(int32_t enable);

/* ko_last_kernel_ms — duration in milliseconds of the simulate kernel of the
 * last timed ko_simulate_batch on the current device.  Blocks until that
 * kernel has finished.  KO_EINVAL if ms_out is NULL or no timed launch
 * happened since timing was enabled. */
int ko_last_kernel_ms(float *ms_out);

/* ko_last_error — text of the last failure on this thread; owned by the library,
 * valid until the next call on this thread.  Never NULL. */
const char *ko_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KO_H */
