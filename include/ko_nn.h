/*
 * ko_nn.h — the learned launch-order surrogate on MI355X (gfx950), libko_nn.so.
 *
 * A set-plus-position network predicts the makespan of a launch order of a
 * kernel set (normalised by the set's area lower bound), so that search can
 * rank far more orders than it can simulate exactly; every order it proposes
 * is re-simulated exactly by libko.  The kernels and launch positions are
 * those of the paper's Table 1 and Algorithm 1 (Li, Narayana & El-Ghazawi,
 * 2015); the network itself is this library's addition.
 *
 * Network (each kernel of a sample is one token of 32 inputs: 8 features, the
 * one-hot of its launch position among 16 positions plus an "unplaced" slot
 * for partial orders, 7 zeros):
 *   Z1 = X W1^T + b1 per token (32->256); S = sum over tokens of relu(Z1);
 *   A2 = relu(S W2^T + b2); A3 = relu(A2 W3^T + b3) (256->256 each);
 *   y = A3 . w4 + b4.   Loss: mean squared error against targets t.
 * Products run on BF16 MFMA operands (X, weights, S, A2, A3 and, backward,
 * dZ1..dZ3) with float32 accumulation; everything else is float32; Adam
 * updates float32 master weights and refreshes their BF16 copies.
 *
 * Conventions as in ko.h: 0 = KO_OK or a negative KO_E* code; "device"
 * pointers are HIP allocations on the current device owned by the caller;
 * all device calls are stream-ordered and asynchronous unless stated.
 */
#ifndef KO_NN_H
#define KO_NN_H

#include <stddef.h>
#include <stdint.h>

#include "ko.h"

#ifdef __cplusplus
extern "C" {
#endif

#define KO_NN_FEAT 8
#define KO_NN_POS 17      /* 16 launch positions + "unplaced" (16) */
#define KO_NN_UNPLACED 16
#define KO_NN_IN 32
#define KO_NN_HID 256
#define KO_NN_MAX_TOKENS 16

/* Number of float parameters, in this order: W1[256][32], b1[256], W2[256][256],
 * b2[256], W3[256][256], b3[256], w4[256], b4[1]  (140289). */
size_t ko_nn_num_params(void);

/* Bytes of the device state block: float32 master weights, gradients, Adam
 * first and second moments, and BF16 working copies. */
size_t ko_nn_state_bytes(void);

/* Bytes of device workspace for a batch of B samples of n tokens. */
size_t ko_nn_work_bytes(int32_t B, int32_t n);

/* ko_nn_load — set the master weights from host float params[ko_nn_num_params()],
 * zero gradients and Adam moments, refresh the BF16 copies.  Synchronous. */
int ko_nn_load(void *state_dev, const float *params_host, void *hip_stream);

/* ko_nn_read — copy master weights (which = 0), gradients (1) or Adam's first
 * (2) or second (3) moments to host float out[ko_nn_num_params()].  Synchronous. */
int ko_nn_read(const void *state_dev, int32_t which, float *out_host, void *hip_stream);

/* ko_nn_features — the 8 per-kernel features (host).  out[n][8]:
 *   log2(N_tblk)/16, waves/wave_cu, regs/reg_cu, lds/lds_cu (per block),
 *   log2(block cycles)/32, log2(R/R_B)/8, occ/blk_cu, log2(1 + N_tblk/(occ N_CU))/8,
 * with occ the blocks of the kernel alone that fit one CU.  Errors: KO_EINVAL. */
int ko_nn_features(const ko_gpu_model *gpu, const ko_kernel *k, int32_t n, float *out_host);

/* ko_nn_lower_bound — the set's area lower bound on any order's makespan (host):
 * max(max_i d_i, max over resources x of ceil(sum_i N_tblk_i d_i u_x,i / (N_CU cap_x))). */
int ko_nn_lower_bound(const ko_gpu_model *gpu, const ko_kernel *k, int32_t n, int64_t *lb_out);

/* ko_nn_tokens — build BF16 tokens x[B][n][32] for B samples.  Sample b reads
 * row r = rows[b] (int64, device; NULL = b) of the sample tables: the set
 * set_of[r] (int32, device; NULL = set 0) and the launch position of each of
 * its kernels pos[r][n] (uint8, device; 0..15, 16 = unplaced); features come
 * from feat[set][n][8] (float32, device).  The row map lets a training loop
 * draw shuffled minibatches from set-major sample tables without copying them. */
int ko_nn_tokens(const float *feat_dev, const int32_t *set_of_dev, const uint8_t *pos_dev,
                 const int64_t *rows_dev, int32_t B, int32_t n, uint16_t *x_dev, void *hip_stream);

/* ko_nn_targets — training targets t[b] = (makespan[r] - center[s]) / scale[s]
 * (float32, device) with r = rows[b] (NULL = b) and s = set_of[r] (NULL = 0):
 * exact int64 makespans (device) shifted and scaled per set by center[s] and
 * scale[s] (int64, device; scale > 0), e.g. the set's best sampled makespan
 * and its area lower bound (ko_nn_lower_bound). */
int ko_nn_targets(const int64_t *makespans_dev, const int32_t *set_of_dev, const int64_t *center_dev,
                  const int64_t *scale_dev, const int64_t *rows_dev, int32_t B, float *t_dev,
                  void *hip_stream);

/* ko_nn_within_set_ranks — for values[n_sets][per_set] (int64, device; e.g.
 * the exact makespans of each set's sampled orders), ranks[s][i] (int64,
 * device) = position of sample i when set s is sorted by (value, i).  With
 * ko_nn_targets (centre 0, scale per_set) this gives rank-quantile targets,
 * which train the scorer on the order of a set's samples rather than on
 * cycles.  per_set <= 8192; a set's values must span less than 2^51. */
int ko_nn_within_set_ranks(const int64_t *values_dev, int32_t n_sets, int32_t per_set, int64_t *ranks_dev,
                           void *hip_stream);

/* ko_nn_forward — y[B] (float32, device) for tokens x[B][n][32].  1 <= n <= 16. */
int ko_nn_forward(const void *state_dev, const uint16_t *x_dev, int32_t B, int32_t n, float *y_dev,
                  void *work_dev, void *hip_stream);

/* ko_nn_backward — forward, loss and gradients (kept in the state block) for
 * targets t[B] (float32, device); loss_dev (float32[1], device, nullable). */
int ko_nn_backward(void *state_dev, const uint16_t *x_dev, const float *t_dev, int32_t B, int32_t n,
                   float *loss_dev, void *work_dev, void *hip_stream);

/* ko_nn_adam — one Adam step (bias-corrected, step >= 1) on the stored gradients.
 * The bias corrections 1 - beta^step are evaluated on the device, as in
 * ko_nn_train_step, so the two give the same weights for the same step and rate. */
int ko_nn_adam(void *state_dev, int32_t step, float lr, float beta1, float beta2, float eps,
               void *hip_stream);

/* Adam's hyper-parameters and rate schedule, kept in device memory so that a
 * training step reads them without the host and a captured step can be
 * replayed.  The rate of step s is lr s / warmup while s <= warmup, then
 * lr (lr_final + (1 - lr_final) (1 + cos(pi p)) / 2) with
 * p = (s - warmup) / max(1, total - warmup). */
typedef struct ko_nn_sched {
    int32_t step;      /* Adam steps taken so far; a training step takes step + 1 and stores it */
    int32_t warmup;    /* steps of linear warm-up (0 = none) */
    int32_t total;     /* the step at which the cosine reaches lr * lr_final */
    int32_t per_epoch; /* minibatches per pass over the sample rows (ko_nn_batch), >= 1 */
    float lr;          /* peak rate */
    float lr_final;    /* final rate as a fraction of lr (1 = constant rate after warm-up) */
    float beta1, beta2, eps;
    int32_t reserved[3];
} ko_nn_sched;

/* ko_nn_train_step — one training step on the device: forward, loss (loss_dev,
 * float32[1], nullable), gradients (kept in the state block, equal bit for
 * bit to ko_nn_backward's) and Adam on them with step sched->step + 1 and the
 * schedule's rate, after which sched->step holds that step.  13 launches on
 * hip_stream: no host synchronisation, no allocation and no memset, so a
 * stream capture of it replays as a training step (see ko_nn_step_capture).
 * sched_dev: device ko_nn_sched.  Errors: KO_EINVAL. */
int ko_nn_train_step(void *state_dev, const uint16_t *x_dev, const float *t_dev, int32_t B, int32_t n,
                     ko_nn_sched *sched_dev, float *loss_dev, void *work_dev, void *hip_stream);

/* ko_nn_batch — a step's minibatch chosen on the device: sample b is row
 * r = perm[(sched->step mod sched->per_epoch) B + b] (perm: int64, device, at
 * least per_epoch B entries), with the tokens of ko_nn_tokens and the targets
 * of ko_nn_targets for that row (x[B][n][32], t[B]).  Run before
 * ko_nn_train_step, it takes the steps' minibatches in the order of perm. */
int ko_nn_batch(const float *feat_dev, const int32_t *set_of_dev, const uint8_t *pos_dev,
                const int64_t *makespans_dev, const int64_t *center_dev, const int64_t *scale_dev,
                const int64_t *perm_dev, const ko_nn_sched *sched_dev, int32_t B, int32_t n, uint16_t *x_dev,
                float *t_dev, void *hip_stream);

/* An instantiated HIP graph of ko_nn_batch followed by ko_nn_train_step. */
typedef struct ko_nn_graph ko_nn_graph;

/* ko_nn_step_capture — capture ko_nn_batch + ko_nn_train_step with these
 * arguments on hip_stream (a created stream, not the null stream).  Each
 * replay is one training step on the next minibatch: the schedule's step
 * advances on the device.  The graph holds every address given: they must
 * outlive it; a caller that rewrites perm (a new pass) does so between
 * replays, on the replay stream.  Errors: KO_EINVAL, KO_EHIP. */
int ko_nn_step_capture(void *state_dev, const float *feat_dev, const int32_t *set_of_dev, const uint8_t *pos_dev,
                       const int64_t *makespans_dev, const int64_t *center_dev, const int64_t *scale_dev,
                       const int64_t *perm_dev, ko_nn_sched *sched_dev, int32_t B, int32_t n, uint16_t *x_dev,
                       float *t_dev, float *loss_dev, void *work_dev, void *hip_stream, ko_nn_graph **out);

/* ko_nn_graph_launch — replay a captured step on hip_stream. */
int ko_nn_graph_launch(ko_nn_graph *graph, void *hip_stream);

/* ko_nn_graph_destroy — wait for the device, free the graph (NULL is a no-op). */
int ko_nn_graph_destroy(ko_nn_graph *graph);

/* ko_nn_layer1_table — the first layer of one set, tabulated for scoring:
 * table[i][p][256] (float32, device, n*17*256 floats) = relu of the first
 * layer's output for kernel i (features feat[n][8], float32, device) at
 * launch position p (0..15, 16 = unplaced).  Because a token is its kernel's
 * features plus a one-hot position, this equals the token path's per-token
 * activation (up to float32 summation order). */
int ko_nn_layer1_table(const void *state_dev, const float *feat_dev, int32_t n, float *table_dev,
                       void *hip_stream);

/* Bytes of device workspace for ko_nn_forward_positions on B samples. */
size_t ko_nn_score_work_bytes(int32_t B);

/* ko_nn_forward_positions — y[B] (float32, device) for B orders of one set
 * given as positions pos[B][n] (uint8, device: position of kernel i, 0..15,
 * 16 = unplaced; larger values count as 16), using that set's layer-1 table.
 * The same network as ko_nn_forward without materialising tokens: S is a
 * gather-sum of n table rows, then the two 256x256 BF16 MFMA layers and the
 * output layer.  1 <= n <= 16. */
int ko_nn_forward_positions(const void *state_dev, const float *table_dev, const uint8_t *pos_dev,
                            int32_t B, int32_t n, float *y_dev, void *work_dev, void *hip_stream);

/* ko_nn_score — y[B] (float32, device) for B orders of one set given as
 * positions pos[B][n] (uint8, device: position of kernel i, 0..15, 16 =
 * unplaced; larger values count as 16), from the set's features feat[n][8]
 * (float32, device).  The same values as ko_nn_layer1_table followed by
 * ko_nn_forward_positions, bit for bit, in one kernel that keeps each tile of
 * 64 orders on chip (layer-1 pooling from the features and position weights,
 * both 256x256 BF16 MFMA layers, the output layer): no table, no workspace,
 * no intermediate in memory.  1 <= n <= 16, B >= 1.  Asynchronous on
 * hip_stream.  Errors: KO_EINVAL. */
int ko_nn_score(const void *state_dev, const float *feat_dev, const uint8_t *pos_dev, int32_t B, int32_t n,
                float *y_dev, void *hip_stream);

/* Scoring with the pooling on the matrix cores.  S = sum over kernels of the
 * layer-1 table row of (kernel, position) is the product of each order's
 * one-hot row with the table.  An order of an n-kernel set puts each kernel
 * at a position 0..n-1 or leaves it unplaced, so the table needs n + 1 slots
 * per kernel (slot p for position p < n, slot n for "unplaced").  Carried as
 * two BF16 matrices hi = bf16(T) and lo = bf16(T - hi) (16 significant bits
 * of T), the pooling runs as BF16 MFMA products with float32 accumulation,
 * like the two layers after it.  The result differs from ko_nn_score by that
 * representation of T and the order of the float32 additions (S, like every
 * path's, is then rounded to BF16).
 *
 * ko_nn_split_table_bytes — bytes of the scoring operand pack of a set of n
 * kernels: (2 x 256 x KP + 2 x 256 x 256) BF16 values, KP = n (n + 1)
 * rounded up to a multiple of 32.
 *
 * ko_nn_split_table — the scoring operand pack of one set (features
 * feat[n][8], float32, device) into split (device, 16-byte aligned, owned by
 * the caller): four BF16 matrices one after the other, the split table's
 * high part hi[j][k] and low part lo[j][k] ([256][KP]: hidden unit j, k =
 * (n + 1) i + slot for kernel i, zero from n (n + 1) to KP; from the same
 * first-layer values as ko_nn_layer1_table), then the BF16 copies of W2 and
 * W3 ([256][256]).  Each matrix M[256][32 KS] is stored in MFMA fragment
 * order: element (h, k) at ((h / 16) KS + k / 32) 512 + (16 ((k % 32) / 8) +
 * h % 16) 8 + k % 8, so the 512 values of one 16 x 32 operand fragment are
 * contiguous.  The pack holds a copy of the weights: after they change, make
 * it again.  1 <= n <= 16.  Errors: KO_EINVAL. */
size_t ko_nn_split_table_bytes(int32_t n);
int ko_nn_split_table(const void *state_dev, const float *feat_dev, int32_t n, uint16_t *split_dev,
                      void *hip_stream);

/* ko_nn_score_split — y[B] (float32, device) for B orders of one set given as
 * positions pos[B][n] (uint8, device: 0..n-1, or 16 and above = unplaced),
 * from the set's operand pack (ko_nn_split_table, made with the current
 * weights).  A position in n..15 is no launch position of an n-kernel order:
 * that order's y is NaN.  One kernel per 128-order tile: the one-hot tile in
 * LDS, the pooling product, both 256x256 layers and the output layer, nothing
 * in memory but y.  1 <= n <= 16, B >= 1.  Errors: KO_EINVAL. */
int ko_nn_score_split(const void *state_dev, const uint16_t *split_dev, const uint8_t *pos_dev, int32_t B,
                      int32_t n, float *y_dev, void *hip_stream);

/* ko_nn_score_split_acc — as ko_nn_score_split, but y[b] = scale * score
 * (accumulate = 0) or y[b] + scale * score (accumulate != 0), in the same
 * kernel: the mean score of an ensemble of networks is one call per member
 * with scale = 1 / members, the first without accumulate. */
int ko_nn_score_split_acc(const void *state_dev, const uint16_t *split_dev, const uint8_t *pos_dev, int32_t B,
                          int32_t n, float scale, int32_t accumulate, float *y_dev, void *hip_stream);

/* Beam search over launch orders of one set, one position per step, on the
 * device (the scores come from ko_nn_score on the candidates' positions; the
 * selection of the best candidates is libko's ko_topk_f32).
 *
 * ko_nn_beam_expand — the candidates of one step: prefix w (prefix[W][d],
 * uint8, device: the kernels at positions 0..d-1; NULL when d = 0 and W = 1)
 * grows by each of its n - d unused kernels in increasing index order.
 * Candidate c = w (n - d) + t gets pos[c][n] (uint8, device: position of
 * every kernel, d for the new one, 16 = unplaced) and cand[c] (int32,
 * device) = w << 8 | new kernel.  1 <= n <= 16, 0 <= d < n, W >= 1. */
int ko_nn_beam_expand(const uint8_t *prefix_dev, int32_t W, int32_t d, int32_t n, uint8_t *pos_dev,
                      int32_t *cand_dev, void *hip_stream);

/* ko_nn_beam_cap — diversity rules on a step's scores (score[W][m], float32,
 * device, in place; m = n - d children per prefix): with temperature > 0 each
 * score first gets temperature * G added, G a standard Gumbel variate from
 * SplitMix64 (Steele, Lea & Flood 2014) at counter (seed, candidate index),
 * i.e. -log(-log(u)) with u = (top 24 bits + 0.5) / 2^24; then with cap > 0
 * only the cap lowest scores among each prefix's children are kept (ties by
 * candidate order) and the others become +inf.  Errors: KO_EINVAL. */
int ko_nn_beam_cap(float *score_dev, int32_t W, int32_t m, int32_t cap, float temperature, uint64_t seed,
                   void *hip_stream);

/* ko_nn_beam_gather — the next step's prefixes: out[r][d+1] (uint8, device)
 * = the prefix of candidate idx[r] (int64, device) followed by its new
 * kernel, r < keep.  Errors: KO_EINVAL. */
int ko_nn_beam_gather(const uint8_t *prefix_dev, int32_t d, const int32_t *cand_dev, const int64_t *idx_dev,
                      int32_t keep, uint8_t *out_dev, void *hip_stream);

const char *ko_nn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KO_NN_H */
