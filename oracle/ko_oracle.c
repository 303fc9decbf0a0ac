/*
 * CPU ORACLE — test infrastructure, not part of the product path.
 *
 * A plain, slow, deliberately unoptimised reference for the discrete-event
 * model of thread-block dispatch that the HIP library evaluates.  Only the
 * tests, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header or table with the library under
 * paper_1511_07983_amd/.
 *
 * What it computes (Section 2, "Fundamental Concept of Reordering", and
 * Table 1 of Li, Narayana & El-Ghazawi, "Reordering GPU Kernel Launches to
 * Enable Efficient Concurrent Execution", 2015):
 *
 *   - every block of the earliest-issued kernel is placed before any block of
 *     the next kernel (Section 2), and the stream of blocks is never
 *     reordered: if the head block fits nowhere, nothing behind it is placed;
 *   - blocks go to SMs/CUs round-robin: a cyclic pointer, the first CU at or
 *     after it whose free registers, shared memory, warps/waves and block
 *     slots all cover the block (Section 2 and the SM limits of Table 1);
 *   - a block occupies its resources for a fixed number of cycles and then
 *     releases them; all blocks that finish at the same cycle release before
 *     any new placement at that cycle;
 *   - the makespan ("total execution time", abstract and Table 3) is the
 *     cycle at which the last block finishes.
 *
 * Per-block quantities (Table 1 rows for kernel i; the readings are the
 * library's documented ones):
 *   registers  = regs per thread * waves per block * wave size
 *   shared mem = bytes per block
 *   waves      = waves per block
 *   blocks     = 1
 *   duration   = ceil(N_inst * max(R_i, R_B) / R_i) cycles, with R in
 *                thousandths (Section 4: a block below the balanced ratio R_B
 *                is memory bound and stretches by R_B / R_i).
 *
 * All arithmetic is integer; makespans are int64 cycles.
 *
 * Array conventions (all row-major, little-endian int64 unless stated):
 *   gpu[7]    = n_cu, wave_size, wave_cu, blk_cu, reg_cu, lds_cu, rb_milli
 *   kern[n*6] = n_tblk, n_inst, lds_blk, waves_blk, regs_thr, r_milli
 *   order[n]  = int32 kernel index launched at each position
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OC_EINVAL (-1)
#define OC_ENOMEM (-3)

enum { G_NCU, G_WSZ, G_WAVE, G_BLK, G_REG, G_LDS, G_RB };
enum { K_TBLK, K_INST, K_LDS, K_WAVES, K_REGS, K_R };
enum { R_REG, R_LDS, R_WAVE, R_BLK };

/* Per-block usage and duration of each kernel. */
int oc_derive(const int64_t *gpu, int32_t n, const int64_t *kern,
              int64_t *use /* n*4 */, int64_t *dur /* n */)
{
    if (n < 1 || gpu[G_NCU] < 1 || gpu[G_WSZ] < 1 || gpu[G_WAVE] < 1 ||
        gpu[G_BLK] < 1 || gpu[G_REG] < 1 || gpu[G_LDS] < 1 || gpu[G_RB] < 1)
        return OC_EINVAL;
    for (int32_t i = 0; i < n; i++) {
        const int64_t *k = kern + 6 * (int64_t)i;
        if (k[K_TBLK] < 1 || k[K_INST] < 1 || k[K_LDS] < 0 || k[K_WAVES] < 1 ||
            k[K_REGS] < 1 || k[K_R] < 1)
            return OC_EINVAL;
        int64_t ureg = k[K_REGS] * k[K_WAVES] * gpu[G_WSZ];
        int64_t ulds = k[K_LDS];
        int64_t uwave = k[K_WAVES];
        /* a block that does not fit an empty CU can never be placed */
        if (ureg > gpu[G_REG] || ulds > gpu[G_LDS] || uwave > gpu[G_WAVE])
            return OC_EINVAL;
        use[4 * i + R_REG] = ureg;
        use[4 * i + R_LDS] = ulds;
        use[4 * i + R_WAVE] = uwave;
        use[4 * i + R_BLK] = 1;
        int64_t hi = k[K_R] > gpu[G_RB] ? k[K_R] : gpu[G_RB];
        dur[i] = (k[K_INST] * hi + k[K_R] - 1) / k[K_R];
    }
    return 0;
}

typedef struct {
    int64_t fin;
    int32_t cu;
    int32_t k;
} oc_block;

typedef struct {
    int32_t n_cu;
    int64_t cap[4];
    int32_t n;
    const int64_t *use;
    const int64_t *dur;
    const int64_t *tblk;
    /* scratch */
    int64_t *freec;   /* n_cu*4 */
    oc_block *run;    /* n_cu*blk_cu */
} oc_sim;

static int fits(const oc_sim *s, int32_t c, int32_t k)
{
    for (int x = 0; x < 4; x++)
        if (s->freec[4 * c + x] < s->use[4 * k + x])
            return 0;
    return 1;
}

/* Makespan of one launch order under the dispatch model above. */
static int64_t simulate(oc_sim *s, const int32_t *order)
{
    const int32_t N = s->n_cu;
    /* every CU empty, pointer at CU 0, head of the stream = first block
     * of the first kernel in launch order */
    for (int32_t c = 0; c < N; c++)
        for (int x = 0; x < 4; x++)
            s->freec[4 * c + x] = s->cap[x];
    int32_t ptr = 0;
    int32_t pos = 0;                       /* launch position of the head block */
    int64_t left = s->tblk[order[0]];      /* blocks of that kernel not yet placed */
    int64_t nrun = 0;
    int64_t t = 0;

    for (;;) {
        /* place blocks in stream order until the head block fits nowhere */
        while (pos < s->n) {
            int32_t k = order[pos];
            int32_t found = -1;
            for (int32_t i = 0; i < N; i++) {
                int32_t c = (ptr + i) % N;
                if (fits(s, c, k)) {
                    found = c;
                    break;
                }
            }
            if (found < 0)
                break;
            for (int x = 0; x < 4; x++)
                s->freec[4 * found + x] -= s->use[4 * k + x];
            s->run[nrun].fin = t + s->dur[k];
            s->run[nrun].cu = found;
            s->run[nrun].k = k;
            nrun++;
            ptr = (found + 1) % N;
            if (--left == 0) {
                pos++;
                if (pos < s->n)
                    left = s->tblk[order[pos]];
            }
        }
        if (nrun == 0)
            break;
        /* advance to the earliest finish and release every block ending then */
        int64_t tmin = s->run[0].fin;
        for (int64_t b = 1; b < nrun; b++)
            if (s->run[b].fin < tmin)
                tmin = s->run[b].fin;
        t = tmin;
        int64_t keep = 0;
        for (int64_t b = 0; b < nrun; b++) {
            if (s->run[b].fin == t) {
                for (int x = 0; x < 4; x++)
                    s->freec[4 * s->run[b].cu + x] += s->use[4 * s->run[b].k + x];
            } else {
                s->run[keep++] = s->run[b];
            }
        }
        nrun = keep;
    }
    /* the last release time is the makespan */
    return t;
}

static int sim_init(oc_sim *s, const int64_t *gpu, int32_t n, const int64_t *kern,
                    int64_t *use, int64_t *dur, int64_t *tblk)
{
    int rc = oc_derive(gpu, n, kern, use, dur);
    if (rc)
        return rc;
    for (int32_t i = 0; i < n; i++)
        tblk[i] = kern[6 * i + K_TBLK];
    s->n_cu = (int32_t)gpu[G_NCU];
    s->cap[R_REG] = gpu[G_REG];
    s->cap[R_LDS] = gpu[G_LDS];
    s->cap[R_WAVE] = gpu[G_WAVE];
    s->cap[R_BLK] = gpu[G_BLK];
    s->n = n;
    s->use = use;
    s->dur = dur;
    s->tblk = tblk;
    s->freec = (int64_t *)malloc(sizeof(int64_t) * 4 * (size_t)s->n_cu);
    s->run = (oc_block *)malloc(sizeof(oc_block) * (size_t)s->n_cu * (size_t)gpu[G_BLK]);
    if (!s->freec || !s->run) {
        free(s->freec);
        free(s->run);
        return OC_ENOMEM;
    }
    return 0;
}

static void sim_free(oc_sim *s)
{
    free(s->freec);
    free(s->run);
}

/* Permutation with lexicographic rank `rank` among all orders of 0..n-1:
 * the factorial-number-system digits pick, position by position, the
 * digit-th smallest index not used yet. */
void oc_unrank(int32_t n, uint64_t rank, int32_t *perm)
{
    int32_t avail[32];
    uint64_t fact[32];
    fact[0] = 1;
    for (int32_t i = 1; i < n; i++)
        fact[i] = fact[i - 1] * (uint64_t)i;
    for (int32_t i = 0; i < n; i++)
        avail[i] = i;
    int32_t m = n;
    for (int32_t p = 0; p < n; p++) {
        uint64_t f = fact[n - 1 - p];
        int32_t digit = (int32_t)(rank / f);
        rank %= f;
        perm[p] = avail[digit];
        for (int32_t j = digit; j < m - 1; j++)
            avail[j] = avail[j + 1];
        m--;
    }
}

/* Lexicographic rank of a permutation of 0..n-1 (inverse of oc_unrank). */
uint64_t oc_rank(int32_t n, const int32_t *perm)
{
    uint64_t r = 0;
    for (int32_t p = 0; p < n; p++) {
        uint64_t smaller = 0;
        for (int32_t q = p + 1; q < n; q++)
            if (perm[q] < perm[p])
                smaller++;
        r = r * (uint64_t)(n - p) + smaller;
    }
    return r;
}

int64_t oc_makespan(const int64_t *gpu, int32_t n, const int64_t *kern, const int32_t *order)
{
    int64_t use[4 * 32], dur[32], tblk[32];
    if (n < 1 || n > 32)
        return OC_EINVAL;
    /* the order must be a permutation */
    int seen[32] = {0};
    for (int32_t p = 0; p < n; p++) {
        if (order[p] < 0 || order[p] >= n || seen[order[p]])
            return OC_EINVAL;
        seen[order[p]] = 1;
    }
    oc_sim s;
    int rc = sim_init(&s, gpu, n, kern, use, dur, tblk);
    if (rc)
        return rc;
    int64_t m = simulate(&s, order);
    sim_free(&s);
    return m;
}

/* ---- many orders, split over threads in contiguous chunks ---- */

typedef struct {
    const int64_t *gpu, *kern;
    int32_t n;
    int32_t mode;           /* 0: ranks lo+i, 1: explicit ranks, 2: explicit orders */
    uint64_t lo;
    const uint64_t *ranks;
    const int32_t *orders;
    int64_t begin, end;
    int64_t *out;
    int rc;
} oc_job;

static void *run_job(void *arg)
{
    oc_job *j = (oc_job *)arg;
    int64_t use[4 * 32], dur[32], tblk[32];
    int32_t perm[32];
    oc_sim s;
    j->rc = sim_init(&s, j->gpu, j->n, j->kern, use, dur, tblk);
    if (j->rc)
        return NULL;
    for (int64_t i = j->begin; i < j->end; i++) {
        const int32_t *ord = perm;
        if (j->mode == 0)
            oc_unrank(j->n, j->lo + (uint64_t)i, perm);
        else if (j->mode == 1)
            oc_unrank(j->n, j->ranks[i], perm);
        else
            ord = j->orders + (int64_t)j->n * i;
        j->out[i] = simulate(&s, ord);
    }
    sim_free(&s);
    return NULL;
}

static int run_many(oc_job base, int64_t count, int32_t threads)
{
    if (base.n < 1 || base.n > 20)
        return OC_EINVAL;
    if (threads < 1)
        threads = 1;
    if (threads > 256)
        threads = 256;
    if (count < threads)
        threads = count > 0 ? (int32_t)count : 1;
    oc_job jobs[256];
    pthread_t tid[256];
    for (int32_t t = 0; t < threads; t++) {
        jobs[t] = base;
        jobs[t].begin = count * t / threads;
        jobs[t].end = count * (t + 1) / threads;
    }
    if (threads == 1) {
        run_job(&jobs[0]);
        return jobs[0].rc;
    }
    int32_t started = 0;
    for (int32_t t = 0; t < threads; t++) {
        if (pthread_create(&tid[t], NULL, run_job, &jobs[t]) != 0)
            break;
        started++;
    }
    for (int32_t t = 0; t < started; t++)
        pthread_join(tid[t], NULL);
    for (int32_t t = started; t < threads; t++)
        run_job(&jobs[t]);
    for (int32_t t = 0; t < threads; t++)
        if (jobs[t].rc)
            return jobs[t].rc;
    return 0;
}

/* Makespans of the orders with lexicographic ranks lo .. lo+count-1. */
int oc_makespans_range(const int64_t *gpu, int32_t n, const int64_t *kern, uint64_t lo,
                       int64_t count, int64_t *out, int32_t threads)
{
    oc_job b = {gpu, kern, n, 0, lo, NULL, NULL, 0, 0, out, 0};
    return run_many(b, count, threads);
}

/* Makespans of the orders with the given lexicographic ranks. */
int oc_makespans_ranks(const int64_t *gpu, int32_t n, const int64_t *kern, const uint64_t *ranks,
                       int64_t count, int64_t *out, int32_t threads)
{
    oc_job b = {gpu, kern, n, 1, 0, ranks, NULL, 0, 0, out, 0};
    return run_many(b, count, threads);
}

/* Makespans of explicit orders (count rows of n int32 kernel indices). */
int oc_makespans_orders(const int64_t *gpu, int32_t n, const int64_t *kern, const int32_t *orders,
                        int64_t count, int64_t *out, int32_t threads)
{
    if (n < 1 || n > 20)
        return OC_EINVAL;
    for (int64_t i = 0; i < count; i++) {
        int seen[32] = {0};
        for (int32_t p = 0; p < n; p++) {
            int32_t k = orders[(int64_t)n * i + p];
            if (k < 0 || k >= n || seen[k])
                return OC_EINVAL;
            seen[k] = 1;
        }
    }
    oc_job b = {gpu, kern, n, 2, 0, NULL, orders, 0, 0, out, 0};
    return run_many(b, count, threads);
}

/* ---- round-synchronous reading of the execution rounds (Section 2) ----
 *
 * Section 2 describes the blocks of a kernel set as split into execution
 * rounds that run one after another.  In this second model a round is
 * closed as soon as the head block of the stream fits on no CU; the next
 * round starts only when every block of the closed round has finished, so
 * each round lasts as long as its longest block, and the makespan is the
 * sum of the round lengths.  Placement inside a round is the one above
 * (stream order, cyclic pointer, first CU that fits); the pointer carries
 * over from one round to the next.  Blocks never release resources in the
 * middle of a round. */
static int64_t simulate_rounds(oc_sim *s, const int32_t *order)
{
    const int32_t N = s->n_cu;
    for (int32_t c = 0; c < N; c++)
        for (int x = 0; x < 4; x++)
            s->freec[4 * c + x] = s->cap[x];
    int32_t ptr = 0;
    int32_t pos = 0;
    int64_t left = s->tblk[order[0]];
    int64_t t = 0;          /* start of the open round */
    int64_t longest = 0;    /* longest block placed in the open round */

    while (pos < s->n) {
        int32_t k = order[pos];
        int32_t found = -1;
        for (int32_t i = 0; i < N; i++) {
            int32_t c = (ptr + i) % N;
            if (fits(s, c, k)) {
                found = c;
                break;
            }
        }
        if (found < 0) {
            /* close the round: wait for all of its blocks, free every CU */
            if (longest == 0)
                return OC_EINVAL;   /* cannot happen for derived kernels */
            t += longest;
            longest = 0;
            for (int32_t c = 0; c < N; c++)
                for (int x = 0; x < 4; x++)
                    s->freec[4 * c + x] = s->cap[x];
            continue;
        }
        for (int x = 0; x < 4; x++)
            s->freec[4 * found + x] -= s->use[4 * k + x];
        if (s->dur[k] > longest)
            longest = s->dur[k];
        ptr = (found + 1) % N;
        if (--left == 0) {
            pos++;
            if (pos < s->n)
                left = s->tblk[order[pos]];
        }
    }
    return t + longest;
}

/* Round-synchronous makespans of `count` explicit orders (orders[count*n],
 * each a permutation of 0..n-1). */
int oc_rounds_makespans(const int64_t *gpu, int32_t n, const int64_t *kern, const int32_t *orders,
                        int64_t count, int64_t *out)
{
    int64_t use[4 * 32], dur[32], tblk[32];
    if (n < 1 || n > 32 || count < 0)
        return OC_EINVAL;
    for (int64_t j = 0; j < count; j++) {
        int seen[32] = {0};
        const int32_t *o = orders + j * n;
        for (int32_t p = 0; p < n; p++) {
            if (o[p] < 0 || o[p] >= n || seen[o[p]])
                return OC_EINVAL;
            seen[o[p]] = 1;
        }
    }
    oc_sim s;
    int rc = sim_init(&s, gpu, n, kern, use, dur, tblk);
    if (rc)
        return rc;
    for (int64_t j = 0; j < count; j++) {
        out[j] = simulate_rounds(&s, orders + j * n);
        if (out[j] < 0) {
            rc = (int)out[j];
            break;
        }
    }
    sim_free(&s);
    return rc;
}

/* ---- memory-bandwidth contention between resident blocks (Section 4) ----
 *
 * Section 4 asks that the blocks running together balance instructions
 * against memory accesses, because R_B, the GPU's balanced
 * instruction/memory ratio, is a property of the whole chip.  This third
 * model lets the resident blocks share the chip's memory throughput:
 *
 *   - mem_blocks = B is how many memory-bound blocks the chip's memory
 *     system serves at their full (isolated) speed at once;
 *   - a block of kernel i alone keeps the memory system busy for the share
 *     u_i = min(R_i, R_B) / R_i of its duration (1 for a memory-bound kernel,
 *     R_B / R_i for a compute-bound one), counted in units of 1/1024 and
 *     rounded up: uq_i = ceil(1024 * min(r_i, r_B) / r_i);
 *   - while the resident blocks' shares add up to U (units of 1/1024) and U
 *     exceeds 1024 * B, every resident block runs slower by the same factor:
 *     per cycle it completes rate = floor(65536 * 1024 * B / U) units of
 *     progress, where an isolated cycle is 65536 units (rate = 65536 when
 *     U <= 1024 * B);
 *   - a block of kernel i needs d_i * 65536 units of progress; it ends at the
 *     first whole cycle at which its progress is complete; all blocks ending
 *     at a cycle release before placement resumes, as in the first model.
 * Placement is the first model's.  With B large enough that U never exceeds
 * 1024 * B, every makespan equals the first model's. */

#define OC_UNIT 65536LL
#define OC_SHARE 1024LL

typedef struct {
    int64_t target;   /* progress at which the block ends */
    int32_t cu;
    int32_t k;
} oc_cblock;

static int64_t contended_rate(int64_t used, int64_t mem_blocks)
{
    const int64_t cap = OC_SHARE * mem_blocks;
    return used <= cap ? OC_UNIT : (OC_UNIT * cap) / used;
}

static int64_t simulate_contended(oc_sim *s, const int32_t *order, const int64_t *share,
                                  int64_t mem_blocks, oc_cblock *run)
{
    const int32_t N = s->n_cu;
    for (int32_t c = 0; c < N; c++)
        for (int x = 0; x < 4; x++)
            s->freec[4 * c + x] = s->cap[x];
    int32_t ptr = 0;
    int32_t pos = 0;
    int64_t left = s->tblk[order[0]];
    int64_t nrun = 0;
    int64_t t = 0;
    int64_t progress = 0;  /* progress of every resident block since t = 0 */
    int64_t used = 0;      /* sum of the resident blocks' shares */

    for (;;) {
        while (pos < s->n) {
            int32_t k = order[pos];
            int32_t found = -1;
            for (int32_t i = 0; i < N; i++) {
                int32_t c = (ptr + i) % N;
                if (fits(s, c, k)) {
                    found = c;
                    break;
                }
            }
            if (found < 0)
                break;
            for (int x = 0; x < 4; x++)
                s->freec[4 * found + x] -= s->use[4 * k + x];
            run[nrun].target = progress + s->dur[k] * OC_UNIT;
            run[nrun].cu = found;
            run[nrun].k = k;
            nrun++;
            used += share[k];
            ptr = (found + 1) % N;
            if (--left == 0) {
                pos++;
                if (pos < s->n)
                    left = s->tblk[order[pos]];
            }
        }
        if (nrun == 0)
            break;
        /* the block with the least progress left ends first; whole cycles */
        int64_t tmin = run[0].target;
        for (int64_t b = 1; b < nrun; b++)
            if (run[b].target < tmin)
                tmin = run[b].target;
        const int64_t rate = contended_rate(used, mem_blocks);
        const int64_t dt = (tmin - progress + rate - 1) / rate;
        t += dt;
        progress += dt * rate;
        int64_t keep = 0;
        for (int64_t b = 0; b < nrun; b++) {
            if (run[b].target <= progress) {
                for (int x = 0; x < 4; x++)
                    s->freec[4 * run[b].cu + x] += s->use[4 * run[b].k + x];
                used -= share[run[b].k];
            } else {
                run[keep++] = run[b];
            }
        }
        nrun = keep;
    }
    return t;
}

/* Memory shares (units of 1/1024) of the kernels, as defined above. */
static void contended_shares(const int64_t *gpu, int32_t n, const int64_t *kern, int64_t *share)
{
    for (int32_t i = 0; i < n; i++) {
        const int64_t r = kern[6 * i + K_R];
        const int64_t lo = r < gpu[G_RB] ? r : gpu[G_RB];
        share[i] = (OC_SHARE * lo + r - 1) / r;
    }
}

/* Contended makespans of `count` explicit orders (orders[count*n]), or, when
 * orders is NULL, of the orders with lexicographic ranks lo .. lo+count-1.
 * mem_blocks >= 1. */
int oc_contended_makespans(const int64_t *gpu, int64_t mem_blocks, int32_t n, const int64_t *kern,
                           const int32_t *orders, uint64_t lo, int64_t count, int64_t *out)
{
    int64_t use[4 * 32], dur[32], tblk[32], share[32];
    int32_t perm[32];
    if (n < 1 || n > 20 || count < 0 || mem_blocks < 1 || mem_blocks > (1LL << 24))
        return OC_EINVAL;
    if (orders) {
        for (int64_t j = 0; j < count; j++) {
            int seen[32] = {0};
            const int32_t *o = orders + j * n;
            for (int32_t p = 0; p < n; p++) {
                if (o[p] < 0 || o[p] >= n || seen[o[p]])
                    return OC_EINVAL;
                seen[o[p]] = 1;
            }
        }
    }
    oc_sim s;
    int rc = sim_init(&s, gpu, n, kern, use, dur, tblk);
    if (rc)
        return rc;
    contended_shares(gpu, n, kern, share);
    oc_cblock *run = (oc_cblock *)malloc(sizeof(oc_cblock) * (size_t)s.n_cu * (size_t)gpu[G_BLK]);
    if (!run) {
        sim_free(&s);
        return OC_ENOMEM;
    }
    for (int64_t j = 0; j < count; j++) {
        const int32_t *o = orders ? orders + j * n : perm;
        if (!orders)
            oc_unrank(n, lo + (uint64_t)j, perm);
        out[j] = simulate_contended(&s, o, share, mem_blocks, run);
    }
    free(run);
    sim_free(&s);
    return 0;
}
