// Host side of libko: the C ABI declared in include/ko.h.
//
// Argument validation, per-block derivation of the kernel records, the
// launch-order heuristic (Algorithm 1), order counting, the per-device
// workspace, and the launches of the gfx950 kernels in ko_sim.hip and
// ko_select.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ko.h"
#include "ko_device.h"
#include "ko_rounds.h"
#include "ko_select.h"

namespace {

thread_local std::string g_error = "no error";

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(KO_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define KO_HIP(call, what)                \
    do {                                  \
        hipError_t e_ = (call);           \
        if (e_ != hipSuccess)             \
            return hip_fail(e_, what);    \
    } while (0)

constexpr int64_t kCapLimit = (int64_t(1) << 24) - 1;  // resources must stay exact in float
constexpr int64_t kDurLimit = (int64_t(1) << 31) - 1;
constexpr int64_t kSerialLimit = int64_t(1) << 46;
constexpr uint64_t kSampleLimit = uint64_t(1) << 40;     // samples per set in SAMPLED mode
constexpr uint64_t kSampleSetLimit = uint64_t(1) << 24;  // sets in SAMPLED mode

// ---------------------------------------------------------------- validation

int check_gpu(const ko_gpu_model *g)
{
    if (!g)
        return fail(KO_EINVAL, "gpu model is NULL");
    if (g->mem_blocks < 0 || g->mem_blocks > (1 << 24))
        return fail(KO_EINVAL, "gpu model: mem_blocks %d outside 0..2^24", g->mem_blocks);
    if (g->n_cu < 1 || g->n_cu > 256)
        return fail(KO_EINVAL, "gpu model: n_cu %d outside 1..256", g->n_cu);
    if (g->wave_size < 1)
        return fail(KO_EINVAL, "gpu model: wave_size must be >= 1");
    if (g->wave_cu < 1 || g->wave_cu > kCapLimit)
        return fail(KO_EINVAL, "gpu model: wave_cu outside 1..2^24-1");
    if (g->blk_cu < 1 || g->blk_cu > 255)
        return fail(KO_EINVAL, "gpu model: blk_cu %d outside 1..255", g->blk_cu);
    if (g->reg_cu < 1 || g->reg_cu > kCapLimit)
        return fail(KO_EINVAL, "gpu model: reg_cu outside 1..2^24-1");
    if (g->lds_cu < 1 || g->lds_cu > kCapLimit)
        return fail(KO_EINVAL, "gpu model: lds_cu outside 1..2^24-1");
    if (g->rb_milli < 1)
        return fail(KO_EINVAL, "gpu model: rb_milli must be >= 1");
    return KO_OK;
}

struct Derived {
    int64_t u_reg, u_lds, u_wave;
    int64_t dur;
};

// Per-block use and duration of one kernel (Table 1; Section 4 for the
// duration: a kernel below the balanced ratio is memory bound and its blocks
// stretch by R_B / R_i).
int derive_kernel(const ko_gpu_model &g, const ko_kernel &k, int idx, Derived *d)
{
    if (k.reserved != 0)
        return fail(KO_EINVAL, "kernel %d: reserved field must be 0", idx);
    if (k.n_tblk < 1 || k.n_tblk > kDurLimit)
        return fail(KO_EINVAL, "kernel %d: n_tblk outside 1..2^31-1", idx);
    if (k.n_inst < 1)
        return fail(KO_EINVAL, "kernel %d: n_inst must be >= 1", idx);
    if (k.lds_blk < 0)
        return fail(KO_EINVAL, "kernel %d: lds_blk must be >= 0", idx);
    if (k.waves_blk < 1 || k.regs_thr < 1 || k.r_milli < 1)
        return fail(KO_EINVAL, "kernel %d: waves_blk, regs_thr and r_milli must be >= 1", idx);
    const __int128 ureg = (__int128)k.regs_thr * k.waves_blk * g.wave_size;
    if (ureg > g.reg_cu || k.lds_blk > g.lds_cu || k.waves_blk > g.wave_cu)
        return fail(KO_EINVAL, "kernel %d: one block does not fit an empty CU", idx);
    const int64_t hi = std::max<int64_t>(k.r_milli, g.rb_milli);
    const __int128 dur = ((__int128)k.n_inst * hi + k.r_milli - 1) / k.r_milli;
    if (dur > kDurLimit)
        return fail(KO_EINVAL, "kernel %d: block duration exceeds 2^31-1 cycles", idx);
    d->u_reg = (int64_t)ureg;
    d->u_lds = k.lds_blk;
    d->u_wave = k.waves_blk;
    d->dur = (int64_t)dur;
    return KO_OK;
}

// 1/u rounded up by three ulps: float(fr) * inv then never falls below fr/u.
float inv_up(int64_t u)
{
    if (u <= 0)
        return 0.0f;
    float f = (float)(1.0 / (double)u);
    for (int i = 0; i < 3; i++)
        f = std::nextafter(f, INFINITY);
    return f;
}

// Memory share of one block of kernel k in 1/1024 units (memory contention,
// include/ko.h): ceil(1024 * min(R_k, R_B) / R_k).
uint32_t memory_share(const ko_gpu_model &g, const ko_kernel &k)
{
    const int64_t lo = std::min<int64_t>(k.r_milli, g.rb_milli);
    return (uint32_t)((1024 * lo + k.r_milli - 1) / k.r_milli);
}

int derive_set(const ko_gpu_model &g, const ko_kernel *k, int32_t n, int32_t first_idx,
               std::vector<ko::KernelRec> *out)
{
    __int128 serial = 0;
    for (int32_t i = 0; i < n; i++) {
        Derived d;
        int rc = derive_kernel(g, k[i], first_idx + i, &d);
        if (rc)
            return rc;
        serial += (__int128)k[i].n_tblk * d.dur;
        ko::KernelRec r;
        r.u_reg = (uint32_t)d.u_reg;
        r.u_lds = (uint32_t)d.u_lds;
        r.u_wave = (uint32_t)d.u_wave;
        r.tblk = (uint32_t)k[i].n_tblk;
        r.inv_reg = inv_up(d.u_reg);
        r.inv_lds = inv_up(d.u_lds);
        r.inv_wave = inv_up(d.u_wave);
        r.dur = (uint32_t)d.dur;
        out->push_back(r);
    }
    if (serial >= kSerialLimit)
        return fail(KO_EINVAL, "set starting at kernel %d: total block time reaches 2^46 cycles",
                    first_idx);
    return KO_OK;
}

uint64_t factorial(int n)
{
    uint64_t f = 1;
    for (int i = 2; i <= n; i++)
        f *= (uint64_t)i;
    return f;
}

int count_orders(const int32_t *off, int32_t n_sets, const ko_order_spec *spec,
                 std::vector<uint64_t> *per_set, uint64_t *total)
{
    if (!off || !spec)
        return fail(KO_EINVAL, "set_offsets and spec must not be NULL");
    if (n_sets < 1)
        return fail(KO_EINVAL, "n_sets must be >= 1");
    if (off[0] != 0)
        return fail(KO_EINVAL, "set_offsets[0] must be 0");
    if (spec->reserved != 0)
        return fail(KO_EINVAL, "spec: reserved field must be 0");
    if (spec->mode < KO_ORDERS_ALL || spec->mode > KO_ORDERS_SAMPLED)
        return fail(KO_EINVAL, "spec: unknown mode %d", spec->mode);
    if (spec->mode == KO_ORDERS_RANK_RANGE && !spec->rank_lo_hi)
        return fail(KO_EINVAL, "spec: RANK_RANGE needs rank_lo_hi");
    if ((spec->mode == KO_ORDERS_EXPLICIT || spec->mode == KO_ORDERS_SAMPLED) &&
        !spec->orders_per_set)
        return fail(KO_EINVAL, "spec: EXPLICIT and SAMPLED need orders_per_set");
    if (spec->mode == KO_ORDERS_SAMPLED && (uint64_t)n_sets > kSampleSetLimit)
        return fail(KO_ERANGE, "spec: SAMPLED takes at most 2^24 sets (got %d)", n_sets);
    per_set->assign(n_sets, 0);
    unsigned __int128 sum = 0;
    for (int32_t s = 0; s < n_sets; s++) {
        const int32_t n = off[s + 1] - off[s];
        if (n < 1 || n > ko::kMaxSet)
            return fail(KO_EINVAL, "set %d has %d kernels (must be 1..%d)", s, n, ko::kMaxSet);
        const uint64_t nf = factorial(n);
        uint64_t c = 0;
        switch (spec->mode) {
        case KO_ORDERS_ALL:
            c = nf;
            break;
        case KO_ORDERS_RANK_RANGE: {
            const uint64_t lo = spec->rank_lo_hi[2 * s], hi = spec->rank_lo_hi[2 * s + 1];
            if (lo > hi || hi > nf)
                return fail(KO_EINVAL, "set %d: rank range [%llu, %llu) outside 0..n!", s,
                            (unsigned long long)lo, (unsigned long long)hi);
            c = hi - lo;
            break;
        }
        default:
            if (spec->orders_per_set[s] < 0)
                return fail(KO_EINVAL, "set %d: negative order count", s);
            c = (uint64_t)spec->orders_per_set[s];
            // a sample's counter is set * 2^40 + index: indices at or past 2^40
            // would repeat another set's stream, sets past 2^24 overflow it
            if (spec->mode == KO_ORDERS_SAMPLED && c > kSampleLimit)
                return fail(KO_ERANGE, "set %d: %llu samples (at most 2^40 per set)", s,
                            (unsigned long long)c);
        }
        (*per_set)[s] = c;
        sum += c;
    }
    if (sum > (unsigned __int128)UINT64_MAX)
        return fail(KO_ERANGE, "total order count exceeds 2^64-1");
    *total = (uint64_t)sum;
    return KO_OK;
}

// ------------------------------------------------------------- Algorithm 1

struct Prof {
    int64_t F[4];  // reg, lds, wave, blk footprints
    double W;      // instruction weight
    double R;      // instruction/memory ratio
};
enum { kReg = 0, kLds = 1, kWaveR = 2, kBlk = 3 };

bool fits(const int64_t cap[4], const Prof &X, const Prof &Y)
{
    for (int x = 0; x < 4; x++)
        if (X.F[x] + Y.F[x] > cap[x])
            return false;
    return true;
}

// ProfileCombine's ratio: the instruction-weighted harmonic mean.
double combined_ratio(const Prof &X, const Prof &Y)
{
    return (X.W + Y.W) / (X.W / X.R + Y.W / Y.R);
}

// ScoreGen for one pair: leftover shared memory, registers and warps (each
// clamped at 0), plus the balance term when R_B lies between the two ratios.
double score(const int64_t cap[4], double rb, const Prof &X, const Prof &Y)
{
    if (!fits(cap, X, Y))
        return 0.0;
    double s = 0.0;
    s += std::max((double)(cap[kLds] - X.F[kLds] - Y.F[kLds]) / (double)cap[kLds], 0.0);
    s += std::max((double)(cap[kReg] - X.F[kReg] - Y.F[kReg]) / (double)cap[kReg], 0.0);
    s += std::max((double)(cap[kWaveR] - X.F[kWaveR] - Y.F[kWaveR]) / (double)cap[kWaveR], 0.0);
    if ((X.R <= rb && rb <= Y.R) || (Y.R <= rb && rb <= X.R)) {
        const double rc = combined_ratio(X, Y);
        s += std::max(1.0 - std::fabs(rc - rb) / rb, 0.0);
    }
    return s;
}

Prof combine(const Prof &X, const Prof &Y)
{
    Prof c;
    for (int x = 0; x < 4; x++)
        c.F[x] = X.F[x] + Y.F[x];
    c.W = X.W + Y.W;
    c.R = combined_ratio(X, Y);
    return c;
}

int heuristic(const ko_gpu_model &g, const ko_kernel *k, int32_t n, uint32_t flags,
              int32_t *order_out, int32_t *round_out)
{
    const int64_t cap[4] = {g.reg_cu, g.lds_cu, (int64_t)g.wave_cu, (int64_t)g.blk_cu};
    const double rb = (double)g.rb_milli / 1000.0;
    std::vector<Prof> P(n);
    for (int32_t i = 0; i < n; i++) {
        Derived d;
        int rc = derive_kernel(g, k[i], i, &d);
        if (rc)
            return rc;
        const int64_t b = (flags & KO_HEUR_PER_BLOCK) ? 1 : (k[i].n_tblk + g.n_cu - 1) / g.n_cu;
        P[i].F[kReg] = b * d.u_reg;
        P[i].F[kLds] = b * d.u_lds;
        P[i].F[kWaveR] = b * d.u_wave;
        P[i].F[kBlk] = b;
        P[i].W = (double)((__int128)b * k[i].n_inst);
        P[i].R = (double)k[i].r_milli / 1000.0;
    }
    // ScoreMatrix over all pairs, computed once
    std::vector<double> S((size_t)n * n, 0.0);
    for (int32_t i = 0; i < n; i++)
        for (int32_t j = i + 1; j < n; j++)
            S[(size_t)i * n + j] = score(cap, rb, P[i], P[j]);

    std::vector<int32_t> remaining(n);
    for (int32_t i = 0; i < n; i++)
        remaining[i] = i;
    int32_t out = 0, round = 0;
    auto emit = [&](const std::vector<int32_t> &members) {
        for (int32_t m : members) {
            order_out[out] = m;
            if (round_out)
                round_out[out] = round;
            out++;
        }
        round++;
    };
    auto erase = [&](int32_t v) {
        remaining.erase(std::find(remaining.begin(), remaining.end(), v));
    };
    while (!remaining.empty()) {
        if (remaining.size() == 1) {
            emit({remaining[0]});
            remaining.clear();
            break;
        }
        // the pair with the highest score; the first in i < j scan order on ties
        int32_t a = -1, b = -1;
        double best = 0.0;
        for (size_t ai = 0; ai < remaining.size(); ai++)
            for (size_t bj = ai + 1; bj < remaining.size(); bj++) {
                const int32_t i = remaining[ai], j = remaining[bj];
                const double s = S[(size_t)i * n + j];
                if (a < 0 || s > best) {
                    a = i;
                    b = j;
                    best = s;
                }
            }
        if (P[b].F[kLds] > P[a].F[kLds])
            std::swap(a, b);  // decreasing shared memory, lower index first on ties
        std::vector<int32_t> members = {a, b};
        erase(a);
        erase(b);
        Prof comb = combine(P[a], P[b]);
        for (;;) {
            int32_t c = -1;
            double cs = 0.0;
            for (int32_t r : remaining) {
                if (!fits(cap, comb, P[r]))
                    continue;
                const double s = score(cap, rb, comb, P[r]);
                if (c < 0 || s > cs) {
                    c = r;
                    cs = s;
                }
            }
            if (c < 0)
                break;
            if (flags & KO_HEUR_FULL_SORT) {
                members.push_back(c);
                std::stable_sort(members.begin(), members.end(), [&](int32_t x, int32_t y) {
                    return P[x].F[kLds] > P[y].F[kLds];
                });
            } else if (P[c].F[kLds] > comb.F[kLds]) {
                members.insert(members.begin(), c);
            } else {
                members.push_back(c);
            }
            comb = combine(comb, P[c]);
            erase(c);
        }
        emit(members);
    }
    return KO_OK;
}

// ---------------------------------------------------------------- workspace

// Device words of a batch: item cursor, items handed from the lane kernel to
// simulate_kernel, cursor over that list, spilled orders, cursor over them,
// status word (last, so that a launch can reset the others alone).
constexpr size_t kCounterWords = 6;
constexpr size_t kStatusWord = 5;

struct Workspace {
    int device = -1;
    bool ready = false;
    int cu_count = 0;
    // device buffers
    ko::KernelRec *krec = nullptr;
    size_t krec_cap = 0;
    ko::SetRec *sets = nullptr;
    size_t sets_cap = 0;
    ko::Partial *partials = nullptr;
    size_t partials_cap = 0;
    uint64_t *block_base = nullptr;
    size_t block_base_cap = 0;
    unsigned long long *counter = nullptr;  // kCounterWords words, see DevTables
    int64_t *scratch_i64 = nullptr;          // rank_percentile: reference makespan
    uint8_t *scratch_order = nullptr;        // rank_percentile: the order
    ko_set_stats *scratch_stats = nullptr;   // rank_percentile: stats
    // pinned host staging
    void *stage = nullptr;
    size_t stage_cap = 0;
    uint32_t *status_host = nullptr;
    ko_set_stats *stats_host = nullptr;
    int64_t *ref_host = nullptr;
    hipEvent_t staged = nullptr;  // after the last upload from `stage`
    hipEvent_t done = nullptr;    // after the last call's work
    bool pending_status = false;
    bool clear_status = false;  // a reported device status must be cleared before the next launch
    // selection: 256 digit counters + 1 cursor (device), their host copy
    // (pinned), and the candidate buffer of a top-k
    unsigned long long *sel_bins = nullptr;
    uint64_t *sel_host = nullptr;
    uint64_t *sel_cand = nullptr;
    size_t sel_cand_cap = 0;
    // radix sort: two (key, index) buffers and the digit counts
    void *sort_buf = nullptr;
    size_t sort_cap = 0;
    // ko_stats_i64: one Partial per workgroup
    ko::Partial *stat_parts = nullptr;
    size_t stat_parts_cap = 0;
    // optional timing of the simulate kernel (ko_set_kernel_timing)
    hipEvent_t sim_begin = nullptr, sim_end = nullptr;
    bool timing = false;
    bool timed = false;  // sim_begin/sim_end bracket a launch made while timing was on
};

std::mutex g_mutex;
std::vector<Workspace> g_ws;

// Grow a workspace buffer.  Kernels of an earlier call may still read the old
// buffer, so the previous call's completion event is awaited before freeing.
int grow_device(hipEvent_t done, void **p, size_t *cap, size_t need)
{
    if (need <= *cap)
        return KO_OK;
    if (*p) {
        hipError_t e = hipEventSynchronize(done);
        if (e != hipSuccess)
            return hip_fail(e, "hipEventSynchronize");
        (void)hipFree(*p);
    }
    *p = nullptr;
    *cap = 0;
    size_t sz = std::max<size_t>(need, 4096);
    hipError_t e = hipMalloc(p, sz);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(KO_ENOMEM, "device allocation of %zu bytes failed: %s", sz, hipGetErrorString(e));
    }
    *cap = sz;
    return KO_OK;
}

int get_workspace(Workspace **out)
{
    int dev = 0;
    KO_HIP(hipGetDevice(&dev), "hipGetDevice");
    if ((int)g_ws.size() <= dev)
        g_ws.resize(dev + 1);
    Workspace &w = g_ws[dev];
    if (!w.ready) {
        w.device = dev;
        KO_HIP(hipDeviceGetAttribute(&w.cu_count, hipDeviceAttributeMultiprocessorCount, dev),
               "hipDeviceGetAttribute");
        KO_HIP(hipMalloc((void **)&w.counter, kCounterWords * sizeof(unsigned long long)), "hipMalloc");
        KO_HIP(hipMalloc((void **)&w.scratch_i64, sizeof(int64_t)), "hipMalloc");
        KO_HIP(hipMalloc((void **)&w.scratch_order, 64), "hipMalloc");
        KO_HIP(hipMalloc((void **)&w.scratch_stats, sizeof(ko_set_stats)), "hipMalloc");
        KO_HIP(hipHostMalloc((void **)&w.status_host, sizeof(uint32_t), hipHostMallocDefault),
               "hipHostMalloc");
        KO_HIP(hipHostMalloc((void **)&w.stats_host, sizeof(ko_set_stats), hipHostMallocDefault),
               "hipHostMalloc");
        KO_HIP(hipHostMalloc((void **)&w.ref_host, sizeof(int64_t), hipHostMallocDefault),
               "hipHostMalloc");
        KO_HIP(hipMemset(w.counter, 0, kCounterWords * sizeof(unsigned long long)), "hipMemset");
        KO_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
        *w.status_host = 0;
        KO_HIP(hipEventCreateWithFlags(&w.staged, hipEventDisableTiming), "hipEventCreate");
        KO_HIP(hipEventCreateWithFlags(&w.done, hipEventDisableTiming), "hipEventCreate");
        KO_HIP(hipMalloc((void **)&w.sel_bins, 257 * sizeof(unsigned long long)), "hipMalloc");
        KO_HIP(hipHostMalloc((void **)&w.sel_host, 257 * sizeof(uint64_t), hipHostMallocDefault),
               "hipHostMalloc");
        KO_HIP(hipEventCreate(&w.sim_begin), "hipEventCreate");
        KO_HIP(hipEventCreate(&w.sim_end), "hipEventCreate");
        KO_HIP(hipEventRecord(w.staged, 0), "hipEventRecord");
        KO_HIP(hipEventRecord(w.done, 0), "hipEventRecord");
        w.ready = true;
    }
    *out = &w;
    return KO_OK;
}

void release_workspace(Workspace &w)
{
    if (!w.ready)
        return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(w.device);
    (void)hipDeviceSynchronize();
    (void)hipFree(w.krec);
    (void)hipFree(w.sets);
    (void)hipFree(w.partials);
    (void)hipFree(w.block_base);
    (void)hipFree(w.counter);
    (void)hipFree(w.scratch_i64);
    (void)hipFree(w.scratch_order);
    (void)hipFree(w.scratch_stats);
    (void)hipHostFree(w.stage);
    (void)hipHostFree(w.status_host);
    (void)hipHostFree(w.stats_host);
    (void)hipHostFree(w.ref_host);
    (void)hipEventDestroy(w.staged);
    (void)hipEventDestroy(w.done);
    (void)hipFree(w.sel_bins);
    (void)hipFree(w.sel_cand);
    (void)hipFree(w.sort_buf);
    (void)hipFree(w.stat_parts);
    (void)hipHostFree(w.sel_host);
    (void)hipEventDestroy(w.sim_begin);
    (void)hipEventDestroy(w.sim_end);
    (void)hipSetDevice(prev);
    w = Workspace();
}

// Device status of earlier calls: the status word is copied to pinned host
// memory at the end of every simulate call; a nonzero value is an error.
int check_status(Workspace &w, bool wait)
{
    if (!w.pending_status)
        return KO_OK;
    if (wait) {
        KO_HIP(hipEventSynchronize(w.done), "hipEventSynchronize");
    } else if (hipEventQuery(w.done) != hipSuccess) {
        return KO_OK;  // still running: reported by a later call
    }
    w.pending_status = false;
    const uint32_t st = *w.status_host;
    if (st)
        w.clear_status = true;
    if (st & ko::kStatusBadOrder)
        return fail(KO_EHIP, "device status: an explicit order was not a permutation");
    if (st)
        return fail(KO_EHIP, "device status: internal inconsistency (0x%x)", st);
    return KO_OK;
}

int stage_upload(Workspace &w, hipStream_t stream, void *dst, const void *src, size_t bytes,
                 size_t stage_off)
{
    std::memcpy((char *)w.stage + stage_off, src, bytes);
    KO_HIP(hipMemcpyAsync(dst, (char *)w.stage + stage_off, bytes, hipMemcpyHostToDevice, stream),
           "hipMemcpyAsync");
    return KO_OK;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

uint64_t pow2_at_least(uint64_t v)
{
    uint64_t p = 1;
    while (p < v)
        p <<= 1;
    return p;
}

// Every check of a batch that needs no device.
int validate_batch(const ko_gpu_model *gpu, const ko_kernel *kernels, const int32_t *set_offsets,
                   int32_t n_sets, const ko_order_spec *spec, const int64_t *makespans_dev,
                   const ko_set_stats *stats_dev, const uint64_t *hist_dev, int32_t n_bins)
{
    int rc = check_gpu(gpu);
    if (rc)
        return rc;
    std::vector<uint64_t> per;
    uint64_t total = 0;
    rc = count_orders(set_offsets, n_sets, spec, &per, &total);
    if (rc)
        return rc;
    if (!kernels)
        return fail(KO_EINVAL, "kernels is NULL");
    if (spec->mode == KO_ORDERS_EXPLICIT && total > 0 && !spec->orders_dev)
        return fail(KO_EINVAL, "spec: EXPLICIT needs orders_dev");
    if (hist_dev) {
        if (!makespans_dev || !stats_dev)
            return fail(KO_EINVAL, "a histogram needs makespans_dev and stats_dev");
        if (n_bins < 1 || n_bins > 65536)
            return fail(KO_EINVAL, "n_bins %d outside 1..65536", n_bins);
    }
    std::vector<ko::KernelRec> tmp;
    for (int32_t s = 0; s < n_sets; s++)
        if ((rc = derive_set(*gpu, kernels + set_offsets[s], set_offsets[s + 1] - set_offsets[s],
                             set_offsets[s], &tmp)))
            return rc;
    return KO_OK;
}

struct BatchPlan {
    std::vector<ko::KernelRec> krec;
    std::vector<uint32_t> share;  // per kernel record, under memory contention only
    std::vector<ko::SetRec> sets;
    std::vector<uint64_t> block_base;
    uint64_t total = 0, n_items = 0, chunk = 0, hist_blocks = 0;
    uint32_t max_n = 0;
    int slots = 1;        // CU slots per lane
    int grid = 1;         // workgroups of the simulate kernel
    int lane_class = 0;   // lane kernel variant (largest set it takes), 0 = simulate_kernel only
    int lane_grid = 0;    // workgroups (one wave each) of the lane kernel
    uint32_t lane_entries = 0;  // group entries per lane, 0 = class default
    uint64_t spill_cap = 1;     // records of spilled orders
};

// Per-batch device memory after the counters: n_items Partials, the list of
// items handed over whole (n_items uint32), their bitmap, and the records of
// spilled orders (at most kSpillCap).
constexpr uint64_t kSpillCap = 1 << 16;

struct ItemArea {
    size_t list_off = 0, bits_off = 0, spill_off = 0, bytes = 0;
    uint64_t bit_words = 0;  // 64-bit words of the bitmap
};

ItemArea item_area(uint64_t n_items, uint64_t spill_cap)
{
    ItemArea r;
    const uint64_t items = std::max<uint64_t>(n_items, 1);
    r.list_off = items * sizeof(ko::Partial);
    r.bits_off = (r.list_off + items * sizeof(uint32_t) + 255) & ~(size_t)255;
    r.bit_words = (items + 63) / 64;
    r.spill_off = (r.bits_off + r.bit_words * 8 + 255) & ~(size_t)255;
    r.bytes = r.spill_off + std::max<uint64_t>(spill_cap, 1) * sizeof(ko::SpillRec);
    return r;
}

constexpr uint64_t kHistPerBlock = 1 << 16;

// ------------------------------------------------------------------ selection

constexpr uint64_t kTopkMax = 16384;         // largest k of ko_topk_f32
constexpr uint64_t kTopkCandidates = 32768;  // values <= the k-th, ties included

// One radix-select pass: count the next 8-bit digit of the keys that match
// `prefix` under `mask`, then fix that digit so that the k-th smallest key
// (1-based `rem` within the class) keeps its place.  Updates prefix, mask and
// rem; *class_count receives the size of the chosen digit's class.
template <typename Launch>
int radix_pass(Workspace &w, hipStream_t stream, uint32_t shift, uint64_t *prefix, uint64_t *mask,
               uint64_t *rem, uint64_t *class_count, Launch launch)
{
    int e = ko::launch_zero_u64((uint64_t *)w.sel_bins, 256, stream);
    if (e)
        return hip_fail((hipError_t)e, "zero digit counters");
    e = launch(*prefix, *mask, shift);
    if (e)
        return hip_fail((hipError_t)e, "radix histogram launch");
    KO_HIP(hipMemcpyAsync(w.sel_host, w.sel_bins, 256 * sizeof(uint64_t), hipMemcpyDeviceToHost, stream),
           "hipMemcpyAsync");
    KO_HIP(hipStreamSynchronize(stream), "hipStreamSynchronize");
    uint64_t cum = 0;
    for (uint32_t d = 0; d < 256; d++) {
        const uint64_t c = w.sel_host[d];
        if (cum + c >= *rem) {
            *prefix |= (uint64_t)d << shift;
            *mask |= (uint64_t)0xFF << shift;
            *rem -= cum;
            *class_count = c;
            return KO_OK;
        }
        cum += c;
    }
    return fail(KO_EHIP, "radix selection lost count (%llu of %llu)", (unsigned long long)cum,
                (unsigned long long)*rem);
}

// The lane kernel packs a CU's free resources into two words (registers
// below 2^23, LDS bytes below 2^18, waves and block slots below 128, CU index
// below 2^8) and takes sets of up to 16 kernels.
// Smallest batch the automatic engine choice sends to the lane engine.
constexpr uint64_t kLaneMinOrders = 8192;

int lane_class_for(const ko_gpu_model &g, uint32_t max_n)
{
    if (g.n_cu > 256 || g.reg_cu >= (1 << 23) || g.lds_cu >= (1 << 18) || g.wave_cu > 127 || g.blk_cu > 127 ||
        max_n > 16)
        return 0;
    return max_n <= 8 ? 8 : (max_n <= 10 ? 10 : (max_n <= 12 ? 12 : 16));
}

int slots_for(int n_cu)
{
    const int s = (n_cu + ko::kWave - 1) / ko::kWave;
    return s == 3 ? 4 : s;
}

// Host half of a batch: derived kernel records, the set table and the work
// decomposition (chunks of consecutive orders per work item, persistent grid
// of wg_per_cu workgroups per CU).  chunk_req = 0 picks the chunk: enough
// items to balance the persistent waves, few enough to keep partials small.
// The chunk grows until whole chunks number at most max_items (each set adds
// one more item at most); the lane engine keeps at most spill_limit records
// of spilled orders.
int make_plan(const ko_gpu_model *gpu, const ko_kernel *kernels, const int32_t *set_offsets,
              int32_t n_sets, const ko_order_spec *spec, int cu_count, uint64_t chunk_req, int wg_per_cu,
              int engine, BatchPlan *plan, uint64_t max_items = uint64_t(1) << 23,
              uint64_t spill_limit = kSpillCap)
{
    std::vector<uint64_t> per_set;
    int rc = count_orders(set_offsets, n_sets, spec, &per_set, &plan->total);
    if (rc)
        return rc;
    plan->krec.reserve(set_offsets[n_sets]);
    for (int32_t s = 0; s < n_sets; s++) {
        const int32_t n = set_offsets[s + 1] - set_offsets[s];
        rc = derive_set(*gpu, kernels + set_offsets[s], n, set_offsets[s], &plan->krec);
        if (rc)
            return rc;
        plan->max_n = std::max<uint32_t>(plan->max_n, (uint32_t)n);
    }
    if (gpu->mem_blocks) {
        plan->share.resize(plan->krec.size());
        for (size_t i = 0; i < plan->share.size(); i++)
            plan->share[i] = memory_share(*gpu, kernels[i]);
    }
    plan->slots = slots_for(gpu->n_cu);
    plan->grid = std::max(1, cu_count * wg_per_cu);
    plan->lane_class = engine == KO_ENGINE_WAVE ? 0 : lane_class_for(*gpu, plan->max_n);
    // a batch too small to fill the lanes finishes sooner with one wavefront
    // per order (one order alone: about 5 us against 0.35 ms for one lane)
    if (engine == KO_ENGINE_AUTO && plan->total < kLaneMinOrders)
        plan->lane_class = 0;
    if (engine == KO_ENGINE_LANES && plan->lane_class == 0)
        return fail(KO_EINVAL, "the lane engine takes sets of at most 16 kernels on at most 256 CUs");
    // one-wave workgroups, at least as many as the chip holds at once (8 to 12
    // per CU at these kernels' register use), never more than there are items
    plan->lane_grid = std::max(1, cu_count * std::min(2 * wg_per_cu, 32));
    uint64_t chunk = chunk_req;
    const bool ranks = spec->mode == KO_ORDERS_ALL || spec->mode == KO_ORDERS_RANK_RANGE;
    if (chunk == 0 && plan->lane_class && ranks) {
        // consecutive ranks: one order per lane per item.  Neighbouring ranks
        // share prefixes, so lanes that start together run similar event
        // sequences in step (measured: n=10 all orders 14.8 ms against 16.6 ms
        // with 2 orders per lane and 18.9 ms with 4; the 4096-set batch alike)
        chunk = 64;
    } else if (chunk == 0 && plan->lane_class) {
        // sampled or given orders are unrelated: up to 4 per lane, so that
        // lanes that finish early take the next one, fewer when that leaves
        // a resident wave without an item (measured: n=12, 4 M sampled orders,
        // 56.8 ms against 65.6 ms with one per lane; n=16, 262,144 orders:
        // 128 per item 43.5 ms, 64: 46.1 ms, 256: 68.1 ms; 1 M orders: 256
        // per item 148 ms, 128: 163 ms)
        const uint64_t waves = (uint64_t)std::max(1, cu_count) * 12;
        chunk = pow2_at_least(std::max<uint64_t>(1, plan->total / waves));
        chunk = std::min<uint64_t>(std::max<uint64_t>(chunk, 64), 256);
    } else if (chunk == 0) {
        // about 8 items per persistent wave; a batch smaller than that gets one
        // order per item, so that every order has a wave of its own (one order
        // is a long serial chain on one wave: tens of microseconds)
        const uint64_t waves = (uint64_t)plan->grid * 4;
        chunk = pow2_at_least(std::max<uint64_t>(1, plan->total / (waves * 8)));
        chunk = std::min<uint64_t>(chunk, 8192);
    }
    if (plan->total / chunk > max_items)
        chunk = pow2_at_least((plan->total + max_items - 1) / max_items);
    plan->chunk = chunk;
    plan->spill_cap =
        plan->lane_class ? std::max<uint64_t>(1, std::min<uint64_t>(plan->total, spill_limit)) : 1;
    uint64_t out_base = 0, item_base = 0, list_base = 0, hist_base = 0;
    plan->sets.resize(n_sets);
    plan->block_base.resize(n_sets + 1);
    for (int32_t s = 0; s < n_sets; s++) {
        ko::SetRec &r = plan->sets[s];
        const int32_t n = set_offsets[s + 1] - set_offsets[s];
        r.n = (uint32_t)n;
        r.kbase = (uint32_t)set_offsets[s];
        r.n_orders = per_set[s];
        r.out_base = out_base;
        r.rank_lo = spec->mode == KO_ORDERS_RANK_RANGE ? spec->rank_lo_hi[2 * s] : 0;
        r.item_base = item_base;
        r.list_base = list_base;
        out_base += per_set[s];
        item_base += (per_set[s] + chunk - 1) / chunk;
        list_base += per_set[s] * (uint64_t)n;
        plan->block_base[s] = hist_base;
        hist_base += (per_set[s] + kHistPerBlock - 1) / kHistPerBlock;
    }
    plan->block_base[n_sets] = hist_base;
    plan->n_items = item_base;
    plan->hist_blocks = hist_base;
    return KO_OK;
}

// Device tables a batch runs on.
struct DevTables {
    const ko::KernelRec *krec;
    const uint32_t *share;  // memory shares per kernel record, or null
    const ko::SetRec *sets;
    const uint64_t *block_base;
    ko::Partial *partials;        // start of the batch's item area (item_area)
    unsigned long long *counter;  // kCounterWords words
};

// Enqueue the device work of a batch on `stream`: cursor (and, when asked,
// status) reset, simulation, per-set reduction, histogram.  Kernel launches
// only (no copies, allocations, memsets or synchronisation), so a caller can
// capture it in a HIP graph.
int enqueue_batch(const DevTables &t, const BatchPlan &p, const ko_gpu_model &gpu, int32_t n_sets,
                  int32_t mode, uint64_t seed, const uint8_t *orders, bool reset_status, const int64_t *ref_dev,
                  int64_t *makespans_dev, ko_set_stats *stats_dev, uint64_t *hist_dev, int32_t n_bins,
                  hipStream_t stream, hipEvent_t sim_begin, hipEvent_t sim_end)
{
    int e = ko::launch_zero_u64((uint64_t *)t.counter, reset_status ? kCounterWords : kStatusWord, stream);
    if (e)
        return hip_fail((hipError_t)e, "zero counters");
    const ItemArea area = item_area(p.n_items, p.spill_cap);
    char *base = reinterpret_cast<char *>(t.partials);
    uint32_t *handed_bits = reinterpret_cast<uint32_t *>(base + area.bits_off);
    ko::SpillRec *spill = reinterpret_cast<ko::SpillRec *>(base + area.spill_off);
    if (p.lane_class && p.n_items > 0) {
        e = ko::launch_zero_u64(reinterpret_cast<uint64_t *>(handed_bits), area.bit_words, stream);
        if (e)
            return hip_fail((hipError_t)e, "zero item bitmap");
    }
    if (p.n_items > 0) {
        ko::SimArgs a;
        a.krec = t.krec;
        a.sets = t.sets;
        a.n_sets = n_sets;
        a.mode = mode;
        a.n_items = p.n_items;
        a.chunk = p.chunk;
        a.seed = seed;
        a.orders = orders;
        a.ref = ref_dev;
        a.makespans = makespans_dev;
        a.partials = t.partials;
        a.item_counter = t.counter;
        a.status = (uint32_t *)(t.counter + kStatusWord);
        a.item_list = nullptr;
        a.item_list_count = nullptr;
        a.ovf_list = reinterpret_cast<uint32_t *>(base + area.list_off);
        a.ovf_count = t.counter + 1;
        a.spill = spill;
        a.spill_count = t.counter + 3;
        a.spill_cap = p.spill_cap;
        a.handed_bits = handed_bits;
        a.n_cu = (uint32_t)gpu.n_cu;
        a.cap_reg = (uint32_t)gpu.reg_cu;
        a.cap_lds = (uint32_t)gpu.lds_cu;
        a.cap_wave = (uint32_t)gpu.wave_cu;
        a.cap_blk = (uint32_t)gpu.blk_cu;
        a.share = gpu.mem_blocks ? t.share : nullptr;
        a.mem_cap = (uint64_t)1024 * (uint64_t)gpu.mem_blocks;
        const int g = (int)std::min<uint64_t>((uint64_t)p.grid, (p.n_items + 3) / 4);
        if (sim_begin)
            KO_HIP(hipEventRecord(sim_begin, stream), "hipEventRecord");
        if (p.lane_class) {
            const int lg = (int)std::min<uint64_t>((uint64_t)p.lane_grid, p.n_items);
            e = ko::launch_simulate_lanes(a, p.lane_class, p.lane_entries, lg, stream);
            if (e)
                return hip_fail((hipError_t)e, "lane kernel launch");
            // orders the lanes spilled, with the wave engine (a short launch
            // that finds no record in the common case)
            const int fg = (int)std::min<uint64_t>((uint64_t)g, 256);
            ko::SimArgs sp = a;
            sp.item_counter = t.counter + 4;
            e = ko::launch_spill(sp, p.slots, p.max_n, fg, stream);
            if (e)
                return hip_fail((hipError_t)e, "spill kernel launch");
            // items handed over whole, again with simulate_kernel (also empty
            // in the common case)
            ko::SimArgs f = a;
            f.item_list = a.ovf_list;
            f.item_list_count = a.ovf_count;
            f.item_counter = t.counter + 2;
            f.ovf_list = nullptr;
            f.ovf_count = nullptr;
            e = ko::launch_simulate(f, p.slots, p.max_n, fg, stream);
            if (e)
                return hip_fail((hipError_t)e, "simulate kernel launch");
        } else {
            e = ko::launch_simulate(a, p.slots, p.max_n, g, stream);
            if (e)
                return hip_fail((hipError_t)e, "simulate kernel launch");
        }
        if (sim_end)
            KO_HIP(hipEventRecord(sim_end, stream), "hipEventRecord");
    }
    if (stats_dev) {
        ko::ReduceArgs r;
        r.sets = t.sets;
        r.n_sets = n_sets;
        r.mode = mode;
        r.chunk = p.chunk;
        r.partials = t.partials;
        r.stats = stats_dev;
        r.ref = ref_dev;
        const bool lanes = p.lane_class && p.n_items > 0;
        r.spill = lanes ? spill : nullptr;
        r.spill_count = lanes ? t.counter + 3 : nullptr;
        r.spill_cap = p.spill_cap;
        r.handed_bits = lanes ? handed_bits : nullptr;
        e = ko::launch_reduce(r, stream);
        if (e)
            return hip_fail((hipError_t)e, "reduce kernel launch");
    }
    if (hist_dev) {
        e = ko::launch_zero_u64(hist_dev, (uint64_t)n_sets * (uint64_t)n_bins, stream);
        if (e)
            return hip_fail((hipError_t)e, "zero histogram");
        ko::HistArgs h;
        h.sets = t.sets;
        h.n_sets = n_sets;
        h.makespans = makespans_dev;
        h.stats = stats_dev;
        h.hist = hist_dev;
        h.n_bins = n_bins;
        h.per_block = kHistPerBlock;
        h.block_base = t.block_base;
        e = ko::launch_hist(h, p.hist_blocks, stream);
        if (e)
            return hip_fail((hipError_t)e, "histogram kernel launch");
    }
    return KO_OK;
}

int simulate_impl(Workspace &w, const ko_gpu_model *gpu, const ko_kernel *kernels,
                  const int32_t *set_offsets, int32_t n_sets, const ko_order_spec *spec,
                  const int64_t *ref_dev, int64_t *makespans_dev, ko_set_stats *stats_dev,
                  uint64_t *hist_dev, int32_t n_bins, hipStream_t stream)
{
    int rc = validate_batch(gpu, kernels, set_offsets, n_sets, spec, makespans_dev, stats_dev,
                            hist_dev, n_bins);
    if (rc)
        return rc;
    BatchPlan plan;
    rc = make_plan(gpu, kernels, set_offsets, n_sets, spec, w.cu_count, 0, 8, KO_ENGINE_AUTO, &plan);
    if (rc)
        return rc;
    rc = check_status(w, false);
    if (rc)
        return rc;

    // device buffers
    // kernel records, then (under memory contention) their shares
    const size_t kbytes = plan.krec.size() * sizeof(ko::KernelRec);
    const size_t sh_off = align256(kbytes);
    const size_t shbytes = plan.share.size() * sizeof(uint32_t);
    const size_t sbytes = plan.sets.size() * sizeof(ko::SetRec);
    const size_t bbytes = plan.block_base.size() * sizeof(uint64_t);
    if ((rc = grow_device(w.done, (void **)&w.krec, &w.krec_cap, sh_off + shbytes)) ||
        (rc = grow_device(w.done, (void **)&w.sets, &w.sets_cap, sbytes)) ||
        (rc = grow_device(w.done, (void **)&w.block_base, &w.block_base_cap, bbytes)) ||
        (rc = grow_device(w.done, (void **)&w.partials, &w.partials_cap,
                          item_area(plan.n_items, plan.spill_cap).bytes)))
        return rc;
    // the previous call on any stream must be done with the workspace
    KO_HIP(hipStreamWaitEvent(stream, w.done, 0), "hipStreamWaitEvent");
    const size_t stage_need = kbytes + shbytes + sbytes + bbytes + 64;
    if (stage_need > w.stage_cap) {
        KO_HIP(hipEventSynchronize(w.staged), "hipEventSynchronize");
        if (w.stage)
            (void)hipHostFree(w.stage);
        w.stage = nullptr;
        w.stage_cap = 0;
        KO_HIP(hipHostMalloc(&w.stage, stage_need * 2, hipHostMallocDefault), "hipHostMalloc");
        w.stage_cap = stage_need * 2;
    } else {
        KO_HIP(hipEventSynchronize(w.staged), "hipEventSynchronize");
    }
    uint32_t *share_dev = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(w.krec) + sh_off);
    if ((rc = stage_upload(w, stream, w.krec, plan.krec.data(), kbytes, 0)) ||
        (rc = stage_upload(w, stream, w.sets, plan.sets.data(), sbytes, kbytes)) ||
        (rc = stage_upload(w, stream, w.block_base, plan.block_base.data(), bbytes, kbytes + sbytes)) ||
        (shbytes && (rc = stage_upload(w, stream, share_dev, plan.share.data(), shbytes, kbytes + sbytes + bbytes))))
        return rc;
    KO_HIP(hipEventRecord(w.staged, stream), "hipEventRecord");

    // the status word is cleared only once a reported status has been seen
    DevTables t{w.krec, shbytes ? share_dev : nullptr, w.sets, w.block_base, w.partials, w.counter};
    const bool timing = w.timing && plan.n_items > 0;
    rc = enqueue_batch(t, plan, *gpu, n_sets, spec->mode, spec->seed, spec->orders_dev, w.clear_status,
                       ref_dev, makespans_dev, stats_dev, hist_dev, n_bins, stream,
                       timing ? w.sim_begin : nullptr, timing ? w.sim_end : nullptr);
    w.clear_status = false;
    if (rc)
        return rc;
    if (timing)
        w.timed = true;
    KO_HIP(hipMemcpyAsync(w.status_host, (const void *)(w.counter + kStatusWord), sizeof(uint32_t),
                          hipMemcpyDeviceToHost, stream),
           "hipMemcpyAsync");
    KO_HIP(hipEventRecord(w.done, stream), "hipEventRecord");
    w.pending_status = true;
    return KO_OK;
}

// Output checks shared by the immediate and the planned path.
int check_outputs(const int64_t *makespans_dev, const ko_set_stats *stats_dev, const uint64_t *hist_dev,
                  int32_t n_bins)
{
    if (hist_dev) {
        if (!makespans_dev || !stats_dev)
            return fail(KO_EINVAL, "a histogram needs makespans_dev and stats_dev");
        if (n_bins < 1 || n_bins > 65536)
            return fail(KO_EINVAL, "n_bins %d outside 1..65536", n_bins);
    }
    return KO_OK;
}

}  // namespace

// ------------------------------------------------- no-allocation entry point
// Device memory of ko_simulate_batch_noalloc: the counters, kernel records,
// set table, histogram bases and work-item area of one batch at a time.  Each
// GPU holds its own copy of the array until the process ends.  In host code
// the name is not a device address: the per-device address comes from
// hipGetSymbolAddress, and only that address is used.
constexpr size_t kStaticScratchBytes = size_t(16) << 20;
constexpr uint64_t kStaticItems = uint64_t(1) << 16;  // whole chunks at most
constexpr uint64_t kStaticSpill = 8192;                // spilled-order records at most
constexpr int kStaticDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

struct StaticScratch {
    void *ptr = nullptr;  // device address of `scratch` on this device
    int cu_count = 0;
};
StaticScratch g_static[kStaticDevices];

// The device's copy of the array, looked up once per device (with it current).
int static_scratch(int dev, StaticScratch **out)
{
    if (dev < 0 || dev >= kStaticDevices)
        return fail(KO_EINVAL, "device %d: the static scratch covers devices 0..%d", dev, kStaticDevices - 1);
    StaticScratch &s = g_static[dev];
    if (!s.ptr) {
        void *p = nullptr;
        KO_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
        if (!p)
            return fail(KO_EHIP, "hipGetSymbolAddress returned a null address");
        KO_HIP(hipDeviceGetAttribute(&s.cu_count, hipDeviceAttributeMultiprocessorCount, dev),
               "hipDeviceGetAttribute");
        s.ptr = p;
    }
    *out = &s;
    return KO_OK;
}

}  // namespace

// A batch prepared once and launched many times (ko_plan_*).
struct ko_plan {
    int device = -1;
    ko_gpu_model gpu{};
    int32_t n_sets = 0;
    int32_t mode = 0;
    uint64_t seed = 0;
    const uint8_t *orders = nullptr;
    BatchPlan plan;
    ko::KernelRec *krec = nullptr;
    uint32_t *share = nullptr;  // inside the krec allocation, under memory contention only
    ko::SetRec *sets = nullptr;
    uint64_t *block_base = nullptr;
    ko::Partial *partials = nullptr;
    unsigned long long *counter = nullptr;
};

struct ko_graph {
    int device = -1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

void free_plan(ko_plan *p)
{
    (void)hipFree(p->krec);
    (void)hipFree(p->sets);
    (void)hipFree(p->block_base);
    (void)hipFree(p->partials);
    (void)hipFree(p->counter);
    delete p;
}

int check_plan_device(const ko_plan *p)
{
    int dev = 0;
    KO_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev != p->device)
        return fail(KO_EINVAL, "the plan was created on device %d, the current device is %d", p->device, dev);
    return KO_OK;
}

}  // namespace

extern "C" {

int ko_heuristic_order(const ko_gpu_model *gpu, const ko_kernel *k, int32_t n, uint32_t flags,
                       int32_t *order_out, int32_t *round_out)
{
    int rc = check_gpu(gpu);
    if (rc)
        return rc;
    if (!k || !order_out)
        return fail(KO_EINVAL, "kernels and order_out must not be NULL");
    if (n < 1 || n > ko::kMaxSet)
        return fail(KO_EINVAL, "n %d outside 1..%d", n, ko::kMaxSet);
    if (flags & ~(KO_HEUR_PER_BLOCK | KO_HEUR_FULL_SORT))
        return fail(KO_EINVAL, "unknown heuristic flags 0x%x", flags);
    try {
        return heuristic(*gpu, k, n, flags, order_out, round_out);
    } catch (const std::bad_alloc &) {
        return fail(KO_ENOMEM, "host allocation failed");
    }
}

int ko_count_orders(const int32_t *set_offsets, int32_t n_sets, const ko_order_spec *spec,
                    uint64_t *per_set_out, uint64_t *total_out)
{
    if (!total_out)
        return fail(KO_EINVAL, "total_out must not be NULL");
    try {
        std::vector<uint64_t> per;
        uint64_t total = 0;
        int rc = count_orders(set_offsets, n_sets, spec, &per, &total);
        if (rc)
            return rc;
        if (per_set_out)
            std::copy(per.begin(), per.end(), per_set_out);
        *total_out = total;
        return KO_OK;
    } catch (const std::bad_alloc &) {
        return fail(KO_ENOMEM, "host allocation failed");
    }
}

int ko_simulate_batch(const ko_gpu_model *gpu, const ko_kernel *kernels, const int32_t *set_offsets,
                      int32_t n_sets, const ko_order_spec *spec, const int64_t *ref_makespan_dev,
                      int64_t *makespans_dev, ko_set_stats *stats_dev, uint64_t *hist_dev,
                      int32_t n_bins, void *hip_stream)
{
    try {
        std::lock_guard<std::mutex> lock(g_mutex);
        Workspace *w = nullptr;
        // validate everything that needs no device before touching the runtime
        int rc = validate_batch(gpu, kernels, set_offsets, n_sets, spec, makespans_dev, stats_dev,
                                hist_dev, n_bins);
        if (rc)
            return rc;
        rc = get_workspace(&w);
        if (rc)
            return rc;
        return simulate_impl(*w, gpu, kernels, set_offsets, n_sets, spec, ref_makespan_dev,
                             makespans_dev, stats_dev, hist_dev, n_bins, (hipStream_t)hip_stream);
    } catch (const std::bad_alloc &) {
        return fail(KO_ENOMEM, "host allocation failed");
    }
}

int ko_simulate_batch_noalloc(const ko_gpu_model *gpu, const ko_kernel *kernels, const int32_t *set_offsets,
                              int32_t n_sets, const ko_order_spec *spec, const int64_t *ref_makespan_dev,
                              int64_t *makespans_dev, ko_set_stats *stats_dev, uint64_t *hist_dev,
                              int32_t n_bins, void *hip_stream)
{
    try {
        // one batch at a time per process: calls never overlap on the array
        std::lock_guard<std::mutex> lock(g_mutex);
        int rc = validate_batch(gpu, kernels, set_offsets, n_sets, spec, makespans_dev, stats_dev, hist_dev,
                                n_bins);
        if (rc)
            return rc;
        int dev = 0;
        KO_HIP(hipGetDevice(&dev), "hipGetDevice");
        StaticScratch *sc = nullptr;
        if ((rc = static_scratch(dev, &sc)))
            return rc;
        BatchPlan plan;
        rc = make_plan(gpu, kernels, set_offsets, n_sets, spec, sc->cu_count, 0, 8, KO_ENGINE_AUTO, &plan,
                       kStaticItems, kStaticSpill);
        if (rc)
            return rc;
        // layout of the array for this batch
        const size_t kbytes = plan.krec.size() * sizeof(ko::KernelRec);
        const size_t sbytes = plan.sets.size() * sizeof(ko::SetRec);
        const size_t bbytes = plan.block_base.size() * sizeof(uint64_t);
        const size_t shbytes = plan.share.size() * sizeof(uint32_t);
        const size_t cnt_off = 0;
        const size_t krec_off = align256(cnt_off + kCounterWords * sizeof(unsigned long long));
        const size_t sh_off = align256(krec_off + kbytes);
        const size_t sets_off = align256(sh_off + shbytes);
        const size_t bb_off = align256(sets_off + sbytes);
        const size_t item_off = align256(bb_off + bbytes);
        const size_t need = item_off + item_area(plan.n_items, plan.spill_cap).bytes;
        if (need > kStaticScratchBytes)
            return fail(KO_ERANGE,
                        "batch needs %zu bytes of device scratch (%zu kernel records, %d sets, %llu work items); "
                        "the static scratch holds %zu",
                        need, plan.krec.size(), n_sets, (unsigned long long)plan.n_items, kStaticScratchBytes);
        char *base = static_cast<char *>(sc->ptr);
        hipStream_t stream = (hipStream_t)hip_stream;
        // a failed copy still waits for the ones enqueued before it: they read
        // host tables that end with this call
        hipError_t ce = hipSuccess;
        if (kbytes)
            ce = hipMemcpyAsync(base + krec_off, plan.krec.data(), kbytes, hipMemcpyHostToDevice, stream);
        if (sbytes && ce == hipSuccess)
            ce = hipMemcpyAsync(base + sets_off, plan.sets.data(), sbytes, hipMemcpyHostToDevice, stream);
        if (ce == hipSuccess)
            ce = hipMemcpyAsync(base + bb_off, plan.block_base.data(), bbytes, hipMemcpyHostToDevice, stream);
        if (shbytes && ce == hipSuccess)
            ce = hipMemcpyAsync(base + sh_off, plan.share.data(), shbytes, hipMemcpyHostToDevice, stream);
        if (ce != hipSuccess) {
            (void)hipStreamSynchronize(stream);
            return hip_fail(ce, "hipMemcpyAsync");
        }
        unsigned long long *counter = reinterpret_cast<unsigned long long *>(base + cnt_off);
        DevTables t{reinterpret_cast<const ko::KernelRec *>(base + krec_off),
                    shbytes ? reinterpret_cast<const uint32_t *>(base + sh_off) : nullptr,
                    reinterpret_cast<const ko::SetRec *>(base + sets_off),
                    reinterpret_cast<const uint64_t *>(base + bb_off), reinterpret_cast<ko::Partial *>(base + item_off),
                    counter};
        // every counter and the status word start at zero in every call
        rc = enqueue_batch(t, plan, *gpu, n_sets, spec->mode, spec->seed, spec->orders_dev, true, ref_makespan_dev,
                           makespans_dev, stats_dev, hist_dev, n_bins, stream, nullptr, nullptr);
        uint32_t status = 0;
        if (!rc)
            ce = hipMemcpyAsync(&status, base + cnt_off + kStatusWord * sizeof(unsigned long long), sizeof(uint32_t),
                                hipMemcpyDeviceToHost, stream);
        // the host tables and `status` must outlive the copies, and the next
        // call must find the array idle
        const hipError_t e = hipStreamSynchronize(stream);
        if (rc)
            return rc;
        if (ce != hipSuccess)
            return hip_fail(ce, "hipMemcpyAsync");
        if (e != hipSuccess)
            return hip_fail(e, "hipStreamSynchronize");
        if (status & ko::kStatusBadOrder)
            return fail(KO_EHIP, "device status: an explicit order was not a permutation");
        if (status)
            return fail(KO_EHIP, "device status: internal inconsistency (0x%x)", status);
        return KO_OK;
    } catch (const std::bad_alloc &) {
        return fail(KO_ENOMEM, "host allocation failed");
    }
}

int ko_plan_create(const ko_gpu_model *gpu, const ko_kernel *kernels, const int32_t *set_offsets,
                   int32_t n_sets, const ko_order_spec *spec, const ko_launch_config *config,
                   ko_plan **out)
{
    try {
        std::lock_guard<std::mutex> lock(g_mutex);
        if (!out)
            return fail(KO_EINVAL, "out must not be NULL");
        *out = nullptr;
        int rc = validate_batch(gpu, kernels, set_offsets, n_sets, spec, nullptr, nullptr, nullptr, 0);
        if (rc)
            return rc;
        uint64_t chunk = 0;
        int wg = 8;
        int engine = KO_ENGINE_AUTO;
        if (config) {
            if (config->engine < KO_ENGINE_AUTO || config->engine > KO_ENGINE_LANES)
                return fail(KO_EINVAL, "config: engine %d unknown", config->engine);
            engine = config->engine;
            if (config->lane_entries < 0 || config->lane_entries > 64)
                return fail(KO_EINVAL, "config: lane_entries %d outside 0..64", config->lane_entries);
            if (config->chunk_log2 < 0 || config->chunk_log2 > 20)
                return fail(KO_EINVAL, "config: chunk_log2 %d outside 0..20", config->chunk_log2);
            if (config->wg_per_cu < 0 || config->wg_per_cu > 64)
                return fail(KO_EINVAL, "config: wg_per_cu %d outside 0..64", config->wg_per_cu);
            if (config->chunk_log2 > 0)
                chunk = uint64_t(1) << config->chunk_log2;
            if (config->wg_per_cu > 0)
                wg = config->wg_per_cu;
        }
        Workspace *w = nullptr;
        if ((rc = get_workspace(&w)))
            return rc;
        ko_plan *p = new ko_plan();
        p->device = w->device;
        p->gpu = *gpu;
        p->n_sets = n_sets;
        p->mode = spec->mode;
        p->seed = spec->seed;
        p->orders = spec->orders_dev;
        rc = make_plan(gpu, kernels, set_offsets, n_sets, spec, w->cu_count, chunk, wg, engine, &p->plan);
        if (rc) {
            delete p;
            return rc;
        }
        if (config && p->plan.lane_class)
            p->plan.lane_entries = std::min<uint32_t>((uint32_t)config->lane_entries,
                                                      ko::lane_entry_max(p->plan.lane_class));
        const size_t kbytes = p->plan.krec.size() * sizeof(ko::KernelRec);
        const size_t sh_off = align256(kbytes);
        const size_t shbytes = p->plan.share.size() * sizeof(uint32_t);
        const size_t sbytes = p->plan.sets.size() * sizeof(ko::SetRec);
        const size_t bbytes = p->plan.block_base.size() * sizeof(uint64_t);
        const size_t pbytes = item_area(p->plan.n_items, p->plan.spill_cap).bytes;
        hipError_t e = hipSuccess;
        if ((e = hipMalloc((void **)&p->krec, std::max<size_t>(sh_off + shbytes, 64))) != hipSuccess ||
            (e = hipMalloc((void **)&p->sets, std::max<size_t>(sbytes, 64))) != hipSuccess ||
            (e = hipMalloc((void **)&p->block_base, std::max<size_t>(bbytes, 64))) != hipSuccess ||
            (e = hipMalloc((void **)&p->partials, pbytes)) != hipSuccess ||
            (e = hipMalloc((void **)&p->counter, kCounterWords * sizeof(unsigned long long))) != hipSuccess) {
            free_plan(p);
            return fail(KO_ENOMEM, "plan device allocation failed: %s", hipGetErrorString(e));
        }
        if (shbytes)
            p->share = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(p->krec) + sh_off);
        if ((kbytes && (e = hipMemcpy(p->krec, p->plan.krec.data(), kbytes, hipMemcpyHostToDevice)) != hipSuccess) ||
            (shbytes && (e = hipMemcpy(p->share, p->plan.share.data(), shbytes, hipMemcpyHostToDevice)) != hipSuccess) ||
            (sbytes && (e = hipMemcpy(p->sets, p->plan.sets.data(), sbytes, hipMemcpyHostToDevice)) != hipSuccess) ||
            (e = hipMemcpy(p->block_base, p->plan.block_base.data(), bbytes, hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemset(p->counter, 0, kCounterWords * sizeof(unsigned long long))) != hipSuccess ||
            (e = hipDeviceSynchronize()) != hipSuccess) {
            free_plan(p);
            return hip_fail(e, "plan upload");
        }
        // the host copies are no longer needed
        p->plan.krec = std::vector<ko::KernelRec>();
        p->plan.share = std::vector<uint32_t>();
        *out = p;
        return KO_OK;
    } catch (const std::bad_alloc &) {
        return fail(KO_ENOMEM, "host allocation failed");
    }
}

int ko_plan_info(const ko_plan *plan, uint64_t *total_orders, uint64_t *work_items, uint64_t *chunk,
                 int32_t *grid)
{
    if (!plan)
        return fail(KO_EINVAL, "plan must not be NULL");
    if (total_orders)
        *total_orders = plan->plan.total;
    if (work_items)
        *work_items = plan->plan.n_items;
    if (chunk)
        *chunk = plan->plan.chunk;
    if (grid)
        *grid = plan->plan.grid;
    return KO_OK;
}

int ko_plan_launch(ko_plan *plan, const int64_t *ref_makespan_dev, int64_t *makespans_dev,
                   ko_set_stats *stats_dev, uint64_t *hist_dev, int32_t n_bins, void *hip_stream)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!plan)
        return fail(KO_EINVAL, "plan must not be NULL");
    int rc = check_outputs(makespans_dev, stats_dev, hist_dev, n_bins);
    if (rc || (rc = check_plan_device(plan)))
        return rc;
    DevTables t{plan->krec, plan->share, plan->sets, plan->block_base, plan->partials, plan->counter};
    return enqueue_batch(t, plan->plan, plan->gpu, plan->n_sets, plan->mode, plan->seed, plan->orders, true,
                         ref_makespan_dev, makespans_dev, stats_dev, hist_dev, n_bins, (hipStream_t)hip_stream,
                         nullptr, nullptr);
}

int ko_plan_status(ko_plan *plan, void *hip_stream)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!plan)
        return fail(KO_EINVAL, "plan must not be NULL");
    int rc = check_plan_device(plan);
    if (rc)
        return rc;
    KO_HIP(hipStreamSynchronize((hipStream_t)hip_stream), "hipStreamSynchronize");
    uint32_t status = 0;
    KO_HIP(hipMemcpy(&status, (const void *)(plan->counter + kStatusWord), sizeof status, hipMemcpyDeviceToHost),
           "hipMemcpy");
    if (status & ko::kStatusBadOrder)
        return fail(KO_EHIP, "device status: an explicit order is not a permutation of 0..n-1");
    if (status)
        return fail(KO_EHIP, "device status 0x%x: internal inconsistency", status);
    return KO_OK;
}

int ko_plan_engine(ko_plan *plan, int32_t *engine_out, int32_t *lane_entries_out, uint64_t *spilled_out,
                   uint64_t *handed_over_out, void *hip_stream)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!plan)
        return fail(KO_EINVAL, "plan must not be NULL");
    const int cls = plan->plan.lane_class;
    const uint32_t ent = plan->plan.lane_entries;
    if (engine_out)
        *engine_out = cls ? KO_ENGINE_LANES : KO_ENGINE_WAVE;
    if (lane_entries_out)
        *lane_entries_out = cls ? (int32_t)(ent ? ent : ko::lane_entry_cap(cls)) : 0;
    if (spilled_out || handed_over_out) {
        int rc = check_plan_device(plan);
        if (rc)
            return rc;
        KO_HIP(hipStreamSynchronize((hipStream_t)hip_stream), "hipStreamSynchronize");
        unsigned long long c[kCounterWords] = {};
        KO_HIP(hipMemcpy(c, (const void *)plan->counter, sizeof c, hipMemcpyDeviceToHost), "hipMemcpy");
        if (spilled_out)
            *spilled_out = c[3];
        if (handed_over_out)
            *handed_over_out = c[1];
    }
    return KO_OK;
}

int ko_plan_destroy(ko_plan *plan)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!plan)
        return KO_OK;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(plan->device);
    // launches of the plan may still be running on any stream
    (void)hipDeviceSynchronize();
    free_plan(plan);
    (void)hipSetDevice(prev);
    return KO_OK;
}

int ko_graph_capture(ko_plan *plan, const int64_t *ref_makespan_dev, int64_t *makespans_dev,
                     ko_set_stats *stats_dev, uint64_t *hist_dev, int32_t n_bins, void *hip_stream,
                     ko_graph **out)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!plan || !out)
        return fail(KO_EINVAL, "plan and out must not be NULL");
    *out = nullptr;
    if (!hip_stream)
        return fail(KO_EINVAL, "capture needs a created stream, not the null stream");
    int rc = check_outputs(makespans_dev, stats_dev, hist_dev, n_bins);
    if (rc || (rc = check_plan_device(plan)))
        return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    KO_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    DevTables t{plan->krec, plan->share, plan->sets, plan->block_base, plan->partials, plan->counter};
    rc = enqueue_batch(t, plan->plan, plan->gpu, plan->n_sets, plan->mode, plan->seed, plan->orders, true,
                       ref_makespan_dev, makespans_dev, stats_dev, hist_dev, n_bins, st, nullptr, nullptr);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(st, &graph);
    if (rc) {
        if (graph)
            (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess)
        return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e, "hipGraphInstantiate");
    }
    ko_graph *g = new ko_graph();
    g->device = plan->device;
    g->graph = graph;
    g->exec = exec;
    *out = g;
    return KO_OK;
}

int ko_graph_launch(ko_graph *graph, void *hip_stream)
{
    if (!graph)
        return fail(KO_EINVAL, "graph must not be NULL");
    KO_HIP(hipGraphLaunch(graph->exec, (hipStream_t)hip_stream), "hipGraphLaunch");
    return KO_OK;
}

int ko_graph_destroy(ko_graph *graph)
{
    if (!graph)
        return KO_OK;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(graph->device);
    (void)hipDeviceSynchronize();
    (void)hipGraphExecDestroy(graph->exec);
    (void)hipGraphDestroy(graph->graph);
    (void)hipSetDevice(prev);
    delete graph;
    return KO_OK;
}

int ko_rank_percentile(const ko_gpu_model *gpu, const ko_kernel *k, int32_t n, const int32_t *order,
                       uint64_t n_samples, uint64_t seed, ko_rank_result *out, void *hip_stream)
{
    try {
        std::lock_guard<std::mutex> lock(g_mutex);
        int rc = check_gpu(gpu);
        if (rc)
            return rc;
        if (!k || !order || !out)
            return fail(KO_EINVAL, "k, order and out must not be NULL");
        if (n < 1 || n > ko::kMaxSet)
            return fail(KO_EINVAL, "n %d outside 1..%d", n, ko::kMaxSet);
        if (n_samples > (uint64_t)INT64_MAX)
            return fail(KO_ERANGE, "n_samples too large");
        uint32_t seen = 0;
        uint8_t ord8[64];
        for (int32_t j = 0; j < n; j++) {
            if (order[j] < 0 || order[j] >= n || (seen >> order[j]) & 1u)
                return fail(KO_EINVAL, "order is not a permutation of 0..n-1");
            seen |= 1u << order[j];
            ord8[j] = (uint8_t)order[j];
        }
        {
            std::vector<ko::KernelRec> tmp;
            if ((rc = derive_set(*gpu, k, n, 0, &tmp)))
                return rc;
        }
        Workspace *w = nullptr;
        rc = get_workspace(&w);
        if (rc)
            return rc;
        hipStream_t stream = (hipStream_t)hip_stream;
        KO_HIP(hipStreamWaitEvent(stream, w->done, 0), "hipStreamWaitEvent");
        KO_HIP(hipMemcpyAsync(w->scratch_order, ord8, (size_t)n, hipMemcpyHostToDevice, stream),
               "hipMemcpyAsync");
        KO_HIP(hipStreamSynchronize(stream), "hipStreamSynchronize");
        const int32_t off[2] = {0, n};
        // 1) the makespan of the given order
        const int64_t one = 1;
        ko_order_spec sp1 = {KO_ORDERS_EXPLICIT, 0, nullptr, w->scratch_order, &one, 0};
        rc = simulate_impl(*w, gpu, k, off, 1, &sp1, nullptr, w->scratch_i64, nullptr, nullptr, 0,
                           stream);
        if (rc)
            return rc;
        // 2) counts against it over all (or sampled) orders
        const int64_t ns = (int64_t)n_samples;
        ko_order_spec sp2 = {n_samples ? KO_ORDERS_SAMPLED : KO_ORDERS_ALL, 0, nullptr, nullptr,
                             &ns, seed};
        rc = simulate_impl(*w, gpu, k, off, 1, &sp2, w->scratch_i64, nullptr, w->scratch_stats,
                           nullptr, 0, stream);
        if (rc)
            return rc;
        KO_HIP(hipMemcpyAsync(w->stats_host, w->scratch_stats, sizeof(ko_set_stats),
                              hipMemcpyDeviceToHost, stream),
               "hipMemcpyAsync");
        KO_HIP(hipMemcpyAsync(w->ref_host, w->scratch_i64, sizeof(int64_t), hipMemcpyDeviceToHost,
                              stream),
               "hipMemcpyAsync");
        KO_HIP(hipStreamSynchronize(stream), "hipStreamSynchronize");
        const int64_t ms = *w->ref_host;
        rc = check_status(*w, true);
        if (rc)
            return rc;
        const ko_set_stats st = *w->stats_host;
        out->makespan = ms;
        out->min_makespan = st.min_makespan;
        out->max_makespan = st.max_makespan;
        out->n_less = st.n_less;
        out->n_equal = st.n_equal;
        out->n_greater = st.n_greater;
        out->n_total = st.n_orders;
        const double N = (double)st.n_orders;
        out->pct_inclusive = N > 0 ? 100.0 * (double)(st.n_greater + st.n_equal) / N : 0.0;
        out->pct_strict = N > 0 ? 100.0 * (double)st.n_greater / N : 0.0;
        out->pct_mid = N > 0 ? 100.0 * ((double)st.n_greater + 0.5 * (double)st.n_equal) / N : 0.0;
        return KO_OK;
    } catch (const std::bad_alloc &) {
        return fail(KO_ENOMEM, "host allocation failed");
    }
}

int ko_sync(void *hip_stream)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    KO_HIP(hipStreamSynchronize((hipStream_t)hip_stream), "hipStreamSynchronize");
    int dev = 0;
    KO_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev < (int)g_ws.size() && g_ws[dev].ready)
        return check_status(g_ws[dev], true);
    return KO_OK;
}

int ko_shutdown(void)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    for (Workspace &w : g_ws)
        release_workspace(w);
    g_ws.clear();
    return KO_OK;
}

int ko_simulate_rounds(const ko_gpu_model *gpu, const ko_kernel *kernels, int32_t n,
                       const uint8_t *orders_dev, uint64_t first, uint64_t count, int64_t *makespans_dev,
                       void *hip_stream)
{
    try {
        int rc = check_gpu(gpu);
        if (rc)
            return rc;
        if (gpu->mem_blocks)
            return fail(KO_EINVAL, "the round-synchronous model has no memory contention (mem_blocks must be 0)");
        if (!kernels)
            return fail(KO_EINVAL, "kernels must not be NULL");
        if (n < 1 || n > ko::kMaxSet)
            return fail(KO_EINVAL, "n %d outside 1..%d", n, ko::kMaxSet);
        if (count > (uint64_t(1) << 40))
            return fail(KO_ERANGE, "count above 2^40");
        if (count && !makespans_dev)
            return fail(KO_EINVAL, "makespans_dev must not be NULL");
        if (orders_dev && first != 0)
            return fail(KO_EINVAL, "first must be 0 with explicit orders");
        if (!orders_dev && (first > factorial(n) || count > factorial(n) - first))
            return fail(KO_ERANGE, "ranks first .. first+count-1 must stay below n!");
        std::vector<ko::KernelRec> recs;
        if ((rc = derive_set(*gpu, kernels, n, 0, &recs)))
            return rc;
        if (count == 0)
            return KO_OK;
        ko::RoundsArgs a{};
        for (int32_t i = 0; i < n; i++) {
            a.k[i] = recs[i];
            int64_t c0 = std::min<int64_t>(gpu->blk_cu, gpu->reg_cu / recs[i].u_reg);
            c0 = std::min<int64_t>(c0, gpu->wave_cu / recs[i].u_wave);
            if (recs[i].u_lds)
                c0 = std::min<int64_t>(c0, gpu->lds_cu / recs[i].u_lds);
            a.c0[i] = (uint32_t)c0;
        }
        a.inv_ncu = inv_up(gpu->n_cu);
        a.orders = orders_dev;
        a.makespans = makespans_dev;
        a.first = first;
        a.count = count;
        a.n = (uint32_t)n;
        a.n_cu = (uint32_t)gpu->n_cu;
        a.cap_reg = (uint32_t)gpu->reg_cu;
        a.cap_lds = (uint32_t)gpu->lds_cu;
        a.cap_wave = (uint32_t)gpu->wave_cu;
        a.cap_blk = (uint32_t)gpu->blk_cu;
        int e = ko::launch_rounds(a, hip_stream);
        if (e)
            return hip_fail((hipError_t)e, "rounds launch");
        return KO_OK;
    } catch (const std::bad_alloc &) {
        return fail(KO_ENOMEM, "host allocation failed");
    }
}

int ko_sample_orders(int32_t n, int32_t set_index, uint64_t seed, uint64_t first,
                     const uint64_t *indices_dev, uint64_t count, uint8_t *orders_dev,
                     uint8_t *positions_dev, void *hip_stream)
{
    if (n < 1 || n > ko::kMaxSet)
        return fail(KO_EINVAL, "n %d outside 1..%d", n, ko::kMaxSet);
    if (set_index < 0 || set_index >= (1 << 24))
        return fail(KO_EINVAL, "set_index %d outside 0..2^24-1", set_index);
    if (!orders_dev && !positions_dev)
        return fail(KO_EINVAL, "orders_dev and positions_dev are both NULL");
    const uint64_t kCounters = uint64_t(1) << 40;
    if (count > kCounters || (!indices_dev && first > kCounters - count))
        return fail(KO_ERANGE, "sample indices must stay below 2^40");
    if (count == 0)
        return KO_OK;
    int e = ko::launch_sample_orders((uint32_t)n, (uint32_t)set_index, seed, first, indices_dev, count,
                                     orders_dev, positions_dev, hip_stream);
    if (e)
        return hip_fail((hipError_t)e, "sample orders launch");
    return KO_OK;
}

int ko_topk_f32(const float *y_dev, uint64_t count, int32_t k, int64_t *idx_out_dev, float *val_out_dev,
                void *hip_stream)
{
    try {
        std::lock_guard<std::mutex> lock(g_mutex);
        if (!y_dev)
            return fail(KO_EINVAL, "y_dev must not be NULL");
        if (!idx_out_dev && !val_out_dev)
            return fail(KO_EINVAL, "idx_out_dev and val_out_dev are both NULL");
        if (count < 1 || count >= (uint64_t(1) << 32))
            return fail(KO_EINVAL, "count must be in 1..2^32-1");
        if (k < 1 || (uint64_t)k > std::min<uint64_t>(count, kTopkMax))
            return fail(KO_EINVAL, "k must be in 1..min(count, %llu)", (unsigned long long)kTopkMax);
        Workspace *w = nullptr;
        int rc = get_workspace(&w);
        if (rc)
            return rc;
        rc = check_status(*w, false);
        if (rc)
            return rc;
        hipStream_t stream = (hipStream_t)hip_stream;
        if ((rc = grow_device(w->done, (void **)&w->sel_cand, &w->sel_cand_cap,
                              kTopkCandidates * sizeof(uint64_t))))
            return rc;
        KO_HIP(hipStreamWaitEvent(stream, w->done, 0), "hipStreamWaitEvent");
        const int grid = std::max(1, w->cu_count * 8);
        uint64_t prefix = 0, mask = 0, rem = (uint64_t)k, cls = 0;
        for (int shift = 24; shift >= 0; shift -= 8) {
            rc = radix_pass(*w, stream, (uint32_t)shift, &prefix, &mask, &rem, &cls,
                            [&](uint64_t p, uint64_t m, uint32_t sh) {
                                return ko::launch_radix_hist_f32(y_dev, count, sh, m, p, w->sel_bins,
                                                                 grid, stream);
                            });
            if (rc)
                return rc;
        }
        // keys < k-th: k - rem of them; keys == k-th: cls
        const uint64_t total = (uint64_t)k - rem + cls;
        if (total > kTopkCandidates)
            return fail(KO_ERANGE, "%llu values tie with the k-th smallest; at most %llu candidates",
                        (unsigned long long)total, (unsigned long long)kTopkCandidates);
        unsigned long long *cursor = w->sel_bins + 256;
        int e = ko::launch_zero_u64((uint64_t *)cursor, 1, stream);
        if (!e)
            e = ko::launch_gather_f32(y_dev, count, (uint32_t)prefix, w->sel_cand, kTopkCandidates, cursor,
                                      grid, stream);
        uint64_t n_pow2 = 1;
        while (n_pow2 < total)
            n_pow2 <<= 1;
        if (!e)
            e = ko::launch_bitonic_sort_u64(w->sel_cand, total, n_pow2, stream);
        if (!e)
            e = ko::launch_unpack_topk(w->sel_cand, (uint32_t)k, idx_out_dev, val_out_dev, stream);
        if (e)
            return hip_fail((hipError_t)e, "top-k launch");
        KO_HIP(hipEventRecord(w->done, stream), "hipEventRecord");
        return KO_OK;
    } catch (const std::bad_alloc &) {
        return fail(KO_ENOMEM, "host allocation failed");
    }
}

int ko_kth_smallest_i64(const int64_t *v_dev, uint64_t count, uint64_t k, int64_t *value_out,
                        uint64_t *count_le_out, void *hip_stream)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!v_dev || !value_out)
        return fail(KO_EINVAL, "v_dev and value_out must not be NULL");
    if (count < 1 || k < 1 || k > count)
        return fail(KO_EINVAL, "need 1 <= k <= count");
    Workspace *w = nullptr;
    int rc = get_workspace(&w);
    if (rc)
        return rc;
    rc = check_status(*w, false);
    if (rc)
        return rc;
    hipStream_t stream = (hipStream_t)hip_stream;
    KO_HIP(hipStreamWaitEvent(stream, w->done, 0), "hipStreamWaitEvent");
    const int grid = std::max(1, w->cu_count * 8);
    uint64_t prefix = 0, mask = 0, rem = k, cls = 0;
    for (int shift = 56; shift >= 0; shift -= 8) {
        rc = radix_pass(*w, stream, (uint32_t)shift, &prefix, &mask, &rem, &cls,
                        [&](uint64_t p, uint64_t m, uint32_t sh) {
                            return ko::launch_radix_hist_i64(v_dev, count, sh, m, p, w->sel_bins, grid,
                                                             stream);
                        });
        if (rc)
            return rc;
    }
    KO_HIP(hipEventRecord(w->done, stream), "hipEventRecord");
    *value_out = (int64_t)(prefix ^ 0x8000000000000000ull);
    if (count_le_out)
        *count_le_out = k - rem + cls;  // below the k-th value, plus its ties
    return KO_OK;
}

int ko_sort_i64(const int64_t *v_dev, uint64_t count, int64_t *sorted_out_dev, uint64_t *index_out_dev,
                void *hip_stream)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!v_dev || (!sorted_out_dev && !index_out_dev))
        return fail(KO_EINVAL, "v_dev and at least one output must not be NULL");
    if (count < 1 || count >= (uint64_t(1) << 32))
        return fail(KO_EINVAL, "count %llu outside 1 .. 2^32-1", (unsigned long long)count);
    Workspace *w = nullptr;
    int rc = get_workspace(&w);
    if (rc)
        return rc;
    rc = check_status(*w, false);
    if (rc)
        return rc;
    const uint64_t tiles = ko::sort_tiles(count);
    const size_t key_bytes = (count * 8 + 255) & ~(size_t)255;
    const size_t idx_bytes = (count * 4 + 255) & ~(size_t)255;
    const size_t need = 2 * key_bytes + 2 * idx_bytes + tiles * 256 * 4;
    if ((rc = grow_device(w->done, &w->sort_buf, &w->sort_cap, need)))
        return rc;
    hipStream_t stream = (hipStream_t)hip_stream;
    KO_HIP(hipStreamWaitEvent(stream, w->done, 0), "hipStreamWaitEvent");
    // the spread of the values fixes the number of digit passes
    int e = ko::launch_zero_u64((uint64_t *)w->sel_bins, 2, stream);
    if (e)
        return hip_fail((hipError_t)e, "zero min/max");
    e = ko::launch_minmax_i64(v_dev, count, w->sel_bins, std::max(1, w->cu_count * 8), stream);
    if (e)
        return hip_fail((hipError_t)e, "min/max launch");
    KO_HIP(hipMemcpyAsync(w->sel_host, w->sel_bins, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, stream),
           "hipMemcpyAsync");
    KO_HIP(hipStreamSynchronize(stream), "hipStreamSynchronize");
    const uint64_t kmin = ~w->sel_host[0], kmax = w->sel_host[1];
    const int64_t vmin = (int64_t)(kmin ^ 0x8000000000000000ull);
    const uint64_t span = kmax - kmin;
    uint32_t passes = 0;
    while (passes < 8 && (span >> (8 * passes)) != 0)
        passes++;
    char *b = static_cast<char *>(w->sort_buf);
    uint64_t *keys_a = reinterpret_cast<uint64_t *>(b);
    uint64_t *keys_b = reinterpret_cast<uint64_t *>(b + key_bytes);
    uint32_t *idx_a = reinterpret_cast<uint32_t *>(b + 2 * key_bytes);
    uint32_t *idx_b = reinterpret_cast<uint32_t *>(b + 2 * key_bytes + idx_bytes);
    uint32_t *counts = reinterpret_cast<uint32_t *>(b + 2 * key_bytes + 2 * idx_bytes);
    e = ko::launch_sort_i64(v_dev, count, vmin, passes, keys_a, idx_a, keys_b, idx_b, counts, sorted_out_dev,
                            index_out_dev, stream);
    if (e)
        return hip_fail((hipError_t)e, "sort launch");
    KO_HIP(hipEventRecord(w->done, stream), "hipEventRecord");
    KO_HIP(hipStreamSynchronize(stream), "hipStreamSynchronize");
    return KO_OK;
}

int ko_stats_i64(const int64_t *v_dev, uint64_t count, const int64_t *ref_dev, ko_set_stats *stats_dev,
                 void *hip_stream)
{
    try {
        std::lock_guard<std::mutex> lock(g_mutex);
        if (!stats_dev)
            return fail(KO_EINVAL, "stats_dev must not be NULL");
        if (count && !v_dev)
            return fail(KO_EINVAL, "v_dev must not be NULL when count > 0");
        if (count > (uint64_t(1) << 40))
            return fail(KO_ERANGE, "count above 2^40");
        Workspace *w = nullptr;
        int rc = get_workspace(&w);
        if (rc)
            return rc;
        // four workgroups per CU, never more than one per 256 values
        const uint32_t parts =
            (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((count + 255) / 256, (uint64_t)w->cu_count * 4));
        if ((rc = grow_device(w->done, (void **)&w->stat_parts, &w->stat_parts_cap, parts * sizeof(ko::Partial))))
            return rc;
        hipStream_t stream = (hipStream_t)hip_stream;
        KO_HIP(hipStreamWaitEvent(stream, w->done, 0), "hipStreamWaitEvent");
        const int e = ko::launch_stats_i64(v_dev, count, ref_dev, w->stat_parts, parts, stats_dev, stream);
        if (e)
            return hip_fail((hipError_t)e, "statistics launch");
        KO_HIP(hipEventRecord(w->done, stream), "hipEventRecord");
        return KO_OK;
    } catch (const std::bad_alloc &) {
        return fail(KO_ENOMEM, "host allocation failed");
    }
}

int ko_set_kernel_timing(int32_t enable)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    Workspace *w = nullptr;
    int rc = get_workspace(&w);
    if (rc)
        return rc;
    w->timing = enable != 0;
    w->timed = false;
    return KO_OK;
}

int ko_last_kernel_ms(float *ms_out)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!ms_out)
        return fail(KO_EINVAL, "ms_out must not be NULL");
    Workspace *w = nullptr;
    int rc = get_workspace(&w);
    if (rc)
        return rc;
    if (!w->timed)
        return fail(KO_EINVAL, "no simulate kernel was launched on this device since timing was enabled");
    KO_HIP(hipEventSynchronize(w->sim_end), "hipEventSynchronize");
    KO_HIP(hipEventElapsedTime(ms_out, w->sim_begin, w->sim_end), "hipEventElapsedTime");
    return KO_OK;
}

const char *ko_last_error(void) { return g_error.c_str(); }

}  // extern "C"
