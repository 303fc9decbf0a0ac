// Hardware validation of the dispatch model (libko): synthetic kernels shaped
// like a kernel set's Table 1 parameters, launched on real hardware in a given
// order, one stream per kernel, with the makespan timed by HIP events.
//
// Kernel i becomes: N_tblk blocks of waves_blk * 64 threads with lds_blk bytes
// of dynamic LDS; each thread runs F = N_inst / scale fused multiply-adds over
// K live accumulators (K sets the register footprint: each variant is a
// separate compiled kernel, and its real VGPR count is reported so that the
// model can be evaluated with what the hardware allocates) and
// L = F * 1000 / r_milli streaming 16-byte loads (R = r_milli / 1000 is the
// kernel's ratio of compute to memory instructions, Section 4).  All memory
// accesses stay inside the buffers; every loop has a fixed trip count.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "ko.h"

namespace {

thread_local std::string g_hw_err = "no error";

int hw_fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_hw_err = buf;
    return code;
}

#define HW_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return hw_fail(KO_EHIP, "%s: %s", #call, hipGetErrorString(e_));           \
    } while (0)

constexpr uint64_t kSrcFloat4 = uint64_t(1) << 26;  // 1 GiB streaming source

template <int K>
__global__ __launch_bounds__(1024) void work_kernel(const float4 *__restrict__ src, float *__restrict__ sink,
                                                    uint32_t fma_iters, uint32_t loads, uint32_t lds_floats)
{
    extern __shared__ float lds[];
    float acc[K];
#pragma unroll
    for (int k = 0; k < K; k++)
        acc[k] = (float)(threadIdx.x + k) * 1e-3f;
    // compute: fma_iters rounds of K independent FMAs
    for (uint32_t it = 0; it < fma_iters; it++) {
#pragma unroll
        for (int k = 0; k < K; k++)
            acc[k] = __builtin_fmaf(acc[k], 0.999f, 0.5f);
    }
    // memory: coalesced 16-byte loads striding through the source
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    float m = 0.f;
    for (uint32_t l = 0; l < loads; l++) {
        const float4 v = src[(tid + (uint64_t)l * stride) & (kSrcFloat4 - 1)];
        m += v.x + v.w;
    }
    float s = m;
#pragma unroll
    for (int k = 0; k < K; k++)
        s += acc[k];
    if (lds_floats) {
        lds[threadIdx.x % lds_floats] = s;
        __syncthreads();
        s += lds[(threadIdx.x + 1) % lds_floats];
    }
    if (s == 12345.678f)  // practically never; keeps the work observable
        sink[blockIdx.x & 0xFFFFu] = s;  // the sink holds 2^18 floats
}

using KernelFn = void (*)(const float4 *, float *, uint32_t, uint32_t, uint32_t);

struct Variant {
    int k;
    KernelFn fn;
    int vgprs = 0;
};

std::vector<Variant> &variants()
{
    static std::vector<Variant> v = {
        {4, work_kernel<4>}, {8, work_kernel<8>}, {16, work_kernel<16>}, {24, work_kernel<24>},
        {32, work_kernel<32>}, {48, work_kernel<48>}, {64, work_kernel<64>}, {96, work_kernel<96>}};
    return v;
}

int query_variants()
{
    for (Variant &v : variants()) {
        if (v.vgprs)
            continue;
        hipFuncAttributes a;
        HW_HIP(hipFuncGetAttributes(&a, reinterpret_cast<const void *>(v.fn)));
        v.vgprs = a.numRegs;
    }
    return KO_OK;
}

// the variant whose register count is closest to regs (ties: the smaller)
const Variant &pick(int regs)
{
    const Variant *best = &variants()[0];
    for (const Variant &v : variants())
        if (std::abs(v.vgprs - regs) < std::abs(best->vgprs - regs))
            best = &v;
    return *best;
}

struct HwState {
    int device = -1;
    float4 *src = nullptr;
    float *sink = nullptr;
};

HwState g_hw;

int hw_state()
{
    int dev = 0;
    HW_HIP(hipGetDevice(&dev));
    if (g_hw.device == dev)
        return KO_OK;
    if (g_hw.src) {
        (void)hipFree(g_hw.src);
        (void)hipFree(g_hw.sink);
    }
    g_hw = HwState();
    HW_HIP(hipMalloc((void **)&g_hw.src, kSrcFloat4 * sizeof(float4)));
    HW_HIP(hipMemset(g_hw.src, 0, kSrcFloat4 * sizeof(float4)));
    HW_HIP(hipMalloc((void **)&g_hw.sink, 1 << 20));
    HW_HIP(hipDeviceSynchronize());
    g_hw.device = dev;
    return query_variants();
}

}  // namespace

extern "C" {

int ko_hw_vgprs(int32_t regs_thr, int32_t *vgprs_out)
{
    if (!vgprs_out)
        return hw_fail(KO_EINVAL, "vgprs_out must not be NULL");
    int rc = hw_state();
    if (rc)
        return rc;
    *vgprs_out = pick(regs_thr).vgprs;
    return KO_OK;
}

int ko_hw_time_orders(const ko_kernel *k, int32_t n, const int32_t *orders, int32_t n_orders, int32_t scale,
                      int32_t reps, double *makespan_ms_out)
{
    if (!k || !orders || !makespan_ms_out)
        return hw_fail(KO_EINVAL, "k, orders and makespan_ms_out must not be NULL");
    if (n < 1 || n > 20 || n_orders < 1 || scale < 1 || reps < 1)
        return hw_fail(KO_EINVAL, "need 1 <= n <= 20, n_orders >= 1, scale >= 1, reps >= 1");
    for (int32_t i = 0; i < n; i++) {
        const ko_kernel &q = k[i];
        if (q.n_tblk < 1 || q.n_tblk > (1 << 20) || q.waves_blk < 1 || q.waves_blk > 16 || q.lds_blk < 0 ||
            q.lds_blk > 160 * 1024 || q.r_milli < 1 || q.n_inst < 1)
            return hw_fail(KO_EINVAL, "kernel %d outside the launchable range", i);
    }
    for (int32_t o = 0; o < n_orders; o++) {
        uint32_t seen = 0;
        for (int32_t j = 0; j < n; j++) {
            const int32_t v = orders[o * n + j];
            if (v < 0 || v >= n || ((seen >> v) & 1u))
                return hw_fail(KO_EINVAL, "order %d is not a permutation of 0..n-1", o);
            seen |= 1u << v;
        }
    }
    int rc = hw_state();
    if (rc)
        return rc;
    std::vector<hipStream_t> streams(n, nullptr);
    std::vector<hipEvent_t> ends(n, nullptr);
    hipEvent_t start = nullptr;
    auto cleanup = [&]() {
        for (auto &s : streams)
            if (s)
                (void)hipStreamDestroy(s);
        for (auto &e : ends)
            if (e)
                (void)hipEventDestroy(e);
        if (start)
            (void)hipEventDestroy(start);
    };
    hipError_t e = hipEventCreate(&start);
    for (int32_t i = 0; i < n && e == hipSuccess; i++) {
        e = hipStreamCreateWithFlags(&streams[i], hipStreamNonBlocking);
        if (e == hipSuccess)
            e = hipEventCreate(&ends[i]);
    }
    if (e != hipSuccess) {
        cleanup();
        return hw_fail(KO_EHIP, "stream/event creation: %s", hipGetErrorString(e));
    }
    for (int32_t o = 0; o < n_orders && e == hipSuccess; o++) {
        double best = 1e300;
        for (int32_t r = 0; r < reps && e == hipSuccess; r++) {
            e = hipDeviceSynchronize();
            const int32_t first = orders[o * n];
            if (e == hipSuccess)
                e = hipEventRecord(start, streams[first]);
            for (int32_t j = 0; j < n && e == hipSuccess; j++) {
                const int32_t i = orders[o * n + j];
                const ko_kernel &q = k[i];
                const Variant &v = pick(q.regs_thr);
                const uint64_t f = std::max<uint64_t>(1, (uint64_t)q.n_inst / (uint64_t)scale);
                const uint32_t fma_iters = (uint32_t)std::max<uint64_t>(1, f / (uint64_t)v.k);
                const uint32_t loads = (uint32_t)std::min<uint64_t>(f * 1000 / (uint64_t)q.r_milli, 1u << 24);
                const uint32_t lds_floats = (uint32_t)(q.lds_blk / 4);
                if (j > 0)
                    e = hipStreamWaitEvent(streams[i], start, 0);
                if (e == hipSuccess) {
                    hipLaunchKernelGGL(v.fn, dim3((uint32_t)q.n_tblk), dim3((uint32_t)q.waves_blk * 64),
                                       (size_t)q.lds_blk, streams[i], g_hw.src, g_hw.sink, fma_iters, loads,
                                       lds_floats);
                    e = hipGetLastError();
                }
                if (e == hipSuccess)
                    e = hipEventRecord(ends[i], streams[i]);
            }
            float worst = 0.f;
            for (int32_t i = 0; i < n && e == hipSuccess; i++) {
                e = hipEventSynchronize(ends[i]);
                float ms = 0.f;
                if (e == hipSuccess)
                    e = hipEventElapsedTime(&ms, start, ends[i]);
                worst = std::max(worst, ms);
            }
            best = std::min(best, (double)worst);
        }
        makespan_ms_out[o] = best;
    }
    cleanup();
    if (e != hipSuccess)
        return hw_fail(KO_EHIP, "hardware timing: %s", hipGetErrorString(e));
    return KO_OK;
}

const char *ko_hw_last_error(void) { return g_hw_err.c_str(); }

}  // extern "C"
