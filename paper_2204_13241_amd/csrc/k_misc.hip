// Speckle-matching loss and position update (the loss of the differentiation
// workload), per-kernel event timing, and the roofline microbenchmarks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "xs_internal.h"

namespace xs {
namespace {

constexpr int kBlock = 256;
constexpr int kLossBlocks = 1024;

// Pass 1: block partial sums of (I - I_t)^2 and I_t^2, grid-stride in fixed order.
__global__ __launch_bounds__(kBlock) void k_loss_partial(const double *__restrict__ I,
                                                         const double *__restrict__ It, int64_t n,
                                                         double *__restrict__ part) {
    __shared__ double s_a[kBlock], s_b[kBlock];
    double a = 0.0, b = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kBlock) {
        const double d = I[i] - It[i];
        a = __builtin_fma(d, d, a);
        b = __builtin_fma(It[i], It[i], b);
    }
    s_a[threadIdx.x] = a;
    s_b[threadIdx.x] = b;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            s_a[threadIdx.x] += s_a[threadIdx.x + off];
            s_b[threadIdx.x] += s_b[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s_a[0];
        part[2 * blockIdx.x + 1] = s_b[0];
    }
}

// Pass 2: loss = sum (I - I_t)^2 / sum I_t^2 (one block, fixed order), then
// dL/dI = 2 (I - I_t) / sum I_t^2.
__global__ __launch_bounds__(kBlock) void k_loss_final(const double *__restrict__ part, int nb,
                                                       double *__restrict__ out) {
    __shared__ double s_a[kBlock], s_b[kBlock];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nb; i += kBlock) {
        a += part[2 * i];
        b += part[2 * i + 1];
    }
    s_a[threadIdx.x] = a;
    s_b[threadIdx.x] = b;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            s_a[threadIdx.x] += s_a[threadIdx.x + off];
            s_b[threadIdx.x] += s_b[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s_a[0] / s_b[0];
        out[1] = s_b[0];
    }
}

__global__ __launch_bounds__(kBlock) void k_loss_grad(const double *__restrict__ I,
                                                      const double *__restrict__ It, int64_t n,
                                                      const double *__restrict__ fin,
                                                      double *__restrict__ w) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    w[i] = 2.0 * (I[i] - It[i]) / fin[1];
}

__global__ __launch_bounds__(kBlock) void k_position_step(double *__restrict__ pos,
                                                          const float *__restrict__ g32,
                                                          const double *__restrict__ g64,
                                                          int64_t n, double step) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    const double g = g64 ? g64[i] : static_cast<double>(g32[i]);
    pos[i] = __builtin_fma(-step, g, pos[i]);
}

// ---------------------------------------------------------------- microbenchmarks
// Eight independent chains per lane keep every issue slot busy; the results are
// consumed by a store that never happens for finite inputs.
__global__ __launch_bounds__(kBlock) void k_probe_trans(float *sink, int iters) {
    float a[8];
    for (int k = 0; k < 8; ++k) a[k] = 0.01f * k + 1e-6f * threadIdx.x;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) a[k] = __builtin_amdgcn_sinf(a[k]);
#pragma unroll
        for (int k = 0; k < 8; ++k) a[k] = __builtin_amdgcn_cosf(a[k]);
    }
    float r = 0.f;
    for (int k = 0; k < 8; ++k) r += a[k];
    if (r == 12345.678f) sink[threadIdx.x] = r;
}

__global__ __launch_bounds__(kBlock) void k_probe_fma32(float *sink, int iters) {
    float a[8];
    for (int k = 0; k < 8; ++k) a[k] = 0.01f * k + 1e-6f * threadIdx.x;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) a[k] = __builtin_fmaf(a[k], 0.999f, 1e-3f);
#pragma unroll
        for (int k = 0; k < 8; ++k) a[k] = __builtin_fmaf(a[k], 0.999f, 1e-3f);
    }
    float r = 0.f;
    for (int k = 0; k < 8; ++k) r += a[k];
    if (r == 12345.678f) sink[threadIdx.x] = r;
}

__global__ __launch_bounds__(kBlock) void k_probe_fma64(double *sink, int iters) {
    double a[8];
    for (int k = 0; k < 8; ++k) a[k] = 0.01 * k + 1e-6 * threadIdx.x;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) a[k] = __builtin_fma(a[k], 0.999, 1e-3);
#pragma unroll
        for (int k = 0; k < 8; ++k) a[k] = __builtin_fma(a[k], 0.999, 1e-3);
    }
    double r = 0.0;
    for (int k = 0; k < 8; ++k) r += a[k];
    if (r == 12345.678) sink[threadIdx.x] = r;
}

// FP16 matrix instructions (v_mfma_f32_32x32x16_f16) on four independent accumulators;
// with MIX each is followed by eight independent FP32 FMAs of the same wavefront, which
// shows whether the vector unit issues while the matrix core works.
typedef _Float16 probe_half8 __attribute__((ext_vector_type(8)));
typedef float probe_float16 __attribute__((ext_vector_type(16)));
template <bool MIX>
__global__ __launch_bounds__(kBlock) void k_probe_mfma(float *sink, int iters) {
    probe_half8 a, b;
    for (int u = 0; u < 8; ++u) {
        a[u] = static_cast<_Float16>(1e-3f * (u + 1));
        b[u] = static_cast<_Float16>(1e-3f * (threadIdx.x & 7));
    }
    probe_float16 c[4];
    for (int k = 0; k < 4; ++k)
        for (int i = 0; i < 16; ++i) c[k][i] = 0.f;
    float x[8];
    for (int k = 0; k < 8; ++k) x[k] = 0.01f * k + 1e-6f * threadIdx.x;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            c[k] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c[k], 0, 0, 0);
            if (MIX)
#pragma unroll
                for (int m = 0; m < 8; ++m) x[m] = __builtin_fmaf(x[m], 0.999f, 1e-3f);
        }
    }
    float r = 0.f;
    for (int k = 0; k < 4; ++k)
        for (int i = 0; i < 16; ++i) r += c[k][i];
    for (int k = 0; k < 8; ++k) r += x[k];
    if (r == 12345.678f) sink[threadIdx.x] = r;
}

// Streaming probes: each block takes runs of kProbeRun * kBlock 16-byte elements
// (grid-stride), every thread with kProbeRun loads in flight.  Copy: b = a.  Read:
// the elements summed into a value that is stored only if it hits a sentinel.
constexpr int kProbeRun = 4;

__global__ __launch_bounds__(kBlock) void k_probe_copy(const float4 *__restrict__ a,
                                                       float4 *__restrict__ b, int64_t n) {
    const int64_t step = static_cast<int64_t>(gridDim.x) * kBlock * kProbeRun;
    for (int64_t base = static_cast<int64_t>(blockIdx.x) * kBlock * kProbeRun; base < n; base += step) {
        float4 v[kProbeRun];
#pragma unroll
        for (int u = 0; u < kProbeRun; ++u) {
            const int64_t i = base + u * kBlock + threadIdx.x;
            v[u] = i < n ? a[i] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < kProbeRun; ++u) {
            const int64_t i = base + u * kBlock + threadIdx.x;
            if (i < n) b[i] = v[u];
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_probe_read(const float4 *__restrict__ a, float *__restrict__ sink,
                                                       int64_t n) {
    const int64_t step = static_cast<int64_t>(gridDim.x) * kBlock * kProbeRun;
    float acc = 0.f;
    for (int64_t base = static_cast<int64_t>(blockIdx.x) * kBlock * kProbeRun; base < n; base += step) {
        float4 v[kProbeRun];
#pragma unroll
        for (int u = 0; u < kProbeRun; ++u) {
            const int64_t i = base + u * kBlock + threadIdx.x;
            v[u] = i < n ? a[i] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < kProbeRun; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
    }
    if (acc == 12345.678f) sink[threadIdx.x] = acc;
}

}  // namespace

// ---------------------------------------------------------------- timing

namespace {
struct TimerRec {
    hipEvent_t a, b;
    double work;
};
std::mutex g_tmu;
bool g_timing = false;
std::vector<TimerRec> g_pending[XS_TIMER_KINDS];
double g_total_ms[XS_TIMER_KINDS];
int64_t g_count[XS_TIMER_KINDS];
double g_work[XS_TIMER_KINDS];
}  // namespace

bool timing_on() {
    std::lock_guard<std::mutex> lk(g_tmu);
    return g_timing;
}

void timer_begin(hipStream_t s, int kind, void **token) {
    *token = nullptr;
    if (!timing_on()) return;
    auto *rec = new TimerRec();
    if (hipEventCreate(&rec->a) != hipSuccess || hipEventCreate(&rec->b) != hipSuccess) {
        delete rec;
        return;
    }
    (void)hipEventRecord(rec->a, s);
    rec->work = 0.0;
    *token = rec;
    (void)kind;
}

void timer_end(hipStream_t s, int kind, void *token, double work) {
    if (!token) return;
    auto *rec = static_cast<TimerRec *>(token);
    (void)hipEventRecord(rec->b, s);
    rec->work = work;
    std::lock_guard<std::mutex> lk(g_tmu);
    g_pending[kind].push_back(*rec);
    delete rec;
}

void timer_discard(void *token) {
    if (!token) return;
    auto *rec = static_cast<TimerRec *>(token);
    (void)hipEventDestroy(rec->a);
    (void)hipEventDestroy(rec->b);
    delete rec;
}

xs_status timing_enable(int on) {
    std::lock_guard<std::mutex> lk(g_tmu);
    for (int k = 0; k < XS_TIMER_KINDS; ++k) {
        for (auto &r : g_pending[k]) {
            (void)hipEventSynchronize(r.b);
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        g_pending[k].clear();
        g_total_ms[k] = 0.0;
        g_count[k] = 0;
        g_work[k] = 0.0;
    }
    g_timing = on != 0;
    return XS_OK;
}

xs_status timing_read(int kind, double *ms, int64_t *launches, double *work) {
    if (kind < 0 || kind >= XS_TIMER_KINDS) return set_error(XS_EINVAL, "timer kind out of range");
    std::lock_guard<std::mutex> lk(g_tmu);
    for (auto &r : g_pending[kind]) {
        XS_HIP(hipEventSynchronize(r.b));
        float t = 0.f;
        XS_HIP(hipEventElapsedTime(&t, r.a, r.b));
        g_total_ms[kind] += t;
        g_count[kind] += 1;
        g_work[kind] += r.work;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_pending[kind].clear();
    if (ms) *ms = g_total_ms[kind];
    if (launches) *launches = g_count[kind];
    if (work) *work = g_work[kind];
    return XS_OK;
}

// ---------------------------------------------------------------- loss

xs_status speckle_loss(hipStream_t s, const double *I, const double *It, int64_t n, double *out,
                       double *dL_dI) {
    void *part = nullptr;
    XS_TRY(scratch(s, SLOT_BWIN, sizeof(double) * 2 * kLossBlocks, &part));
    int nb = static_cast<int>((n + kBlock - 1) / kBlock);
    nb = nb < 1 ? 1 : (nb > kLossBlocks ? kLossBlocks : nb);
    hipLaunchKernelGGL(k_loss_partial, dim3(nb), dim3(kBlock), 0, s, I, It, n, static_cast<double *>(part));
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(kBlock), 0, s, static_cast<const double *>(part), nb, out);
    if (dL_dI && n > 0)
        hipLaunchKernelGGL(k_loss_grad, dim3(static_cast<unsigned>((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                           I, It, n, static_cast<const double *>(out), dL_dI);
    XS_HIP(hipGetLastError());
    return XS_OK;
}

xs_status position_step(hipStream_t s, double *pos, const float *g32, const double *g64, int64_t n,
                        double step) {
    if (n == 0) return XS_OK;
    hipLaunchKernelGGL(k_position_step, dim3(static_cast<unsigned>((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       pos, g32, g64, n, step);
    XS_HIP(hipGetLastError());
    return XS_OK;
}

// ---------------------------------------------------------------- probes

xs_status roofline_probe(hipStream_t s, int kind, int64_t bytes, double *rate) {
    if (kind < 0 || kind > 6 || !rate) return set_error(XS_EINVAL, "probe kind must be 0..6, rate non-NULL");
    int dev = 0, cus = 0;
    XS_HIP(hipGetDevice(&dev));
    XS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int blocks = cus * 16, iters = 2048;
    void *sink = nullptr, *src = nullptr;
    hipEvent_t e0, e1;
    XS_HIP(hipEventCreate(&e0));
    XS_HIP(hipEventCreate(&e1));
    double ops = 0.0;
    float ms = 0.f;
    if (kind == 0 || kind == 1 || kind == 2) {
        XS_TRY(scratch(s, SLOT_BWIN, sizeof(double) * kBlock, &sink));
        auto launch = [&]() {
            if (kind == 0) hipLaunchKernelGGL(k_probe_trans, dim3(blocks), dim3(kBlock), 0, s, static_cast<float *>(sink), iters);
            if (kind == 1) hipLaunchKernelGGL(k_probe_fma32, dim3(blocks), dim3(kBlock), 0, s, static_cast<float *>(sink), iters);
            if (kind == 2) hipLaunchKernelGGL(k_probe_fma64, dim3(blocks), dim3(kBlock), 0, s, static_cast<double *>(sink), iters);
        };
        launch();
        XS_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < 5; ++r) launch();
        XS_HIP(hipEventRecord(e1, s));
        ops = 5.0 * blocks * kBlock * static_cast<double>(iters) * 16.0;
    } else if (kind == 4 || kind == 5) {
        XS_TRY(scratch(s, SLOT_BWIN, sizeof(double) * kBlock, &sink));
        const int mb = cus * 8, mi = 1024;
        auto launch = [&]() {
            if (kind == 4) hipLaunchKernelGGL(k_probe_mfma<false>, dim3(mb), dim3(kBlock), 0, s, static_cast<float *>(sink), mi);
            else hipLaunchKernelGGL(k_probe_mfma<true>, dim3(mb), dim3(kBlock), 0, s, static_cast<float *>(sink), mi);
        };
        launch();
        XS_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < 5; ++r) launch();
        XS_HIP(hipEventRecord(e1, s));
        ops = 5.0 * mb * (kBlock / 64) * static_cast<double>(mi) * 4.0 * 2.0 * 32 * 32 * 16;
    } else if (kind == 3) {
        if (bytes < 16) bytes = 16;
        const int64_t nv = bytes / 16;
        XS_TRY(scratch(s, SLOT_LEVEL_A, nv * 16, &src));
        XS_TRY(scratch(s, SLOT_LEVEL_B, nv * 16, &sink));
        hipLaunchKernelGGL(k_probe_copy, dim3(cus * 32), dim3(kBlock), 0, s, static_cast<const float4 *>(src),
                           static_cast<float4 *>(sink), nv);
        XS_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < 5; ++r)
            hipLaunchKernelGGL(k_probe_copy, dim3(cus * 32), dim3(kBlock), 0, s, static_cast<const float4 *>(src),
                               static_cast<float4 *>(sink), nv);
        XS_HIP(hipEventRecord(e1, s));
        ops = 5.0 * 2.0 * static_cast<double>(nv) * 16.0;  // bytes read + written
    } else if (kind == 6) {
        if (bytes < 16) bytes = 16;
        const int64_t nv = bytes / 16;
        XS_TRY(scratch(s, SLOT_LEVEL_A, nv * 16, &src));
        XS_TRY(scratch(s, SLOT_BWIN, sizeof(double) * kBlock, &sink));
        hipLaunchKernelGGL(k_probe_read, dim3(cus * 32), dim3(kBlock), 0, s, static_cast<const float4 *>(src),
                           static_cast<float *>(sink), nv);
        XS_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < 5; ++r)
            hipLaunchKernelGGL(k_probe_read, dim3(cus * 32), dim3(kBlock), 0, s, static_cast<const float4 *>(src),
                               static_cast<float *>(sink), nv);
        XS_HIP(hipEventRecord(e1, s));
        ops = 5.0 * static_cast<double>(nv) * 16.0;  // bytes read
    } else {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return set_error(XS_EINVAL, "probe kind must be 0..6");
    }
    XS_HIP(hipGetLastError());
    XS_HIP(hipEventSynchronize(e1));
    XS_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *rate = ops / (static_cast<double>(ms) * 1e-3);
    return XS_OK;
}

int resident_blocks(const void *kernel, int block) {
    static std::mutex mu;
    static std::vector<std::pair<std::pair<const void *, int>, int>> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(mu);
    for (auto &e : cache)
        if (e.first.first == kernel && e.first.second == dev) return e.second;
    int cus = 0, per = 1;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, block, 0);
    const int n = std::max(1, cus) * std::max(1, per);
    cache.emplace_back(std::make_pair(kernel, dev), n);
    return n;
}

}  // namespace xs
