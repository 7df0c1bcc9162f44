// Host side of the xs C ABI: argument validation, batch -> segment expansion,
// scratch management and dispatch to the kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <mutex>
#include <string>
#include <vector>

#include "xs_internal.h"

namespace xs {

// ---------------------------------------------------------------- errors

namespace {
thread_local std::string g_last_error;
}

xs_status set_error(xs_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

xs_status hip_error(hipError_t e, const char *what) {
    return set_error(e == hipErrorOutOfMemory ? XS_ENOMEM : XS_EDEVICE, "%s: %s (%d)", what,
                     hipGetErrorString(e), static_cast<int>(e));
}

// ---------------------------------------------------------------- scratch

namespace {

struct Buffer {
    void *dev = nullptr;
    size_t bytes = 0;
    void *pinned = nullptr;      // host staging for uploads into this slot
    size_t pinned_bytes = 0;
    hipEvent_t copied = nullptr;  // last upload from `pinned` has been read
};

struct StreamScratch {
    int device = 0;
    hipStream_t stream = nullptr;
    Buffer slot[SLOT_COUNT];
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, StreamScratch *> g_scratch;

StreamScratch *scratch_for(hipStream_t s) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_pair(dev, s);
    auto it = g_scratch.find(key);
    if (it != g_scratch.end()) return it->second;
    auto *ss = new StreamScratch();
    ss->device = dev;
    ss->stream = s;
    g_scratch[key] = ss;
    return ss;
}

xs_status refuse_if_capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone)
        return set_error(XS_EINVAL,
                         "scratch must grow while the stream is being captured; run the same "
                         "call once outside capture first");
    return XS_OK;
}

}  // namespace

xs_status scratch(hipStream_t s, Slot slot, size_t bytes, void **ptr) {
    StreamScratch *ss = scratch_for(s);
    Buffer &b = ss->slot[slot];
    if (bytes == 0) bytes = 1;
    if (b.bytes < bytes) {
        XS_TRY(refuse_if_capturing(s));
        XS_HIP(hipStreamSynchronize(s));  // earlier work on this stream may use the old buffer
        if (b.dev) XS_HIP(hipFree(b.dev));
        b.dev = nullptr;
        b.bytes = 0;
        const size_t want = bytes + bytes / 4;  // headroom against frequent regrowth
        hipError_t e = hipMalloc(&b.dev, want);
        if (e != hipSuccess) {
            b.dev = nullptr;
            (void)hipGetLastError();
            return set_error(XS_ENOMEM, "scratch slot %d: cannot allocate %zu bytes (%s)", int(slot),
                             want, hipGetErrorString(e));
        }
        b.bytes = want;
    }
    *ptr = b.dev;
    return XS_OK;
}

xs_status upload(hipStream_t s, Slot slot, const void *host, size_t bytes, void **dev) {
    XS_TRY(scratch(s, slot, bytes, dev));
    StreamScratch *ss = scratch_for(s);
    Buffer &b = ss->slot[slot];
    if (b.pinned_bytes < bytes) {
        XS_TRY(refuse_if_capturing(s));
        if (b.copied) XS_HIP(hipEventSynchronize(b.copied));
        if (b.pinned) XS_HIP(hipHostFree(b.pinned));
        b.pinned = nullptr;
        b.pinned_bytes = 0;
        XS_HIP(hipHostMalloc(&b.pinned, bytes + bytes / 4, hipHostMallocDefault));
        b.pinned_bytes = bytes + bytes / 4;
    }
    if (!b.copied) XS_HIP(hipEventCreateWithFlags(&b.copied, hipEventDisableTiming));
    else XS_HIP(hipEventSynchronize(b.copied));  // previous copy out of `pinned` finished
    std::memcpy(b.pinned, host, bytes);
    XS_HIP(hipMemcpyAsync(*dev, b.pinned, bytes, hipMemcpyHostToDevice, s));
    XS_HIP(hipEventRecord(b.copied, s));
    return XS_OK;
}

xs_status stage_copy(hipStream_t s, Slot slot, const void *host, size_t bytes, void *dst) {
    StreamScratch *ss = scratch_for(s);
    Buffer &b = ss->slot[slot];
    if (b.pinned_bytes < bytes) {
        XS_TRY(refuse_if_capturing(s));
        if (b.copied) XS_HIP(hipEventSynchronize(b.copied));
        if (b.pinned) XS_HIP(hipHostFree(b.pinned));
        b.pinned = nullptr;
        b.pinned_bytes = 0;
        XS_HIP(hipHostMalloc(&b.pinned, bytes + bytes / 4, hipHostMallocDefault));
        b.pinned_bytes = bytes + bytes / 4;
    }
    if (!b.copied) XS_HIP(hipEventCreateWithFlags(&b.copied, hipEventDisableTiming));
    else XS_HIP(hipEventSynchronize(b.copied));
    std::memcpy(b.pinned, host, bytes);
    XS_HIP(hipMemcpyAsync(dst, b.pinned, bytes, hipMemcpyHostToDevice, s));
    XS_HIP(hipEventRecord(b.copied, s));
    return XS_OK;
}

void release_all_scratch() {
    std::lock_guard<std::mutex> lk(g_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &kv : g_scratch) {
        StreamScratch *ss = kv.second;
        (void)hipSetDevice(ss->device);
        (void)hipDeviceSynchronize();
        for (auto &b : ss->slot) {
            if (b.dev) (void)hipFree(b.dev);
            if (b.pinned) (void)hipHostFree(b.pinned);
            if (b.copied) (void)hipEventDestroy(b.copied);
        }
        delete ss;
    }
    g_scratch.clear();
    (void)hipSetDevice(cur);
}

// ---------------------------------------------------------------- validation

namespace {

// Defaults: the per-pair form (one sine and cosine per atom-pixel pair in the forward,
// one sine per pair in the adjoint); the factorized lattice forms are opt-in.
xs_tile_shape g_shape[2] = {{64, 4, 64, 0, 0, 0}, {64, 2, 128, 2048, 0, 0}};
std::mutex g_shape_mu;

xs_status expand_batch(const xs_batch *b, std::vector<Segment> &segs, int &max_atoms,
                       int &max_q) {
    if (!b) return set_error(XS_EINVAL, "batch descriptor is NULL");
    if (b->n_sys < 1) return set_error(XS_EINVAL, "n_sys must be >= 1 (got %d)", b->n_sys);
    if (!b->n_atoms || !b->n_q || !b->n_frames || !b->pos_off || !b->f_off || !b->q_off ||
        !b->out_off)
        return set_error(XS_EINVAL, "batch descriptor has a NULL array");
    max_atoms = 0;
    max_q = 0;
    segs.clear();
    for (int s = 0; s < b->n_sys; ++s) {
        const int64_t n = b->n_atoms[s], nq = b->n_q[s];
        const int32_t nf = b->n_frames[s];
        if (n < 0 || n >= (int64_t(1) << 31))
            return set_error(XS_EINVAL, "system %d: n_atoms %lld out of range", s, (long long)n);
        if (nq < 0 || nq >= (int64_t(1) << 31))
            return set_error(XS_EINVAL, "system %d: n_q %lld out of range", s, (long long)nq);
        if (nf < 1) return set_error(XS_EINVAL, "system %d: n_frames must be >= 1", s);
        if (b->pos_off[s] < 0 || b->f_off[s] < 0 || b->q_off[s] < 0 || b->out_off[s] < 0)
            return set_error(XS_EINVAL, "system %d: negative offset", s);
        for (int32_t t = 0; t < nf; ++t) {
            Segment sg;
            sg.pos = b->pos_off[s] + static_cast<int64_t>(t) * n;
            sg.f = b->f_off[s];
            sg.q = b->q_off[s];
            sg.out = b->out_off[s] + static_cast<int64_t>(t) * nq;
            sg.n_atoms = static_cast<int32_t>(n);
            sg.n_q = static_cast<int32_t>(nq);
            sg.sys = s;
            sg.frame = t;
            segs.push_back(sg);
        }
        max_atoms = std::max<int>(max_atoms, static_cast<int>(n));
        max_q = std::max<int>(max_q, static_cast<int>(nq));
    }
    if (segs.size() > 65535)
        return set_error(XS_ENOTSUP, "at most 65535 (system, frame) segments per call (got %zu)",
                         segs.size());
    return XS_OK;
}

xs_status check_box(const xs_batch *b) {
    if (!b->box) return set_error(XS_EINVAL, "FP32C needs the box edges (box is NULL)");
    for (int s = 0; s < b->n_sys; ++s)
        for (int c = 0; c < 3; ++c) {
            const double L = b->box[3 * s + c];
            if (!(L > 0.0) || !std::isfinite(L))
                return set_error(XS_EINVAL, "system %d: box edge %d must be finite and > 0", s, c);
        }
    return XS_OK;
}

xs_status read_edges(const double *edges, int32_t n_rings, RingEdges &out) {
    if (!edges) return set_error(XS_EINVAL, "ring_edges is NULL");
    if (n_rings < 1 || n_rings > kMaxRings)
        return set_error(n_rings > kMaxRings ? XS_ENOTSUP : XS_EINVAL,
                         "n_rings must be in [1, %d] (got %d)", kMaxRings, n_rings);
    for (int r = 0; r <= n_rings; ++r) {
        if (!std::isfinite(edges[r])) return set_error(XS_EINVAL, "ring edge %d is not finite", r);
        if (r > 0 && !(edges[r - 1] < edges[r]))
            return set_error(XS_EINVAL, "ring edges must increase strictly (edge %d)", r);
        out.e[r] = edges[r];
    }
    for (int r = n_rings + 1; r <= kMaxRings; ++r) out.e[r] = 0.0;
    out.n_rings = n_rings;
    return XS_OK;
}

xs_status begin(void *stream) {
    (void)stream;
    g_last_error.clear();
    return XS_OK;
}

}  // namespace
}  // namespace xs

using namespace xs;

extern "C" {

xs_status xs_intensity_direct(const xs_batch *b, const double *pos, const double *f,
                              const double *q, int32_t precision, double *I_out,
                              double *amp_out, void *stream) {
    XS_TRY(begin(stream));
    std::vector<Segment> segs;
    int max_atoms = 0, max_q = 0;
    XS_TRY(expand_batch(b, segs, max_atoms, max_q));
    if (max_q > 0 && (!q || !I_out)) return set_error(XS_EINVAL, "q / I_out is NULL");
    if (max_atoms > 0 && (!pos || !f)) return set_error(XS_EINVAL, "pos / f is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (precision == XS_FP64)
        return fp64_forward(s, segs.data(), static_cast<int>(segs.size()), max_q, pos, f, q, I_out,
                            amp_out);
    if (precision == XS_FP32C) {
        XS_TRY(check_box(b));
        xs_tile_shape fsh, gsh;
        {
            std::lock_guard<std::mutex> lk(g_shape_mu);
            fsh = g_shape[0];
            gsh = g_shape[1];
        }
        return fp32c_forward(s, segs.data(), static_cast<int>(segs.size()), b->box, pos, f, q, I_out,
                             amp_out, fsh, gsh);
    }
    return set_error(XS_EINVAL, "precision must be XS_FP64 (0) or XS_FP32C (1), got %d", precision);
}

xs_status xs_intensity_grad(const xs_batch *b, const double *pos, const double *f,
                            const double *q, const double *amp, const double *dL_dI,
                            int32_t precision, float *dL_dr, double *dL_dr64, void *stream) {
    XS_TRY(begin(stream));
    std::vector<Segment> segs;
    int max_atoms = 0, max_q = 0;
    XS_TRY(expand_batch(b, segs, max_atoms, max_q));
    if (!dL_dr && !dL_dr64) return set_error(XS_EINVAL, "both dL_dr and dL_dr64 are NULL");
    if (max_atoms > 0 && (!pos || !f)) return set_error(XS_EINVAL, "pos / f is NULL");
    if (max_q > 0 && (!q || !amp || !dL_dI)) return set_error(XS_EINVAL, "q / amp / dL_dI is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (precision == XS_FP64)
        return fp64_grad(s, segs.data(), static_cast<int>(segs.size()), max_atoms, pos, f, q, amp,
                         dL_dI, dL_dr, dL_dr64);
    if (precision == XS_FP32C) {
        XS_TRY(check_box(b));
        xs_tile_shape fsh, gsh;
        {
            std::lock_guard<std::mutex> lk(g_shape_mu);
            fsh = g_shape[0];
            gsh = g_shape[1];
        }
        return fp32c_grad(s, segs.data(), static_cast<int>(segs.size()), b->box, pos, f, q, amp,
                          dL_dI, dL_dr, dL_dr64, fsh, gsh);
    }
    return set_error(XS_EINVAL, "precision must be XS_FP64 (0) or XS_FP32C (1), got %d", precision);
}

static xs_status check_species_args(int32_t n_species, const double *coef) {
    if (n_species < 1 || n_species > 4096) return set_error(XS_EINVAL, "n_species must be in [1, 4096]");
    if (!coef) return set_error(XS_EINVAL, "form-factor coefficients are NULL");
    for (int i = 0; i < 9 * n_species; ++i)
        if (!std::isfinite(coef[i])) return set_error(XS_EINVAL, "form-factor coefficient %d is not finite", i);
    return XS_OK;
}

xs_status xs_intensity_species(const xs_batch *b, const double *pos, const int32_t *species, int32_t n_species,
                               const double *ff_coef, const double *q, int32_t precision, double *I_out,
                               double *amp_out, void *stream) {
    XS_TRY(begin(stream));
    std::vector<Segment> segs;
    int max_atoms = 0, max_q = 0;
    XS_TRY(expand_batch(b, segs, max_atoms, max_q));
    XS_TRY(check_species_args(n_species, ff_coef));
    if (max_q > 0 && (!q || !I_out)) return set_error(XS_EINVAL, "q / I_out is NULL");
    if (max_atoms > 0 && (!pos || !species)) return set_error(XS_EINVAL, "pos / species is NULL");
    if (precision != XS_FP64 && precision != XS_FP32C)
        return set_error(XS_EINVAL, "precision must be XS_FP64 (0) or XS_FP32C (1), got %d", precision);
    if (precision == XS_FP32C) XS_TRY(check_box(b));
    xs_tile_shape fsh, gsh;
    {
        std::lock_guard<std::mutex> lk(g_shape_mu);
        fsh = g_shape[0];
        gsh = g_shape[1];
    }
    return species_forward(static_cast<hipStream_t>(stream), segs, b->box, pos, species, n_species, ff_coef, q,
                           precision, I_out, amp_out, fsh, gsh);
}

xs_status xs_intensity_species_grad(const xs_batch *b, const double *pos, const int32_t *species,
                                    int32_t n_species, const double *ff_coef, const double *q, const double *amp,
                                    const double *dL_dI, int32_t precision, float *dL_dr, double *dL_dr64,
                                    void *stream) {
    XS_TRY(begin(stream));
    std::vector<Segment> segs;
    int max_atoms = 0, max_q = 0;
    XS_TRY(expand_batch(b, segs, max_atoms, max_q));
    XS_TRY(check_species_args(n_species, ff_coef));
    if (!dL_dr && !dL_dr64) return set_error(XS_EINVAL, "both dL_dr and dL_dr64 are NULL");
    if (max_atoms > 0 && (!pos || !species)) return set_error(XS_EINVAL, "pos / species is NULL");
    if (max_q > 0 && (!q || !amp || !dL_dI)) return set_error(XS_EINVAL, "q / amp / dL_dI is NULL");
    if (precision != XS_FP64 && precision != XS_FP32C)
        return set_error(XS_EINVAL, "precision must be XS_FP64 (0) or XS_FP32C (1), got %d", precision);
    if (precision == XS_FP32C) XS_TRY(check_box(b));
    xs_tile_shape fsh, gsh;
    {
        std::lock_guard<std::mutex> lk(g_shape_mu);
        fsh = g_shape[0];
        gsh = g_shape[1];
    }
    return species_grad(static_cast<hipStream_t>(stream), segs, b->box, pos, species, n_species, ff_coef, q, amp,
                        dL_dI, precision, dL_dr, dL_dr64, fsh, gsh);
}

xs_status xs_g2_rings(const double *I, int64_t n_frames, int64_t n_q, const double *q,
                      const double *ring_edges, int32_t n_rings, int32_t n_tau, double *g2_out,
                      int32_t *ring_count, void *stream) {
    XS_TRY(begin(stream));
    if (n_frames < 1) return set_error(XS_EINVAL, "n_frames must be >= 1");
    if (n_q < 0 || n_q >= (int64_t(1) << 31)) return set_error(XS_EINVAL, "n_q out of range");
    if (n_tau < 1 || n_tau > n_frames) return set_error(XS_EINVAL, "n_tau must be in [1, n_frames]");
    if (!g2_out) return set_error(XS_EINVAL, "g2_out is NULL");
    if (n_q > 0 && (!I || !q)) return set_error(XS_EINVAL, "I / q is NULL");
    RingEdges e;
    XS_TRY(read_edges(ring_edges, n_rings, e));
    return g2_rings(static_cast<hipStream_t>(stream), I, n_frames, n_q, q, e, n_tau, g2_out,
                    ring_count);
}

xs_status xs_g2_rings_noalloc(const double *I, int64_t n_frames, int64_t n_q, const double *q,
                              const double *ring_edges, int32_t n_rings, int32_t n_tau, double *g2_out,
                              int32_t *ring_count, void *stream) {
    XS_TRY(begin(stream));
    if (n_frames < 1) return set_error(XS_EINVAL, "n_frames must be >= 1");
    if (n_q < 0 || n_q >= (int64_t(1) << 31)) return set_error(XS_EINVAL, "n_q out of range");
    if (n_tau < 1 || n_tau > n_frames) return set_error(XS_EINVAL, "n_tau must be in [1, n_frames]");
    if (!g2_out) return set_error(XS_EINVAL, "g2_out is NULL");
    if (n_q > 0 && (!I || !q)) return set_error(XS_EINVAL, "I / q is NULL");
    // the largest working set (per-pixel lag rows) must fit the fixed array; the call
    // re-checks the exact total as it carves the buffers
    if (static_cast<double>(n_q) * n_tau * sizeof(double) > static_cast<double>(g2_fixed_scratch_bytes()))
        return set_error(XS_EINVAL, "n_q * n_tau * 8 = %.0f bytes exceeds the %zu-byte fixed scratch",
                         static_cast<double>(n_q) * n_tau * sizeof(double), g2_fixed_scratch_bytes());
    RingEdges e;
    XS_TRY(read_edges(ring_edges, n_rings, e));
    return g2_rings_fixed(static_cast<hipStream_t>(stream), I, n_frames, n_q, q, e, n_tau, g2_out, ring_count);
}

xs_status xs_xsvs_contrast(const double *I, int64_t n_frames, int64_t n_q, const double *q,
                           const double *ring_edges, int32_t n_rings, int32_t n_levels,
                           double *beta_out, double *beta_win, void *stream) {
    XS_TRY(begin(stream));
    if (n_frames < 1) return set_error(XS_EINVAL, "n_frames must be >= 1");
    if (n_q < 0 || n_q >= (int64_t(1) << 31)) return set_error(XS_EINVAL, "n_q out of range");
    if (n_levels < 1 || n_levels > 62 || (int64_t(1) << (n_levels - 1)) > n_frames)
        return set_error(XS_EINVAL, "n_levels must satisfy 1 <= n_levels and 2^(n_levels-1) <= n_frames");
    if (!beta_out) return set_error(XS_EINVAL, "beta_out is NULL");
    if (n_q > 0 && (!I || !q)) return set_error(XS_EINVAL, "I / q is NULL");
    RingEdges e;
    XS_TRY(read_edges(ring_edges, n_rings, e));
    return xsvs_contrast(static_cast<hipStream_t>(stream), I, n_frames, n_q, q, e, n_levels,
                         beta_out, beta_win);
}

xs_status xs_isf_rings(const double *amp, int64_t n_frames, int64_t n_q, const double *q,
                       const double *ring_edges, int32_t n_rings, int32_t n_tau, double f2_sum,
                       double *F_out, int32_t *ring_count, void *stream) {
    XS_TRY(begin(stream));
    if (n_frames < 1) return set_error(XS_EINVAL, "n_frames must be >= 1");
    if (n_q < 0 || n_q >= (int64_t(1) << 31)) return set_error(XS_EINVAL, "n_q out of range");
    if (n_tau < 1 || n_tau > n_frames) return set_error(XS_EINVAL, "n_tau must be in [1, n_frames]");
    if (!(f2_sum > 0.0) || !std::isfinite(f2_sum)) return set_error(XS_EINVAL, "f2_sum must be finite and > 0");
    if (!F_out) return set_error(XS_EINVAL, "F_out is NULL");
    if (n_q > 0 && (!amp || !q)) return set_error(XS_EINVAL, "amp / q is NULL");
    if (n_q > 0 && (reinterpret_cast<uintptr_t>(amp) & 15))
        return set_error(XS_EINVAL, "amp must be 16-byte aligned");
    RingEdges e;
    XS_TRY(read_edges(ring_edges, n_rings, e));
    return isf_rings(static_cast<hipStream_t>(stream), amp, n_frames, n_q, q, e, n_tau, f2_sum, F_out,
                     ring_count);
}

xs_status xs_siegert(const double *g2, const double *F, int32_t n_rings, int32_t n_tau, int32_t n_levels,
                     double *lhs_out, double *fhat2_out, double *beta_out, void *stream) {
    XS_TRY(begin(stream));
    if (n_rings < 1) return set_error(XS_EINVAL, "n_rings must be >= 1");
    if (n_tau < 1) return set_error(XS_EINVAL, "n_tau must be >= 1");
    if (n_levels < 0 || n_levels > 30 || (n_levels > 0 && (int64_t(1) << (n_levels - 1)) > n_tau))
        return set_error(XS_EINVAL, "n_levels must satisfy 0 <= n_levels and 2^(n_levels-1) <= n_tau");
    if (!g2 || !F) return set_error(XS_EINVAL, "g2 / F is NULL");
    if (n_levels > 0 && !beta_out) return set_error(XS_EINVAL, "beta_out is NULL with n_levels > 0");
    return siegert(static_cast<hipStream_t>(stream), g2, F, n_rings, n_tau, n_levels, lhs_out, fhat2_out,
                   beta_out);
}

xs_status xs_frame_sums(const double *I, int64_t n_frames, int64_t n_q, int64_t n_out, int64_t s_out,
                        int64_t n_sum, int64_t s_sum, double scale, double *J_out, void *stream) {
    XS_TRY(begin(stream));
    if (n_frames < 1) return set_error(XS_EINVAL, "n_frames must be >= 1");
    if (n_q < 0 || n_q >= (int64_t(1) << 31)) return set_error(XS_EINVAL, "n_q out of range");
    if (n_out < 1 || n_sum < 1 || s_out < 0 || s_sum < 0)
        return set_error(XS_EINVAL, "need n_out >= 1, n_sum >= 1, s_out >= 0, s_sum >= 0");
    if (n_out > (int64_t(1) << 40) || n_sum > (int64_t(1) << 40) || s_out > (int64_t(1) << 40) ||
        s_sum > (int64_t(1) << 40) || (n_out - 1) * s_out + (n_sum - 1) * s_sum >= n_frames)
        return set_error(XS_EINVAL, "frame index (n_out-1)*s_out + (n_sum-1)*s_sum must be < n_frames");
    if (n_q > 0 && (!I || !J_out)) return set_error(XS_EINVAL, "I / J_out is NULL");
    if (!std::isfinite(scale)) return set_error(XS_EINVAL, "scale must be finite");
    return frame_sums(static_cast<hipStream_t>(stream), I, n_q, n_out, s_out, n_sum, s_sum, scale, J_out);
}

xs_status xs_ring_histogram(const double *I, int64_t n_frames, int64_t n_q, const double *q,
                            const double *ring_edges, int32_t n_rings, int32_t n_bins, double kappa_max,
                            int64_t *counts_out, double *mean_out, void *stream) {
    XS_TRY(begin(stream));
    if (n_frames < 1 || n_frames > 65535) return set_error(XS_EINVAL, "n_frames must be in [1, 65535]");
    if (n_q < 0 || n_q >= (int64_t(1) << 31)) return set_error(XS_EINVAL, "n_q out of range");
    if (n_bins < 1) return set_error(XS_EINVAL, "n_bins must be >= 1");
    if (!(kappa_max > 0.0) || !std::isfinite(kappa_max)) return set_error(XS_EINVAL, "kappa_max must be > 0");
    if (!counts_out) return set_error(XS_EINVAL, "counts_out is NULL");
    if (n_q > 0 && (!I || !q)) return set_error(XS_EINVAL, "I / q is NULL");
    RingEdges e;
    XS_TRY(read_edges(ring_edges, n_rings, e));
    return ring_histogram(static_cast<hipStream_t>(stream), I, n_frames, n_q, q, e, n_bins, kappa_max, counts_out,
                          mean_out);
}

const char *xs_last_error(void) { return g_last_error.c_str(); }

int32_t xs_version(void) { return 100; }

xs_status xs_shutdown(void) {
    release_fft_plans();
    release_all_scratch();
    return XS_OK;
}

xs_status xs_fft_intensity(const double *pos, const double *f, int64_t n_atoms, double box, int32_t n_grid,
                           double eta, int32_t k, double *I_out, double *amp_out, void *stream) {
    XS_TRY(begin(stream));
    if (n_atoms < 0 || n_atoms >= (int64_t(1) << 40)) return set_error(XS_EINVAL, "n_atoms out of range");
    if (n_grid < 2 || n_grid > 1024) return set_error(XS_EINVAL, "n_grid must be in [2, 1024]");
    if (!(box > 0.0) || !std::isfinite(box)) return set_error(XS_EINVAL, "box must be positive and finite");
    if (!(eta > 0.0) || !std::isfinite(eta)) return set_error(XS_EINVAL, "eta must be positive and finite");
    if (k < 1 || k > n_grid) return set_error(XS_EINVAL, "k must be in [1, n_grid]");
    if (!I_out) return set_error(XS_EINVAL, "I_out is NULL");
    if (n_atoms > 0 && (!pos || !f)) return set_error(XS_EINVAL, "pos / f is NULL");
    return fft_intensity(static_cast<hipStream_t>(stream), pos, f, n_atoms, box, n_grid, eta, k, I_out, amp_out);
}

xs_status xs_speckle_loss(const double *I, const double *I_target, int64_t n, double *loss_out,
                          double *dL_dI, void *stream) {
    XS_TRY(begin(stream));
    if (n < 0) return set_error(XS_EINVAL, "n must be >= 0");
    if (!loss_out) return set_error(XS_EINVAL, "loss_out is NULL");
    if (n > 0 && (!I || !I_target)) return set_error(XS_EINVAL, "I / I_target is NULL");
    return speckle_loss(static_cast<hipStream_t>(stream), I, I_target, n, loss_out, dL_dI);
}

xs_status xs_position_step(double *pos, const float *dL_dr, const double *dL_dr64, int64_t n,
                           double step, void *stream) {
    XS_TRY(begin(stream));
    if (n < 0) return set_error(XS_EINVAL, "n must be >= 0");
    if (!std::isfinite(step)) return set_error(XS_EINVAL, "step must be finite");
    if (n > 0 && (!pos || (!dL_dr && !dL_dr64))) return set_error(XS_EINVAL, "pos / gradient is NULL");
    return position_step(static_cast<hipStream_t>(stream), pos, dL_dr, dL_dr64, n, step);
}

xs_status xs_timing_enable(int32_t on) { return timing_enable(on); }

xs_status xs_timing_read(int32_t kind, double *total_ms, int64_t *launches, double *work) {
    return timing_read(kind, total_ms, launches, work);
}

xs_status xs_roofline_probe(int32_t kind, int64_t bytes, double *rate, void *stream) {
    XS_TRY(begin(stream));
    if (!rate) return set_error(XS_EINVAL, "rate is NULL");
    return roofline_probe(static_cast<hipStream_t>(stream), kind, bytes, rate);
}

namespace {
// Work lists, buffers and pixel order of an FP32C pair-sum plan over `segs`.
xs_status build_pair_plan(hipStream_t s, xs::Plan &plan, const std::vector<Segment> &segs, const double *box,
                          const double *q, const xs_tile_shape &fsh, const xs_tile_shape &gsh,
                          bool with_grad = true) {
    const int n = static_cast<int>(segs.size());
    plan.with_grad = with_grad;
    XS_TRY(plan.find_lattices(s, segs.data(), n, q));
    XS_TRY(plan.build(segs.data(), n, box, fsh, gsh));
    XS_TRY(plan.allocate(s, true));
    return plan.sort_pixels(s, q);
}
}  // namespace

struct xs_plan {
    xs::Plan plan;                         // pair sums (of the species segments for a species plan)
    xs::SpeciesPlan *species = nullptr;    // species split and buffers, or NULL
    int device = 0;
    const double *q = nullptr;
    int64_t total_out = 0;
    int64_t total_pos = 0;
    ~xs_plan() {
        if (species) xs::species_plan_destroy(species);
    }
};

namespace {
xs_status plan_create(const xs_batch *b, const double *q, xs_plan **out, void *stream, bool with_grad) {
    XS_TRY(begin(stream));
    if (!out) return set_error(XS_EINVAL, "plan output pointer is NULL");
    *out = nullptr;
    std::vector<Segment> segs;
    int max_atoms = 0, max_q = 0;
    XS_TRY(expand_batch(b, segs, max_atoms, max_q));
    XS_TRY(check_box(b));
    if (max_q > 0 && !q) return set_error(XS_EINVAL, "q is NULL");
    xs_tile_shape fsh, gsh;
    {
        std::lock_guard<std::mutex> lk(g_shape_mu);
        fsh = g_shape[0];
        gsh = g_shape[1];
    }
    auto *p = new (std::nothrow) xs_plan();
    if (!p) return set_error(XS_ENOMEM, "plan: host allocation failed");
    hipStream_t s = static_cast<hipStream_t>(stream);
    xs_status st = build_pair_plan(s, p->plan, segs, b->box, q, fsh, gsh, with_grad);
    if (st != XS_OK) {
        delete p;
        return st;
    }
    (void)hipGetDevice(&p->device);
    p->q = q;
    for (const Segment &g : segs) {
        p->total_out += g.n_q;
        p->total_pos += g.n_atoms;
    }
    *out = p;
    return XS_OK;
}
}  // namespace

xs_status xs_plan_create(const xs_batch *b, const double *q, xs_plan **out, void *stream) {
    return plan_create(b, q, out, stream, true);
}

xs_status xs_plan_create_forward(const xs_batch *b, const double *q, xs_plan **out, void *stream) {
    return plan_create(b, q, out, stream, false);
}

xs_status xs_plan_create_species(const xs_batch *b, const double *q, const int32_t *species, int32_t n_species,
                                 const double *ff_coef, xs_plan **out, void *stream) {
    XS_TRY(begin(stream));
    if (!out) return set_error(XS_EINVAL, "plan output pointer is NULL");
    *out = nullptr;
    std::vector<Segment> segs;
    int max_atoms = 0, max_q = 0;
    XS_TRY(expand_batch(b, segs, max_atoms, max_q));
    XS_TRY(check_box(b));
    XS_TRY(check_species_args(n_species, ff_coef));
    if (max_q > 0 && !q) return set_error(XS_EINVAL, "q is NULL");
    if (max_atoms > 0 && !species) return set_error(XS_EINVAL, "species is NULL");
    xs_tile_shape fsh, gsh;
    {
        std::lock_guard<std::mutex> lk(g_shape_mu);
        fsh = g_shape[0];
        gsh = g_shape[1];
    }
    auto *p = new (std::nothrow) xs_plan();
    if (!p) return set_error(XS_ENOMEM, "plan: host allocation failed");
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<Segment> sub;
    xs_status st = species_plan_create(s, segs, species, n_species, ff_coef, &p->species, &sub);
    if (st == XS_OK && !sub.empty()) st = build_pair_plan(s, p->plan, sub, b->box, q, fsh, gsh);
    if (st != XS_OK) {
        delete p;
        return st;
    }
    (void)hipGetDevice(&p->device);
    p->q = q;
    for (const Segment &g : segs) {
        p->total_out += g.n_q;
        p->total_pos += g.n_atoms;
    }
    *out = p;
    return XS_OK;
}

xs_status xs_plan_intensity(xs_plan *p, const double *pos, const double *f, double *I_out,
                            double *amp_out, void *stream) {
    XS_TRY(begin(stream));
    if (!p) return set_error(XS_EINVAL, "plan is NULL");
    if (p->species) return set_error(XS_EINVAL, "species plan: use xs_plan_intensity_species");
    if (p->total_out > 0 && !I_out) return set_error(XS_EINVAL, "I_out is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    XS_TRY(p->plan.tile_atoms(s, pos, f));
    return p->plan.forward(s, p->q, I_out, amp_out);
}

xs_status xs_plan_grad(xs_plan *p, const double *pos, const double *f, const double *amp,
                       const double *dL_dI, int32_t retile, float *dL_dr, double *dL_dr64,
                       void *stream) {
    XS_TRY(begin(stream));
    if (!p) return set_error(XS_EINVAL, "plan is NULL");
    if (p->species) return set_error(XS_EINVAL, "species plan: use xs_plan_grad_species");
    if (!p->plan.with_grad) return set_error(XS_EINVAL, "the plan was created for the forward only");
    if (p->total_pos > 0 && !dL_dr && !dL_dr64) return set_error(XS_EINVAL, "both dL_dr and dL_dr64 are NULL");
    if (p->total_out > 0 && (!amp || !dL_dI)) return set_error(XS_EINVAL, "amp / dL_dI is NULL");
    if (!retile && !p->plan.tiled)
        return set_error(XS_EINVAL, "retile = 0 needs the atom tiles of an earlier xs_plan_intensity on this plan");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (retile) XS_TRY(p->plan.tile_atoms(s, pos, f));
    return p->plan.grad(s, p->q, f, amp, dL_dI, dL_dr, dL_dr64);
}

xs_status xs_plan_intensity_species(xs_plan *p, const double *pos, double *I_out, double *amp_out,
                                    void *stream) {
    XS_TRY(begin(stream));
    if (!p) return set_error(XS_EINVAL, "plan is NULL");
    if (!p->species) return set_error(XS_EINVAL, "not a species plan: use xs_plan_intensity");
    if (p->total_out > 0 && !I_out) return set_error(XS_EINVAL, "I_out is NULL");
    return species_plan_forward(static_cast<hipStream_t>(stream), p->species, p->plan, p->q, pos, I_out, amp_out);
}

xs_status xs_plan_grad_species(xs_plan *p, const double *pos, const double *amp, const double *dL_dI,
                               int32_t retile, float *dL_dr, double *dL_dr64, void *stream) {
    XS_TRY(begin(stream));
    if (!p) return set_error(XS_EINVAL, "plan is NULL");
    if (!p->species) return set_error(XS_EINVAL, "not a species plan: use xs_plan_grad");
    if (p->total_pos > 0 && !dL_dr && !dL_dr64) return set_error(XS_EINVAL, "both dL_dr and dL_dr64 are NULL");
    if (p->total_out > 0 && (!amp || !dL_dI)) return set_error(XS_EINVAL, "amp / dL_dI is NULL");
    return species_plan_grad(static_cast<hipStream_t>(stream), p->species, p->plan, p->q, pos, amp, dL_dI, retile,
                             dL_dr, dL_dr64);
}

xs_status xs_plan_destroy(xs_plan *p) {
    if (!p) return XS_OK;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    delete p;
    (void)hipSetDevice(cur);
    return XS_OK;
}

xs_status xs_plan_describe(const xs_plan *p, xs_plan_info *info) {
    if (!p || !info) return set_error(XS_EINVAL, "plan and info must be non-NULL");
    int nl = 0, nr = 0, nf = 0, ng = 0;
    p->plan.describe(&nl, &nr, &nf, &ng);
    info->n_segments = p->plan.n_seg;
    info->n_lattice_segments = nl;
    info->n_row_segments = nr;
    info->pad = 0;
    info->n_forward_items = nf;
    info->n_gradient_items = ng;
    info->device_bytes = static_cast<int64_t>(p->plan.device_bytes) +
                         (p->species ? static_cast<int64_t>(species_plan_bytes(p->species)) : 0);
    return XS_OK;
}

xs_status xs_get_tile_shape(int32_t kind, xs_tile_shape *out) {
    if ((kind != 0 && kind != 1) || !out) return set_error(XS_EINVAL, "kind must be 0 or 1, out non-NULL");
    std::lock_guard<std::mutex> lk(g_shape_mu);
    *out = g_shape[kind];
    return XS_OK;
}

xs_status xs_set_tile_shape(int32_t kind, const xs_tile_shape *shape) {
    if ((kind != 0 && kind != 1) || !shape) return set_error(XS_EINVAL, "kind must be 0 or 1, shape non-NULL");
    const int ql = shape->q_per_lane;
    if (shape->atoms_per_tile != 64)
        return set_error(XS_ENOTSUP, "atoms_per_tile: only 64 is built (got %d)", shape->atoms_per_tile);
    if (ql != 1 && ql != 2 && ql != 4 && ql != 8 && ql != 32)
        return set_error(XS_EINVAL, "q_per_lane must be 1, 2, 4, 8 or 32 (got %d)", ql);
    if (ql == 32 && shape->waves_per_simd != 0 && !(kind == 0 && shape->waves_per_simd == 3))
        return set_error(XS_ENOTSUP, "the matrix-core lattice form (q_per_lane 32) is built without a register bound, "
                                     "and for the forward also bounded to 3 waves per SIMD");
    if (kind == 0 && shape->atom_split < 1) return set_error(XS_EINVAL, "atom_split must be >= 1");
    if (kind == 1 && (shape->pixel_split < 64 || shape->pixel_split % 64))
        return set_error(XS_EINVAL, "pixel_split must be a positive multiple of 64");
    if (shape->waves_per_simd != 0 && shape->waves_per_simd != 3 && shape->waves_per_simd != 4 &&
        shape->waves_per_simd != 5)
        return set_error(XS_EINVAL, "waves_per_simd must be 0, 3, 4 or 5");
    if (shape->waves_per_simd == 3 && !(kind == 0 && (ql == 32 || ql == 8)))
        return set_error(XS_ENOTSUP, "the 3-waves-per-SIMD variant is built for the forward at q_per_lane 8 (row "
                                     "form) and 32 (matrix-core form)");
    if (shape->waves_per_simd == 4 && !((kind == 0 && (ql == 2 || ql == 4 || ql == 8)) || (kind == 1 && ql == 4)))
        return set_error(XS_ENOTSUP, "the 4-waves-per-SIMD variant is built for forward q_per_lane 2, 4, 8 "
                                     "and gradient q_per_lane 4");
    if (shape->waves_per_simd == 5 && !(kind == 1 && ql == 2))
        return set_error(XS_ENOTSUP, "the 5-waves-per-SIMD variant is built for gradient q_per_lane 2");
    if (shape->lattice < 0 || shape->lattice > 2) return set_error(XS_EINVAL, "lattice must be 0, 1 or 2");
    std::lock_guard<std::mutex> lk(g_shape_mu);
    g_shape[kind] = *shape;
    return XS_OK;
}

}  // extern "C"
