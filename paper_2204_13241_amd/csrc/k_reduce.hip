// Reductions of the speckle intensities (Sec. 2.3):
//   g2 on |q| rings, Eq. (g2_def) with the ring mean of Sec. 4.2;
//   XSVS contrast versus exposure, Eqs. (inte_Iq), (bq_Iq).
// Every floating-point sum has a fixed order (time sums sequential in t, ring
// sums sequential in ascending pixel index, window sums pairwise), so results
// are bit-for-bit reproducible.  Inputs are HBM-resident FP64 intensities
// I[t][p] (pixel fastest); these kernels are bandwidth/latency bound.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "xs_internal.h"

namespace xs {
namespace {

constexpr int kBlock = 256;
constexpr int kPartChunk = 1024;  // pixels per partition block

// Ring of each pixel: r with e_r <= |q| < e_{r+1}, |q| = sqrt(fma(qz,qz,fma(qy,qy,qx*qx))),
// else -1.  If `I` is given (g2), a pixel whose time mean squares to zero gets -1.
__global__ __launch_bounds__(kBlock) void k_ring_key(const double *__restrict__ q, int64_t n_q,
                                                     RingEdges edges, int32_t *__restrict__ key) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (p >= n_q) return;
    const double qx = q[3 * p], qy = q[3 * p + 1], qz = q[3 * p + 2];
    const double qn = __builtin_sqrt(__builtin_fma(qz, qz, __builtin_fma(qy, qy, qx * qx)));
    int32_t r = -1;
    if (edges.e[0] <= qn && qn < edges.e[edges.n_rings]) {
        int lo = 0, hi = edges.n_rings;  // invariant: e[lo] <= qn < e[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (edges.e[mid] <= qn) lo = mid; else hi = mid;
        }
        r = lo;
    }
    key[p] = r;
}

// Per-block ring counts: cnt[b * R + r] = #pixels of block b with key r.
__global__ __launch_bounds__(kBlock) void k_part_count(const int32_t *__restrict__ key,
                                                       int64_t n_q, int32_t R,
                                                       int32_t *__restrict__ cnt) {
    __shared__ int32_t h[kMaxRings];
    for (int r = threadIdx.x; r < R; r += kBlock) h[r] = 0;
    __syncthreads();
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kPartChunk;
    for (int i = threadIdx.x; i < kPartChunk; i += kBlock) {
        const int64_t p = base + i;
        if (p < n_q) {
            const int32_t k = key[p];
            if (k >= 0) atomicAdd(&h[k], 1);
        }
    }
    __syncthreads();
    for (int r = threadIdx.x; r < R; r += kBlock) cnt[static_cast<int64_t>(blockIdx.x) * R + r] = h[r];
}

// Exclusive offsets: off[b*R + r] = start[r] + sum_{b'<b} cnt[b'*R + r];
// start[r] = sum_{r'<r} total[r'];  ring_start[r] for r = 0..R.  One block.
__global__ __launch_bounds__(kBlock) void k_part_scan(int32_t *__restrict__ cnt, int32_t n_blocks,
                                                      int32_t R, int32_t *__restrict__ ring_start) {
    __shared__ int32_t tot[kMaxRings + 1];
    for (int r = threadIdx.x; r < R; r += kBlock) {
        int32_t run = 0;
        for (int32_t b = 0; b < n_blocks; ++b) {
            const int32_t c = cnt[static_cast<int64_t>(b) * R + r];
            cnt[static_cast<int64_t>(b) * R + r] = run;
            run += c;
        }
        tot[r] = run;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int r = 0; r < R; ++r) {
            const int32_t c = tot[r];
            tot[r] = run;
            ring_start[r] = run;
            run += c;
        }
        ring_start[R] = run;
        tot[R] = run;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < R; r += kBlock)
        for (int32_t b = 0; b < n_blocks; ++b) cnt[static_cast<int64_t>(b) * R + r] += tot[r];
}

// Stable scatter: the pixels of ring r appear in ascending index order.
// Thread r walks the block's keys in order and appends its ring's pixels.
__global__ __launch_bounds__(kBlock) void k_part_scatter(const int32_t *__restrict__ key,
                                                         int64_t n_q, int32_t R,
                                                         const int32_t *__restrict__ off,
                                                         int32_t *__restrict__ list) {
    __shared__ int32_t k_s[kPartChunk];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kPartChunk;
    for (int i = threadIdx.x; i < kPartChunk; i += kBlock) {
        const int64_t p = base + i;
        k_s[i] = p < n_q ? key[p] : -1;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < R; r += kBlock) {
        int32_t o = off[static_cast<int64_t>(blockIdx.x) * R + r];
        for (int i = 0; i < kPartChunk; ++i)
            if (k_s[i] == r) list[o++] = static_cast<int32_t>(base + i);
    }
}

// g2, per pixel: mean over all F frames, then G_p(tau) for tau < n_tau.
// A block owns `pw` consecutive pixels whose time series sit in LDS as
// lds[t * pw + pp]; thread (pp, tau-slot) loops over its lags.
// used[p] = 1 if <I>_t^2 != 0.
__global__ __launch_bounds__(kBlock) void k_g2_pixel(const double *__restrict__ I, int64_t F,
                                                     int64_t n_q, int32_t n_tau, int32_t pw,
                                                     double *__restrict__ G,
                                                     int32_t *__restrict__ used) {
    extern __shared__ double lds[];
    double *den_s = lds + F * pw;
    const int64_t p0 = static_cast<int64_t>(blockIdx.x) * pw;
    for (int64_t i = threadIdx.x; i < F * pw; i += kBlock) {
        const int64_t t = i / pw, pp = i - t * pw;
        const int64_t p = p0 + pp;
        lds[i] = p < n_q ? I[t * n_q + p] : 0.0;
    }
    __syncthreads();
    if (threadIdx.x < pw) {
        double S = 0.0;
        for (int64_t t = 0; t < F; ++t) S = S + lds[t * pw + threadIdx.x];
        const double mean = S / static_cast<double>(F);
        den_s[threadIdx.x] = mean * mean;
    }
    __syncthreads();
    const int pp = threadIdx.x % pw;
    const int slot = threadIdx.x / pw, n_slots = kBlock / pw;
    const int64_t p = p0 + pp;
    if (p >= n_q) return;
    const double den = den_s[pp];
    if (slot == 0) used[p] = den != 0.0;
    for (int tau = slot; tau < n_tau; tau += n_slots) {
        double acc = 0.0;
        for (int64_t t = 0; t + tau < F; ++t)
            acc = __builtin_fma(lds[t * pw + pp], lds[(t + tau) * pw + pp], acc);
        G[p * n_tau + tau] = (acc / static_cast<double>(F - tau)) / den;
    }
}

// Same per-pixel step reading global memory directly (series too long for LDS).
__global__ __launch_bounds__(kBlock) void k_g2_pixel_global(const double *__restrict__ I, int64_t F,
                                                            int64_t n_q, int32_t n_tau,
                                                            double *__restrict__ G,
                                                            int32_t *__restrict__ used) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (p >= n_q) return;
    double S = 0.0;
    for (int64_t t = 0; t < F; ++t) S = S + I[t * n_q + p];
    const double mean = S / static_cast<double>(F);
    const double den = mean * mean;
    used[p] = den != 0.0;
    for (int tau = 0; tau < n_tau; ++tau) {
        double acc = 0.0;
        for (int64_t t = 0; t + tau < F; ++t)
            acc = __builtin_fma(I[t * n_q + p], I[(t + tau) * n_q + p], acc);
        G[p * n_tau + tau] = (acc / static_cast<double>(F - tau)) / den;
    }
}

__global__ __launch_bounds__(kBlock) void k_mask_unused(int32_t *__restrict__ key,
                                                        const int32_t *__restrict__ used,
                                                        int64_t n_q) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (p < n_q && !used[p]) key[p] = -1;
}

// g2 ring mean: thread (r, tau), pixels of ring r in ascending order.
__global__ __launch_bounds__(kBlock) void k_g2_ring(const double *__restrict__ G, int32_t n_tau,
                                                    int32_t R, const int32_t *__restrict__ list,
                                                    const int32_t *__restrict__ ring_start,
                                                    double *__restrict__ g2,
                                                    int32_t *__restrict__ count) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= static_cast<int64_t>(R) * n_tau) return;
    const int r = static_cast<int>(i / n_tau), tau = static_cast<int>(i - static_cast<int64_t>(r) * n_tau);
    const int32_t a = ring_start[r], b = ring_start[r + 1];
    double sum = 0.0;
    for (int32_t k = a; k < b; ++k) sum = sum + G[static_cast<int64_t>(list[k]) * n_tau + tau];
    const int32_t n = b - a;
    g2[i] = n > 0 ? sum / static_cast<double>(n) : __builtin_nan("");
    if (count && tau == 0) count[r] = n;
}

// XSVS: next dyadic level, J_{l+1}[k][p] = J_l[2k][p] + J_l[2k+1][p].
__global__ __launch_bounds__(kBlock) void k_level_up(const double *__restrict__ src,
                                                     double *__restrict__ dst, int64_t K_next,
                                                     int64_t n_q) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= K_next * n_q) return;
    const int64_t k = i / n_q, p = i - k * n_q;
    dst[i] = src[(2 * k) * n_q + p] + src[(2 * k + 1) * n_q + p];
}

// XSVS per window: thread (r, k); lanes run over consecutive windows k of one
// ring r, pixels of the ring in ascending order; two-pass mean and variance.
__global__ __launch_bounds__(kBlock) void k_xsvs_window(const double *__restrict__ J, int64_t K,
                                                        int64_t n_q, int32_t R,
                                                        const int32_t *__restrict__ list,
                                                        const int32_t *__restrict__ ring_start,
                                                        double *__restrict__ bwin) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= static_cast<int64_t>(R) * K) return;
    const int r = static_cast<int>(i / K);
    const int64_t k = i - static_cast<int64_t>(r) * K;
    const int32_t a = ring_start[r], b = ring_start[r + 1];
    const int32_t n = b - a;
    double beta = __builtin_nan("");
    if (n > 0) {
        const double *row = J + k * n_q;
        double s = 0.0;
        for (int32_t m = a; m < b; ++m) s = s + row[list[m]];
        const double mu = s / static_cast<double>(n);
        double v = 0.0;
        for (int32_t m = a; m < b; ++m) {
            const double d = row[list[m]] - mu;
            v = __builtin_fma(d, d, v);
        }
        const double var = v / static_cast<double>(n);
        beta = var / (mu * mu);
    }
    bwin[k * R + r] = beta;
}

// Mean over windows: beta_out[r] = sum_k bwin[k][r] / K; optional copy to the
// per-window output (rows k >= K filled with NaN).
__global__ __launch_bounds__(kBlock) void k_xsvs_mean(const double *__restrict__ bwin, int64_t K,
                                                      int64_t F, int32_t R,
                                                      double *__restrict__ beta_out,
                                                      double *__restrict__ beta_win_level) {
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= R) return;
    double acc = 0.0;
    for (int64_t k = 0; k < K; ++k) acc = acc + bwin[k * R + r];
    beta_out[r] = acc / static_cast<double>(K);
    if (beta_win_level)
        for (int64_t k = 0; k < F; ++k) beta_win_level[k * R + r] = k < K ? bwin[k * R + r] : __builtin_nan("");
}

unsigned blocks_for(int64_t n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }

// Build the ring-ordered pixel list.  key[] must hold the pixel keys.
xs_status partition(hipStream_t s, int32_t *key, int64_t n_q, int32_t R, int32_t **list_out,
                    int32_t **start_out) {
    const int64_t nb = (n_q + kPartChunk - 1) / kPartChunk;
    void *cnt = nullptr, *list = nullptr;
    XS_TRY(scratch(s, SLOT_RING_CNT, sizeof(int32_t) * (nb * R + R + 1), &cnt));
    XS_TRY(scratch(s, SLOT_RING_LIST, sizeof(int32_t) * std::max<int64_t>(n_q, 1), &list));
    int32_t *c = static_cast<int32_t *>(cnt);
    int32_t *start = c + nb * R;
    if (nb > 0) hipLaunchKernelGGL(k_part_count, dim3(nb), dim3(kBlock), 0, s, key, n_q, R, c);
    hipLaunchKernelGGL(k_part_scan, dim3(1), dim3(kBlock), 0, s, c, static_cast<int32_t>(nb), R, start);
    if (nb > 0)
        hipLaunchKernelGGL(k_part_scatter, dim3(nb), dim3(kBlock), 0, s, key, n_q, R, c,
                           static_cast<int32_t *>(list));
    XS_HIP(hipGetLastError());
    *list_out = static_cast<int32_t *>(list);
    *start_out = start;
    return XS_OK;
}

}  // namespace

xs_status g2_rings(hipStream_t s, const double *I, int64_t F, int64_t n_q, const double *q,
                   const RingEdges &edges, int32_t n_tau, double *g2_out, int32_t *ring_count) {
    const int32_t R = edges.n_rings;
    void *tok = nullptr;
    timer_begin(s, TIMER_G2, &tok);
    void *key = nullptr, *G = nullptr, *used = nullptr;
    XS_TRY(scratch(s, SLOT_RING_KEY, sizeof(int32_t) * std::max<int64_t>(n_q, 1), &key));
    XS_TRY(scratch(s, SLOT_PIXEL2, sizeof(int32_t) * std::max<int64_t>(n_q, 1), &used));
    XS_TRY(scratch(s, SLOT_G, sizeof(double) * std::max<int64_t>(n_q * n_tau, 1), &G));
    int32_t *k = static_cast<int32_t *>(key);
    if (n_q > 0) {
        hipLaunchKernelGGL(k_ring_key, dim3(blocks_for(n_q)), dim3(kBlock), 0, s, q, n_q, edges, k);
        // pixels per block for the LDS path: largest power of two <= 64 with
        // the series (and the per-pixel denominators) in at most 64 KiB
        int pw = 64;
        while (pw > 1 && (F * pw + pw) * static_cast<int64_t>(sizeof(double)) > 65536) pw >>= 1;
        if ((F * pw + pw) * static_cast<int64_t>(sizeof(double)) <= 65536) {
            const size_t lds = sizeof(double) * (F * pw + pw);
            hipLaunchKernelGGL(k_g2_pixel, dim3(static_cast<unsigned>((n_q + pw - 1) / pw)),
                               dim3(kBlock), lds, s, I, F, n_q, n_tau, pw,
                               static_cast<double *>(G), static_cast<int32_t *>(used));
        } else {
            hipLaunchKernelGGL(k_g2_pixel_global, dim3(blocks_for(n_q)), dim3(kBlock), 0, s, I, F,
                               n_q, n_tau, static_cast<double *>(G), static_cast<int32_t *>(used));
        }
        hipLaunchKernelGGL(k_mask_unused, dim3(blocks_for(n_q)), dim3(kBlock), 0, s, k,
                           static_cast<const int32_t *>(used), n_q);
        XS_HIP(hipGetLastError());
    }
    int32_t *list = nullptr, *start = nullptr;
    XS_TRY(partition(s, k, n_q, R, &list, &start));
    hipLaunchKernelGGL(k_g2_ring, dim3(blocks_for(static_cast<int64_t>(R) * n_tau)), dim3(kBlock), 0, s,
                       static_cast<const double *>(G), n_tau, R, list, start, g2_out, ring_count);
    timer_end(s, TIMER_G2, tok, static_cast<double>(F) * n_q * sizeof(double));
    XS_HIP(hipGetLastError());
    return XS_OK;
}

xs_status xsvs_contrast(hipStream_t s, const double *I, int64_t F, int64_t n_q, const double *q,
                        const RingEdges &edges, int32_t n_levels, double *beta_out,
                        double *beta_win) {
    const int32_t R = edges.n_rings;
    void *tok = nullptr;
    timer_begin(s, TIMER_XSVS, &tok);
    void *key = nullptr, *bwin = nullptr, *la = nullptr, *lb = nullptr;
    XS_TRY(scratch(s, SLOT_RING_KEY, sizeof(int32_t) * std::max<int64_t>(n_q, 1), &key));
    XS_TRY(scratch(s, SLOT_BWIN, sizeof(double) * F * R, &bwin));
    if (n_levels > 1) {
        XS_TRY(scratch(s, SLOT_LEVEL_A, sizeof(double) * std::max<int64_t>((F / 2) * n_q, 1), &la));
        if (n_levels > 2)
            XS_TRY(scratch(s, SLOT_LEVEL_B, sizeof(double) * std::max<int64_t>((F / 4) * n_q, 1), &lb));
    }
    int32_t *k = static_cast<int32_t *>(key);
    if (n_q > 0)
        hipLaunchKernelGGL(k_ring_key, dim3(blocks_for(n_q)), dim3(kBlock), 0, s, q, n_q, edges, k);
    int32_t *list = nullptr, *start = nullptr;
    XS_TRY(partition(s, k, n_q, R, &list, &start));
    const double *J = I;
    int64_t K = F;
    for (int32_t l = 0; l < n_levels; ++l) {
        if (l > 0) {
            const int64_t Kn = K / 2;
            double *dst = static_cast<double *>((l & 1) ? la : lb);
            if (Kn * n_q > 0)
                hipLaunchKernelGGL(k_level_up, dim3(blocks_for(Kn * n_q)), dim3(kBlock), 0, s, J, dst,
                                   Kn, n_q);
            J = dst;
            K = Kn;
        }
        hipLaunchKernelGGL(k_xsvs_window, dim3(blocks_for(static_cast<int64_t>(R) * K)), dim3(kBlock), 0,
                           s, J, K, n_q, R, list, start, static_cast<double *>(bwin));
        hipLaunchKernelGGL(k_xsvs_mean, dim3(blocks_for(R)), dim3(kBlock), 0, s,
                           static_cast<const double *>(bwin), K, F, R,
                           beta_out + static_cast<int64_t>(l) * R,
                           beta_win ? beta_win + static_cast<int64_t>(l) * F * R : nullptr);
        XS_HIP(hipGetLastError());
    }
    timer_end(s, TIMER_XSVS, tok, static_cast<double>(F) * n_q * sizeof(double));
    return XS_OK;
}

}  // namespace xs
