// Reductions of the speckle intensities (Sec. 2.3):
//   g2 on |q| rings, Eq. (g2_def) with the ring mean of Sec. 4.2;
//   XSVS contrast versus exposure, Eqs. (inte_Iq), (bq_Iq).
// Every floating-point sum has a fixed order (time sums sequential in t, ring
// sums sequential in ascending pixel index, window sums pairwise), so results
// are bit-for-bit reproducible.  The sequential chains are kept fast by the
// data layout: pixels are renumbered in ring order (ascending index within a
// ring, `rank`), the per-pixel quantities a ring sums over (g2's lag values,
// XSVS's window sums) are stored as rows in that order with the summed-over
// index contiguous, and a block stages a chunk of rows of one ring in LDS with
// all its threads before the owning lanes walk the rows in order.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "xs_internal.h"

namespace xs {
namespace {

constexpr int kBlock = 256;
constexpr int kPartChunk = 1024;  // pixels per partition block
constexpr int kLagBlock = 8;      // lags per thread in the g2 lag kernel
constexpr int kTr = 64;           // transpose tile (frames x pixels)
constexpr int kColTile = 64;      // columns (lags / windows) per ring-sum block
constexpr int kColChunk = 8192;   // doubles staged per chunk (64 KiB of LDS)
constexpr int kColLoads = kColChunk / kBlock;

unsigned blocks_for(int64_t n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }

__global__ __launch_bounds__(kBlock) void k_fill_i32(int32_t *__restrict__ p, int64_t n, int32_t v) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kBlock)
        p[i] = v;
}

// Ring of each pixel: r with e_r <= |q| < e_{r+1}, |q| = sqrt(fma(qz,qz,fma(qy,qy,qx*qx))),
// else -1.
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

// Block r: exclusive scan of cnt[b * R + r] over b in place; tot[r] = total.
__global__ __launch_bounds__(kBlock) void k_part_scan_ring(int32_t *__restrict__ cnt, int64_t nb, int32_t R,
                                                           int32_t *__restrict__ tot) {
    __shared__ int32_t s[kBlock];
    const int r = blockIdx.x;
    int32_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kBlock) {
        const int64_t b = b0 + threadIdx.x;
        const int32_t c = b < nb ? cnt[b * R + r] : 0;
        s[threadIdx.x] = c;
        __syncthreads();
        for (int off = 1; off < kBlock; off <<= 1) {
            const int32_t v = threadIdx.x >= static_cast<unsigned>(off) ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += v;
            __syncthreads();
        }
        if (b < nb) cnt[b * R + r] = carry + s[threadIdx.x] - c;
        carry += s[kBlock - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) tot[r] = carry;
}

// ring_start[r] = sum_{r' < r} tot[r'], r = 0..R.  One block.
__global__ __launch_bounds__(kBlock) void k_part_start(const int32_t *__restrict__ tot, int32_t R,
                                                       int32_t *__restrict__ ring_start) {
    __shared__ int32_t t_s[kMaxRings];
    for (int r = threadIdx.x; r < R; r += kBlock) t_s[r] = tot[r];
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int r = 0; r < R; ++r) {
            ring_start[r] = run;
            run += t_s[r];
        }
        ring_start[R] = run;
    }
}

// Stable ranks: the pixels of ring r get ranks ring_start[r], ring_start[r] + 1, ...
// in ascending pixel index.  Thread r walks the block's keys in order.
__global__ __launch_bounds__(kBlock) void k_part_rank(const int32_t *__restrict__ key, int64_t n_q,
                                                      int32_t R, const int32_t *__restrict__ off,
                                                      const int32_t *__restrict__ ring_start,
                                                      int32_t *__restrict__ rank) {
    __shared__ int32_t k_s[kPartChunk];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kPartChunk;
    for (int i = threadIdx.x; i < kPartChunk; i += kBlock) {
        const int64_t p = base + i;
        k_s[i] = p < n_q ? key[p] : -1;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < R; r += kBlock) {
        int32_t o = ring_start[r] + off[static_cast<int64_t>(blockIdx.x) * R + r];
#pragma unroll 8
        for (int i = 0; i < kPartChunk; ++i)
            if (k_s[i] == r) rank[base + i] = o++;
    }
}

// Per ring r and column k of a ring-ordered row table X[m][k] (row m = rank):
//   pass 1: s = sum over the ring's rows in order; mu = s / n.
// kVariance = false (g2):  out[r * K + k] = mu (NaN for an empty ring), count[r] = n.
// kVariance = true (XSVS): pass 2: v = sum fma(d, d, v), d = X[m][k] - mu;
//   out[k * R + r] = (v / n) / mu^2; if `next`, also the next dyadic level
//   next[m][j] = X[m][2j] + X[m][2j + 1].
// Block (column tile, ring): all threads stage chunks of rows into LDS; lane k
// of the first wave owns column k0 + k and adds the staged rows in order.
template <bool kVariance>
__global__ __launch_bounds__(kBlock) void k_ring_columns(const double *__restrict__ X, int64_t K, int32_t R,
                                                         const int32_t *__restrict__ ring_start,
                                                         double *__restrict__ out, int32_t *__restrict__ count,
                                                         double *__restrict__ next, int64_t K_next) {
    __shared__ double tile[kColChunk];
    const int r = blockIdx.y;
    const int64_t k0 = static_cast<int64_t>(blockIdx.x) * kColTile;
    const int W = static_cast<int>(std::min<int64_t>(kColTile, K - k0));
    const int C = kColChunk / W;  // rows per chunk
    const int32_t a = ring_start[r], b = ring_start[r + 1];
    const int32_t n = b - a;
    // this thread's first staged element is (row q0, column c0); each further
    // load advances the flat index by kBlock = dq rows + dc columns
    const int q0 = threadIdx.x / W, c0 = threadIdx.x - (threadIdx.x / W) * W;
    const int dq = kBlock / W, dc = kBlock - (kBlock / W) * W;
    const bool owner = threadIdx.x < static_cast<unsigned>(W);
    const int lane = threadIdx.x;

    double mu = 0.0, v = 0.0;
    for (int pass = 0; pass < (kVariance ? 2 : 1); ++pass) {
        double s = 0.0;
        for (int32_t m0 = a; m0 < b; m0 += C) {
            const int rows = std::min<int32_t>(C, b - m0);
            double val[kColLoads];
            int qq = q0, cc = c0;
#pragma unroll
            for (int j = 0; j < kColLoads; ++j) {
                val[j] = qq < rows ? X[static_cast<int64_t>(m0 + qq) * K + k0 + cc] : 0.0;
                qq += dq;
                cc += dc;
                if (cc >= W) { cc -= W; ++qq; }
            }
            __syncthreads();  // previous chunk consumed
#pragma unroll
            for (int j = 0; j < kColLoads; ++j) {
                const int i = threadIdx.x + j * kBlock;
                if (i < rows * W) tile[i] = val[j];
            }
            __syncthreads();
            if (owner) {
                if (pass == 0) {
#pragma unroll 16
                    for (int q = 0; q < rows; ++q) s = s + tile[q * W + lane];
                } else {
                    const bool pair = next && !(lane & 1) && k0 + lane + 1 < K;
#pragma unroll 8
                    for (int q = 0; q < rows; ++q) {
                        const double x = tile[q * W + lane];
                        const double d = x - mu;
                        v = __builtin_fma(d, d, v);
                        if (pair)
                            next[static_cast<int64_t>(m0 + q) * K_next + ((k0 + lane) >> 1)] =
                                x + tile[q * W + lane + 1];
                    }
                }
            }
        }
        if (pass == 0) mu = s / static_cast<double>(n);
    }
    if (!owner) return;
    const int64_t k = k0 + lane;
    if (kVariance) {
        out[k * R + r] = n > 0 ? (v / static_cast<double>(n)) / (mu * mu) : __builtin_nan("");
    } else {
        out[static_cast<int64_t>(r) * K + k] = n > 0 ? mu : __builtin_nan("");
        if (count && k == 0) count[r] = n;
    }
}

// ---------------------------------------------------------------- g2

// Per pixel: S = sum_t I_t (sequential), mean = S / F, den = mean^2; pixels
// with den = 0 leave the ring partition (key -1).
__global__ __launch_bounds__(kBlock) void k_pixel_mean(const double *__restrict__ I, int64_t F,
                                                       int64_t n_q, int32_t *__restrict__ key,
                                                       double *__restrict__ den) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (p >= n_q) return;
    double S = 0.0;
#pragma unroll 8
    for (int64_t t = 0; t < F; ++t) S = S + I[t * n_q + p];
    const double mean = S / static_cast<double>(F);
    const double d = mean * mean;
    den[p] = d;
    if (d == 0.0) key[p] = -1;
}

// G[rank[p]][tau] = (sum_{t < F - tau} fma-accumulated I_t I_{t+tau} / (F - tau)) / den_p.
// A block stages `pw` consecutive pixels' series in LDS (lds[t * pw + pp]); a
// thread owns one pixel and kLagBlock consecutive lags, sliding a window of
// the kLagBlock later values along t, so each lag's sum runs t = 0, 1, ... in
// order.
__global__ __launch_bounds__(kBlock) void k_g2_lags(const double *__restrict__ I, int64_t F,
                                                    int64_t n_q, int32_t n_tau, int32_t pw,
                                                    const int32_t *__restrict__ rank,
                                                    const double *__restrict__ den,
                                                    double *__restrict__ G) {
    extern __shared__ double lds[];
    const int64_t p0 = static_cast<int64_t>(blockIdx.x) * pw;
    for (int64_t i = threadIdx.x; i < F * pw; i += kBlock) {
        const int64_t t = i / pw, pp = i - t * pw;
        const int64_t p = p0 + pp;
        lds[i] = p < n_q ? I[t * n_q + p] : 0.0;
    }
    __syncthreads();
    const int pp = threadIdx.x % pw;
    const int slot = threadIdx.x / pw, n_slots = kBlock / pw;
    const int64_t p = p0 + pp;
    if (p >= n_q) return;
    const int32_t row = rank[p];
    if (row < 0) return;
    const double dn = den[p];
    const int n_lb = (n_tau + kLagBlock - 1) / kLagBlock;
    for (int lb = slot; lb < n_lb; lb += n_slots) {
        const int tau0 = lb * kLagBlock;
        double acc[kLagBlock], y[kLagBlock];
#pragma unroll
        for (int j = 0; j < kLagBlock; ++j) {
            acc[j] = 0.0;
            y[j] = tau0 + j < F ? lds[(tau0 + j) * pw + pp] : 0.0;
        }
        for (int64_t t = 0; t + tau0 < F; ++t) {
            const double x = lds[t * pw + pp];
#pragma unroll
            for (int j = 0; j < kLagBlock; ++j)
                if (t + tau0 + j < F) acc[j] = __builtin_fma(x, y[j], acc[j]);
#pragma unroll
            for (int j = 0; j + 1 < kLagBlock; ++j) y[j] = y[j + 1];
            const int64_t nt = t + tau0 + kLagBlock;
            y[kLagBlock - 1] = nt < F ? lds[nt * pw + pp] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < kLagBlock; ++j) {
            const int tau = tau0 + j;
            if (tau < n_tau)
                G[static_cast<int64_t>(row) * n_tau + tau] = (acc[j] / static_cast<double>(F - tau)) / dn;
        }
    }
}

// Same lag step reading global memory (series too long for LDS): one thread
// per (pixel, lag block).
__global__ __launch_bounds__(kBlock) void k_g2_lags_global(const double *__restrict__ I, int64_t F,
                                                           int64_t n_q, int32_t n_tau,
                                                           const int32_t *__restrict__ rank,
                                                           const double *__restrict__ den,
                                                           double *__restrict__ G) {
    const int n_lb = (n_tau + kLagBlock - 1) / kLagBlock;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n_q * n_lb) return;
    const int64_t p = i % n_q;
    const int lb = static_cast<int>(i / n_q);
    const int32_t row = rank[p];
    if (row < 0) return;
    const double dn = den[p];
    const int tau0 = lb * kLagBlock;
    double acc[kLagBlock];
#pragma unroll
    for (int j = 0; j < kLagBlock; ++j) acc[j] = 0.0;
    for (int64_t t = 0; t + tau0 < F; ++t) {
        const double x = I[t * n_q + p];
#pragma unroll
        for (int j = 0; j < kLagBlock; ++j)
            if (t + tau0 + j < F) acc[j] = __builtin_fma(x, I[(t + tau0 + j) * n_q + p], acc[j]);
    }
#pragma unroll
    for (int j = 0; j < kLagBlock; ++j) {
        const int tau = tau0 + j;
        if (tau < n_tau)
            G[static_cast<int64_t>(row) * n_tau + tau] = (acc[j] / static_cast<double>(F - tau)) / dn;
    }
}

// ---------------------------------------------------------------- XSVS

// Jt[rank[p]][t] = I[t][p] for pixels in a ring, through 64 x 64 LDS tiles:
// rows of I are read contiguously and each store writes 64 consecutive frames
// of one pixel.
__global__ __launch_bounds__(kBlock) void k_transpose_rank(const double *__restrict__ I, int64_t F,
                                                           int64_t n_q, const int32_t *__restrict__ rank,
                                                           double *__restrict__ Jt) {
    __shared__ double tile[kTr][kTr + 1];
    const int64_t p0 = static_cast<int64_t>(blockIdx.x) * kTr;
    const int64_t t0 = static_cast<int64_t>(blockIdx.y) * kTr;
    const int lane = threadIdx.x & (kTr - 1), wave = threadIdx.x / kTr;
    for (int r = wave; r < kTr; r += kBlock / kTr) {
        const int64_t t = t0 + r, p = p0 + lane;
        tile[r][lane] = (t < F && p < n_q) ? I[t * n_q + p] : 0.0;
    }
    __syncthreads();
    for (int c = wave; c < kTr; c += kBlock / kTr) {
        const int64_t p = p0 + c;
        if (p >= n_q) break;
        const int32_t row = rank[p];
        if (row >= 0 && t0 + lane < F) Jt[static_cast<int64_t>(row) * F + t0 + lane] = tile[lane][c];
    }
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

// Ring starts and ring-order ranks (-1 for pixels with key -1) from the keys.
xs_status partition(hipStream_t s, const int32_t *key, int64_t n_q, int32_t R, int32_t **start_out,
                    int32_t **rank_out) {
    const int64_t nb = (n_q + kPartChunk - 1) / kPartChunk;
    void *cnt = nullptr, *rk = nullptr;
    XS_TRY(scratch(s, SLOT_RING_CNT, sizeof(int32_t) * (nb * R + 2 * R + 1), &cnt));
    XS_TRY(scratch(s, SLOT_RING_LIST, sizeof(int32_t) * std::max<int64_t>(n_q, 1), &rk));
    int32_t *c = static_cast<int32_t *>(cnt);
    int32_t *tot = c + nb * R;
    int32_t *start = tot + R;
    int32_t *rank = static_cast<int32_t *>(rk);
    if (n_q > 0) {
        hipLaunchKernelGGL(k_fill_i32, dim3(std::min<unsigned>(blocks_for(n_q), 4096u)), dim3(kBlock), 0, s,
                           rank, n_q, -1);
        hipLaunchKernelGGL(k_part_count, dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, key, n_q, R, c);
    }
    hipLaunchKernelGGL(k_part_scan_ring, dim3(static_cast<unsigned>(R)), dim3(kBlock), 0, s, c, nb, R, tot);
    hipLaunchKernelGGL(k_part_start, dim3(1), dim3(kBlock), 0, s, tot, R, start);
    if (n_q > 0)
        hipLaunchKernelGGL(k_part_rank, dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, key, n_q, R, c,
                           start, rank);
    XS_HIP(hipGetLastError());
    *start_out = start;
    *rank_out = rank;
    return XS_OK;
}

dim3 column_grid(int64_t K, int32_t R) {
    return dim3(static_cast<unsigned>((K + kColTile - 1) / kColTile), static_cast<unsigned>(R));
}

}  // namespace

xs_status g2_rings(hipStream_t s, const double *I, int64_t F, int64_t n_q, const double *q,
                   const RingEdges &edges, int32_t n_tau, double *g2_out, int32_t *ring_count) {
    const int32_t R = edges.n_rings;
    void *tok = nullptr;
    timer_begin(s, TIMER_G2, &tok);
    void *key = nullptr, *G = nullptr, *den = nullptr;
    XS_TRY(scratch(s, SLOT_RING_KEY, sizeof(int32_t) * std::max<int64_t>(n_q, 1), &key));
    XS_TRY(scratch(s, SLOT_PIXEL2, sizeof(double) * std::max<int64_t>(n_q, 1), &den));
    XS_TRY(scratch(s, SLOT_G, sizeof(double) * std::max<int64_t>(n_q * n_tau, 1), &G));
    int32_t *k = static_cast<int32_t *>(key);
    double *dn = static_cast<double *>(den);
    if (n_q > 0) {
        hipLaunchKernelGGL(k_ring_key, dim3(blocks_for(n_q)), dim3(kBlock), 0, s, q, n_q, edges, k);
        hipLaunchKernelGGL(k_pixel_mean, dim3(blocks_for(n_q)), dim3(kBlock), 0, s, I, F, n_q, k, dn);
        XS_HIP(hipGetLastError());
    }
    int32_t *start = nullptr, *rank = nullptr;
    XS_TRY(partition(s, k, n_q, R, &start, &rank));
    if (n_q > 0) {
        // pixels per block for the LDS path: largest power of two <= 64 with the
        // series in at most 64 KiB
        int pw = 64;
        while (pw > 1 && F * pw * static_cast<int64_t>(sizeof(double)) > 65536) pw >>= 1;
        if (F * pw * static_cast<int64_t>(sizeof(double)) <= 65536) {
            const size_t lds = sizeof(double) * F * pw;
            hipLaunchKernelGGL(k_g2_lags, dim3(static_cast<unsigned>((n_q + pw - 1) / pw)), dim3(kBlock), lds, s,
                               I, F, n_q, n_tau, pw, rank, dn, static_cast<double *>(G));
        } else {
            const int64_t n_lb = (n_tau + kLagBlock - 1) / kLagBlock;
            hipLaunchKernelGGL(k_g2_lags_global, dim3(blocks_for(n_q * n_lb)), dim3(kBlock), 0, s, I, F, n_q,
                               n_tau, rank, dn, static_cast<double *>(G));
        }
        XS_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_ring_columns<false>, column_grid(n_tau, R), dim3(kBlock), 0, s,
                       static_cast<const double *>(G), static_cast<int64_t>(n_tau), R, start, g2_out, ring_count,
                       nullptr, int64_t(0));
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
    void *key = nullptr, *bwin = nullptr, *j0 = nullptr, *la = nullptr, *lb = nullptr;
    XS_TRY(scratch(s, SLOT_RING_KEY, sizeof(int32_t) * std::max<int64_t>(n_q, 1), &key));
    XS_TRY(scratch(s, SLOT_BWIN, sizeof(double) * F * R, &bwin));
    // row tables in ring order; n_q rows bound the number of pixels in rings
    const int64_t rows = std::max<int64_t>(n_q, 1);
    XS_TRY(scratch(s, SLOT_LEVEL_0, sizeof(double) * rows * F, &j0));
    if (n_levels > 1)
        XS_TRY(scratch(s, SLOT_LEVEL_A, sizeof(double) * rows * std::max<int64_t>(F / 2, 1), &la));
    if (n_levels > 2)
        XS_TRY(scratch(s, SLOT_LEVEL_B, sizeof(double) * rows * std::max<int64_t>(F / 4, 1), &lb));
    int32_t *k = static_cast<int32_t *>(key);
    if (n_q > 0)
        hipLaunchKernelGGL(k_ring_key, dim3(blocks_for(n_q)), dim3(kBlock), 0, s, q, n_q, edges, k);
    int32_t *start = nullptr, *rank = nullptr;
    XS_TRY(partition(s, k, n_q, R, &start, &rank));
    if (n_q > 0) {
        const dim3 gt(static_cast<unsigned>((n_q + kTr - 1) / kTr), static_cast<unsigned>((F + kTr - 1) / kTr));
        hipLaunchKernelGGL(k_transpose_rank, gt, dim3(kBlock), 0, s, I, F, n_q, rank, static_cast<double *>(j0));
    }
    // level l reads J (K windows per row) and, unless it is the last, writes
    // level l + 1 into the other ping-pong buffer
    const double *J = static_cast<const double *>(j0);
    int64_t K = F;
    for (int32_t l = 0; l < n_levels; ++l) {
        const bool more = l + 1 < n_levels;
        double *dst = more ? static_cast<double *>((l & 1) ? lb : la) : nullptr;
        const int64_t Kn = more ? K / 2 : 0;
        hipLaunchKernelGGL(k_ring_columns<true>, column_grid(K, R), dim3(kBlock), 0, s, J, K, R, start,
                           static_cast<double *>(bwin), static_cast<int32_t *>(nullptr), dst, Kn);
        hipLaunchKernelGGL(k_xsvs_mean, dim3(blocks_for(R)), dim3(kBlock), 0, s,
                           static_cast<const double *>(bwin), K, F, R,
                           beta_out + static_cast<int64_t>(l) * R,
                           beta_win ? beta_win + static_cast<int64_t>(l) * F * R : nullptr);
        XS_HIP(hipGetLastError());
        J = dst;
        K = Kn;
    }
    timer_end(s, TIMER_XSVS, tok, static_cast<double>(F) * n_q * sizeof(double));
    return XS_OK;
}

}  // namespace xs
