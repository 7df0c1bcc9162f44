// Reductions of the speckle intensities (Sec. 2.3):
//   g2 on |q| rings, Eq. (g2_def) with the ring mean of Sec. 4.2;
//   XSVS contrast versus exposure, Eqs. (inte_Iq), (bq_Iq).
// Every floating-point sum has a fixed order (time sums sequential in t, ring
// sums sequential in ascending pixel index, window sums pairwise), so results
// are bit-for-bit reproducible.  The sequential ring chains are kept fast by
// the data layout: pixels are renumbered in ring order (ascending index within
// a ring: `rank`, and its inverse `list`), and a block stages a chunk of one
// ring's rows in LDS with all its threads while the owning lanes walk the
// previous chunk in order.  g2 writes its per-pixel lag values as rank-ordered
// rows; XSVS gathers a ring's frames through `list` and forms six exposure
// levels per pass over them.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "xs_internal.h"

namespace xs {
namespace {

constexpr int kBlock = 256;
constexpr int kPartChunk = 1024;  // pixels per partition block
constexpr int kLagBlock = 8;      // lags per thread in the g2 lag kernel
constexpr int kColTile = 64;      // columns (lags / windows) per ring-sum block
constexpr int kColChunk = 4096;   // doubles staged per chunk (32 KiB of LDS)
constexpr int kColLoads = kColChunk / kBlock;
constexpr int kSumBatch = 8;      // LDS reads in flight per ring-sum lane
constexpr int kLvTile = 64;       // XSVS: base windows per block
constexpr int kLvDepth = 6;       // XSVS: levels per launch (base and 5 coarser)
constexpr int kLvRows = 32;       // XSVS: ring rows per staged chunk
constexpr int kLvStride = 2 * kLvTile + 1;  // LDS row: 127 windows of 7 levels, odd stride
constexpr int kLvLoads = kLvRows * kLvTile / kBlock;
static_assert(kLvRows * 8 == kBlock && kLvTile == 64 && (1 << kLvDepth) == kLvTile,
              "XSVS level kernel: thread (row, group of 8 windows) covers one chunk");

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
// in ascending pixel index, and list[rank[p]] = p.  Thread r walks the block's
// keys in order.
__global__ __launch_bounds__(kBlock) void k_part_rank(const int32_t *__restrict__ key, int64_t n_q,
                                                      int32_t R, const int32_t *__restrict__ off,
                                                      const int32_t *__restrict__ ring_start,
                                                      int32_t *__restrict__ rank, int32_t *__restrict__ list) {
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
            if (k_s[i] == r) {
                rank[base + i] = o;
                list[o] = static_cast<int32_t>(base + i);
                ++o;
            }
    }
}

// One chunk of a ring's rows: val[j] = X[m0 + row][k0 + col] for the flat
// index i = tid + j * kBlock = row * W + col, rows < `rows`.  The thread's
// first element is (q0, c0); each step advances by kBlock = dq rows + dc columns.
__device__ inline void stage_rows(double (&val)[kColLoads], const double *__restrict__ X, int64_t K,
                                  int32_t m0, int rows, int64_t k0, int W, int q0, int c0, int dq, int dc) {
    int qq = q0, cc = c0;
#pragma unroll
    for (int j = 0; j < kColLoads; ++j) {
        val[j] = qq < rows ? X[static_cast<int64_t>(m0 + qq) * K + k0 + cc] : 0.0;
        qq += dq;
        cc += dc;
        if (cc >= W) {
            cc -= W;
            ++qq;
        }
    }
}

// Ring mean of each column of a ring-ordered row table X[m][k] (row m = rank):
// out[r * K + k] = (sum over the ring's rows in order) / n (NaN for an empty
// ring), count[r] = n.  Block (column tile of width Wt, ring): all threads
// stage chunks of rows into LDS, loading chunk c + 1 into registers while lanes
// 0..W-1 of the first wave, one per column, add the rows of chunk c in order.
__global__ __launch_bounds__(kBlock) void k_ring_mean(const double *__restrict__ X, int64_t K, int32_t Wt,
                                                      const int32_t *__restrict__ ring_start,
                                                      double *__restrict__ out, int32_t *__restrict__ count) {
    __shared__ double tile[kColChunk];
    const int r = blockIdx.y;
    const int64_t k0 = static_cast<int64_t>(blockIdx.x) * Wt;
    const int W = static_cast<int>(std::min<int64_t>(Wt, K - k0));
    const int C = kColChunk / W;  // rows per chunk
    const int32_t a = ring_start[r], b = ring_start[r + 1];
    const int32_t n = b - a;
    const int q0 = threadIdx.x / W, c0 = threadIdx.x - (threadIdx.x / W) * W;
    const int dq = kBlock / W, dc = kBlock - (kBlock / W) * W;
    const int lane = threadIdx.x;
    const bool owner = lane < W;

    double s = 0.0;
    double val[kColLoads];
    int32_t m0 = a;
    int rows = std::min<int32_t>(C, b - a);
    stage_rows(val, X, K, m0, rows, k0, W, q0, c0, dq, dc);
    while (m0 < b) {
        __syncthreads();  // previous chunk consumed
#pragma unroll
        for (int j = 0; j < kColLoads; ++j) {
            const int i = threadIdx.x + j * kBlock;
            if (i < rows * W) tile[i] = val[j];
        }
        __syncthreads();
        const int32_t m1 = m0 + rows;
        const int rows1 = std::min<int32_t>(C, b - m1);
        if (rows1 > 0) stage_rows(val, X, K, m1, rows1, k0, W, q0, c0, dq, dc);
        if (owner) {
            // LDS reads in batches of kSumBatch issued ahead of the dependent adds
            const double *col = tile + lane;
            int q = 0;
            for (; q + kSumBatch <= rows; q += kSumBatch) {
                double x[kSumBatch];
#pragma unroll
                for (int j = 0; j < kSumBatch; ++j) x[j] = col[(q + j) * W];
#pragma unroll
                for (int j = 0; j < kSumBatch; ++j) s = s + x[j];
            }
            for (; q < rows; ++q) s = s + col[q * W];
        }
        m0 = m1;
        rows = rows1;
    }
    if (!owner) return;
    const int64_t k = k0 + lane;
    out[static_cast<int64_t>(r) * K + k] = n > 0 ? s / static_cast<double>(n) : __builtin_nan("");
    if (count && k == 0) count[r] = n;
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
// A block stages 2^lpw consecutive pixels' series in LDS (lds[t * pw + pp]); a
// thread owns one pixel and kLagBlock consecutive lags, sliding a window of
// the kLagBlock later values along t, so each lag's sum runs t = 0, 1, ... in
// order.  The main loop covers the t where every lag of the block is in range.
__global__ __launch_bounds__(kBlock) void k_g2_lags(const double *__restrict__ I, int32_t F,
                                                    int64_t n_q, int32_t n_tau, int32_t lpw,
                                                    const int32_t *__restrict__ rank,
                                                    const double *__restrict__ den,
                                                    double *__restrict__ G) {
    extern __shared__ double lds[];
    const int pw = 1 << lpw;
    const int64_t p0 = static_cast<int64_t>(blockIdx.x) * pw;
    for (int i = threadIdx.x; i < F * pw; i += kBlock) {
        const int t = i >> lpw, pp = i & (pw - 1);
        const int64_t p = p0 + pp;
        lds[i] = p < n_q ? I[static_cast<int64_t>(t) * n_q + p] : 0.0;
    }
    __syncthreads();
    const int pp = threadIdx.x & (pw - 1);
    const int slot = threadIdx.x >> lpw, n_slots = kBlock >> lpw;
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
        const int t_main = F - tau0 - kLagBlock;  // t < t_main: lags and the next load in range
        int t = 0;
#pragma unroll 8
        for (; t < t_main; ++t) {
            const double x = lds[t * pw + pp];
#pragma unroll
            for (int j = 0; j < kLagBlock; ++j) acc[j] = __builtin_fma(x, y[j], acc[j]);
#pragma unroll
            for (int j = 0; j + 1 < kLagBlock; ++j) y[j] = y[j + 1];
            y[kLagBlock - 1] = lds[(t + tau0 + kLagBlock) * pw + pp];
        }
        for (; t + tau0 < F; ++t) {
            const double x = lds[t * pw + pp];
#pragma unroll
            for (int j = 0; j < kLagBlock; ++j)
                if (t + tau0 + j < F) acc[j] = __builtin_fma(x, y[j], acc[j]);
#pragma unroll
            for (int j = 0; j + 1 < kLagBlock; ++j) y[j] = y[j + 1];
            const int nt = t + tau0 + kLagBlock;
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

// Exposure levels handled by one k_xsvs_levels launch: level base + d for
// d < depths, with bwin[d] = [R][K_d] per-window contrast, K_d = K_base >> d.
struct LevelOut {
    double *bwin[kLvDepth];
    int64_t K[kLvDepth];
};

// Windows of base level L (K per row) and the next kLvDepth - 1 levels, per ring.
// Block (64-window tile k0.., ring r).  A chunk of kLvRows ring rows of the
// tile's 64 base windows is staged in LDS (row stride kLvStride):
//   columns [0, 64)    level L windows,
//   [64, 96) L+1,  [96, 112) L+2,  [112, 120) L+3,  [120, 124) L+4,
//   [124, 126) L+5, [126] L+6,
// the coarser levels formed by pairwise sums J_{l+1}[j] = J_l[2j] + J_l[2j+1].  Thread t < 126 owns column t (one window of one level) and runs its
// two-pass mean / variance over the ring's rows in order: the levels of a tile
// advance together instead of one launch (and one walk of the ring) per level.
// Level L+6 (one window per full tile) is written to `next` [rank][K >> 6] for
// the launch that continues from it.
// kGather: base rows gathered from the frames I[k][list[m]] (ld = pixels);
// otherwise read from a ring-ordered table X[m][k] (ld = K).
template <bool kGather>
__global__ __launch_bounds__(kBlock) void k_xsvs_levels(const double *__restrict__ X, int64_t K, int64_t ld,
                                                        const int32_t *__restrict__ list,
                                                        const int32_t *__restrict__ ring_start, int32_t depths,
                                                        LevelOut lo, double *__restrict__ next) {
    __shared__ double tile[kLvRows * kLvStride];
    const int r = blockIdx.y;
    const int64_t k0 = static_cast<int64_t>(blockIdx.x) * kLvTile;
    const int W = static_cast<int>(std::min<int64_t>(kLvTile, K - k0));
    const int32_t a = ring_start[r], b = ring_start[r + 1];
    const int32_t n = b - a;
    const int t = threadIdx.x;
    // the window this thread owns: level depth d, local index j, column t
    int d = -1, j = 0;
#pragma unroll
    for (int dd = 0; dd < kLvDepth; ++dd) {
        const int o = 2 * kLvTile - ((2 * kLvTile) >> dd), w = kLvTile >> dd;
        if (dd < depths && t >= o && t < o + w) {
            d = dd;
            j = t - o;
        }
    }
    const bool owner = d >= 0 && k0 + (static_cast<int64_t>(j) + 1) * (int64_t(1) << d) <= K;
    const bool want_next = next != nullptr && k0 + kLvTile <= K;
    const int64_t K_next = K >> kLvDepth;

    // staging map: element i of thread t is (row q_t + i * dqi, column c_t + i * dci)
    //   table:  lanes along a row (64 windows), 4 rows per step
    //   gather: lanes along the ring (kLvRows rows), 8 windows per step; the
    //           thread's row, hence its pixel list[m0 + q_t], is fixed
    const int q_t = kGather ? (t & (kLvRows - 1)) : (t / kLvTile);
    const int c_t = kGather ? (t / kLvRows) : (t & (kLvTile - 1));
    constexpr int dqi = kGather ? 0 : kBlock / kLvTile;
    constexpr int dci = kGather ? kBlock / kLvRows : 0;
    auto load_chunk = [&](double (&val)[kLvLoads], int32_t m0, int rows) {
        if (kGather) {
            const bool ok = q_t < rows;
            const int64_t p = ok ? list[m0 + q_t] : 0;
#pragma unroll
            for (int i = 0; i < kLvLoads; ++i) {
                const int c = c_t + i * dci;
                val[i] = ok && c < W ? X[(k0 + c) * ld + p] : 0.0;
            }
        } else {
#pragma unroll
            for (int i = 0; i < kLvLoads; ++i) {
                const int q = q_t + i * dqi;
                val[i] = q < rows && c_t < W ? X[static_cast<int64_t>(m0 + q) * ld + k0 + c_t] : 0.0;
            }
        }
    };

    double mu = 0.0, v = 0.0;
#pragma unroll 1
    for (int pass = 0; pass < 2; ++pass) {
        double s = 0.0;
        // the next chunk is loaded into registers while the current one is summed
        double buf[kLvLoads];
        int32_t mc = a, rc = std::min<int32_t>(kLvRows, b - a);
        load_chunk(buf, mc, rc);
        int32_t m = a + rc;
        while (rc > 0) {
            const int32_t mrow = mc;
            const int rows = rc;
            __syncthreads();  // previous chunk consumed
#pragma unroll
            for (int i = 0; i < kLvLoads; ++i) tile[(q_t + i * dqi) * kLvStride + c_t + i * dci] = buf[i];
            __syncthreads();
            // coarser levels of the chunk: thread (row q, group g of 8 level-L windows)
            // forms levels L+1..L+3 of its group; the 8 lanes of a row (one wave)
            // then pair up their level-L+3 sums for L+4..L+6 by lane exchange
            {
                const int q = t >> 3, g = t & 7;
                double *row = tile + q * kLvStride;
                double x[8], y1[4], y2[2];
#pragma unroll
                for (int i = 0; i < 8; ++i) x[i] = row[8 * g + i];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    y1[i] = x[2 * i] + x[2 * i + 1];
                    row[64 + 4 * g + i] = y1[i];
                }
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    y2[i] = y1[2 * i] + y1[2 * i + 1];
                    row[96 + 2 * g + i] = y2[i];
                }
                const double y3 = y2[0] + y2[1];
                row[112 + g] = y3;
                const double y4 = y3 + __shfl_xor(y3, 1);  // lanes g = 0, 2, 4, 6
                if (!(g & 1)) row[120 + (g >> 1)] = y4;
                const double y5 = y4 + __shfl_xor(y4, 2);  // lanes g = 0, 4
                if (!(g & 3)) row[124 + (g >> 2)] = y5;
                const double y6 = y5 + __shfl_xor(y5, 4);  // lane g = 0
                if (g == 0) {
                    row[126] = y6;
                    if (pass == 0 && want_next && q < rows)
                        next[static_cast<int64_t>(mrow + q) * K_next + (k0 >> kLvDepth)] = y6;
                }
            }
            __syncthreads();
            mc = m;
            rc = std::min<int32_t>(kLvRows, b - m);
            if (rc > 0) load_chunk(buf, mc, rc);
            m += rc;
            if (owner) {
                const double *col = tile + t;
                int q = 0;
                if (pass == 0) {
                    for (; q + kSumBatch <= rows; q += kSumBatch) {
                        double x[kSumBatch];
#pragma unroll
                        for (int i = 0; i < kSumBatch; ++i) x[i] = col[(q + i) * kLvStride];
#pragma unroll
                        for (int i = 0; i < kSumBatch; ++i) s = s + x[i];
                    }
                    for (; q < rows; ++q) s = s + col[q * kLvStride];
                } else {
                    for (; q + kSumBatch <= rows; q += kSumBatch) {
                        double x[kSumBatch];
#pragma unroll
                        for (int i = 0; i < kSumBatch; ++i) x[i] = col[(q + i) * kLvStride];
#pragma unroll
                        for (int i = 0; i < kSumBatch; ++i) {
                            const double e = x[i] - mu;
                            v = __builtin_fma(e, e, v);
                        }
                    }
                    for (; q < rows; ++q) {
                        const double e = col[q * kLvStride] - mu;
                        v = __builtin_fma(e, e, v);
                    }
                }
            }
        }
        if (pass == 0) mu = s / static_cast<double>(n);
    }
    if (!owner) return;
    const int64_t Kd = lo.K[d];
    const int64_t k = (k0 >> d) + j;
    lo.bwin[d][static_cast<int64_t>(r) * Kd + k] =
        n > 0 ? (v / static_cast<double>(n)) / (mu * mu) : __builtin_nan("");
}


// Mean over windows, block per ring r: beta_out[r] = (sum_k bwin[r][k] in order) / K;
// optional per-window output beta_win_level[k][r] (rows k >= K filled with NaN).
__global__ __launch_bounds__(kBlock) void k_xsvs_mean(const double *__restrict__ bwin, int64_t K,
                                                      int64_t F, int32_t R,
                                                      double *__restrict__ beta_out,
                                                      double *__restrict__ beta_win_level) {
    __shared__ double buf[kBlock];
    const int r = blockIdx.x;
    const double *row = bwin + static_cast<int64_t>(r) * K;
    double acc = 0.0;
    for (int64_t k0 = 0; k0 < K; k0 += kBlock) {
        const int64_t k = k0 + threadIdx.x;
        const double x = k < K ? row[k] : 0.0;
        if (beta_win_level && k < K) beta_win_level[k * R + r] = x;
        __syncthreads();
        buf[threadIdx.x] = x;
        __syncthreads();
        if (threadIdx.x == 0) {
            const int nk = static_cast<int>(std::min<int64_t>(kBlock, K - k0));
            for (int i = 0; i < nk; ++i) acc = acc + buf[i];
        }
    }
    if (beta_win_level)
        for (int64_t k = K + threadIdx.x; k < F; k += kBlock) beta_win_level[k * R + r] = __builtin_nan("");
    if (threadIdx.x == 0) beta_out[r] = acc / static_cast<double>(K);
}

// Ring starts and ring-order ranks (-1 for pixels with key -1) from the keys.
xs_status partition(hipStream_t s, const int32_t *key, int64_t n_q, int32_t R, int32_t **start_out,
                    int32_t **rank_out, int32_t **list_out) {
    const int64_t nb = (n_q + kPartChunk - 1) / kPartChunk;
    void *cnt = nullptr, *rk = nullptr;
    XS_TRY(scratch(s, SLOT_RING_CNT, sizeof(int32_t) * (nb * R + 2 * R + 1), &cnt));
    XS_TRY(scratch(s, SLOT_RING_LIST, sizeof(int32_t) * 2 * std::max<int64_t>(n_q, 1), &rk));
    int32_t *c = static_cast<int32_t *>(cnt);
    int32_t *tot = c + nb * R;
    int32_t *start = tot + R;
    int32_t *rank = static_cast<int32_t *>(rk);
    int32_t *list = rank + std::max<int64_t>(n_q, 1);
    if (n_q > 0) {
        hipLaunchKernelGGL(k_fill_i32, dim3(std::min<unsigned>(blocks_for(n_q), 4096u)), dim3(kBlock), 0, s,
                           rank, n_q, -1);
        hipLaunchKernelGGL(k_part_count, dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, key, n_q, R, c);
    }
    hipLaunchKernelGGL(k_part_scan_ring, dim3(static_cast<unsigned>(R)), dim3(kBlock), 0, s, c, nb, R, tot);
    hipLaunchKernelGGL(k_part_start, dim3(1), dim3(kBlock), 0, s, tot, R, start);
    if (n_q > 0)
        hipLaunchKernelGGL(k_part_rank, dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, key, n_q, R, c,
                           start, rank, list);
    XS_HIP(hipGetLastError());
    *start_out = start;
    *rank_out = rank;
    *list_out = list;
    return XS_OK;
}

// Column tile width for k_ring_columns: 64, halved while the grid stays within
// the blocks the device holds at once, so short tables still spread their
// (long, sequential) ring chains over the whole chip.
int column_tile(const void *kernel, int64_t K, int32_t R, int min_width) {
    const int64_t slots = resident_blocks(kernel, kBlock);
    auto blocks = [&](int w) { return static_cast<int64_t>(R) * ((K + w - 1) / w); };
    int W = kColTile;
    while (W / 2 >= min_width && blocks(W) < slots && blocks(W / 2) <= slots) W /= 2;
    return W;
}

dim3 column_grid(int64_t K, int32_t R, int W) {
    return dim3(static_cast<unsigned>((K + W - 1) / W), static_cast<unsigned>(R));
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
    int32_t *start = nullptr, *rank = nullptr, *list = nullptr;
    XS_TRY(partition(s, k, n_q, R, &start, &rank, &list));
    if (n_q > 0) {
        // pixels per block for the LDS path: largest power of two <= 64 with the
        // series in at most 64 KiB
        int lpw = 6;
        while (lpw > 0 && (F << lpw) * static_cast<int64_t>(sizeof(double)) > 65536) --lpw;
        if ((F << lpw) * static_cast<int64_t>(sizeof(double)) <= 65536) {
            const size_t lds = sizeof(double) * (F << lpw);
            const int64_t pw = int64_t(1) << lpw;
            hipLaunchKernelGGL(k_g2_lags, dim3(static_cast<unsigned>((n_q + pw - 1) / pw)), dim3(kBlock), lds, s,
                               I, static_cast<int32_t>(F), n_q, n_tau, static_cast<int32_t>(lpw), rank, dn,
                               static_cast<double *>(G));
        } else {
            const int64_t n_lb = (n_tau + kLagBlock - 1) / kLagBlock;
            hipLaunchKernelGGL(k_g2_lags_global, dim3(blocks_for(n_q * n_lb)), dim3(kBlock), 0, s, I, F, n_q,
                               n_tau, rank, dn, static_cast<double *>(G));
        }
        XS_HIP(hipGetLastError());
    }
    const int W = column_tile(reinterpret_cast<const void *>(k_ring_mean), n_tau, R, 1);
    hipLaunchKernelGGL(k_ring_mean, column_grid(n_tau, R, W), dim3(kBlock), 0, s,
                       static_cast<const double *>(G), static_cast<int64_t>(n_tau), W, start, g2_out,
                       ring_count);
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
    void *key = nullptr, *bwin = nullptr;
    XS_TRY(scratch(s, SLOT_RING_KEY, sizeof(int32_t) * std::max<int64_t>(n_q, 1), &key));
    // per-window contrast of level l: R x (F >> l) at offset off[l]
    int64_t off[64], total = 0;
    for (int32_t l = 0; l < n_levels; ++l) {
        off[l] = total;
        total += static_cast<int64_t>(R) * (F >> l);
    }
    XS_TRY(scratch(s, SLOT_BWIN, sizeof(double) * std::max<int64_t>(total, 1), &bwin));
    double *bw = static_cast<double *>(bwin);
    int32_t *k = static_cast<int32_t *>(key);
    if (n_q > 0)
        hipLaunchKernelGGL(k_ring_key, dim3(blocks_for(n_q)), dim3(kBlock), 0, s, q, n_q, edges, k);
    int32_t *start = nullptr, *rank = nullptr, *list = nullptr;
    XS_TRY(partition(s, k, n_q, R, &start, &rank, &list));
    const int64_t rows = std::max<int64_t>(n_q, 1);  // bounds the pixels in rings
    const double *src = nullptr;
    // launches of kLvDepth levels each; a launch that does not reach the last
    // level writes the level after its own into a ring-ordered table
    int64_t K = F;
    int pong = 0;
    for (int32_t L = 0; L < n_levels; L += kLvDepth) {
        const int32_t depths = std::min<int32_t>(kLvDepth, n_levels - L);
        double *dst = nullptr;
        if (L + kLvDepth < n_levels) {
            void *nx = nullptr;
            XS_TRY(scratch(s, pong ? SLOT_LEVEL_B : SLOT_LEVEL_A,
                           sizeof(double) * rows * std::max<int64_t>(K >> kLvDepth, 1), &nx));
            dst = static_cast<double *>(nx);
            pong ^= 1;
        }
        LevelOut lo{};
        for (int32_t d = 0; d < depths; ++d) {
            lo.bwin[d] = bw + off[L + d];
            lo.K[d] = K >> d;
        }
        const dim3 grid(static_cast<unsigned>((K + kLvTile - 1) / kLvTile), static_cast<unsigned>(R));
        if (L == 0)
            hipLaunchKernelGGL(k_xsvs_levels<true>, grid, dim3(kBlock), 0, s, I, K, n_q,
                               static_cast<const int32_t *>(list), start, depths, lo, dst);
        else
            hipLaunchKernelGGL(k_xsvs_levels<false>, grid, dim3(kBlock), 0, s, src, K, K,
                               static_cast<const int32_t *>(nullptr), start, depths, lo, dst);
        for (int32_t d = 0; d < depths; ++d)
            hipLaunchKernelGGL(k_xsvs_mean, dim3(static_cast<unsigned>(R)), dim3(kBlock), 0, s,
                               static_cast<const double *>(lo.bwin[d]), K >> d, F, R,
                               beta_out + static_cast<int64_t>(L + d) * R,
                               beta_win ? beta_win + static_cast<int64_t>(L + d) * F * R : nullptr);
        XS_HIP(hipGetLastError());
        src = dst;
        K >>= kLvDepth;
    }
    timer_end(s, TIMER_XSVS, tok, static_cast<double>(F) * n_q * sizeof(double));
    return XS_OK;
}

}  // namespace xs
