// Reductions of the speckle intensities (Sec. 2.3):
//   g2 on |q| rings, Eq. (g2_def) with the ring mean of Sec. 4.2;
//   XSVS contrast versus exposure, Eqs. (inte_Iq), (bq_Iq).
// Every floating-point sum has a fixed order, so results are bit-for-bit
// reproducible: time sums sequential in t, window sums pairwise (dyadic), the
// mean over windows sequential in k, and ring sums pairwise over the ring's
// pixels in ascending index — adjacent pairs added level by level, an odd last
// element carried up unchanged.  That ring tree is computed in parallel:
// aligned groups of 32 consecutive elements form exact subtrees (a partial
// last group is the fold from the right of the complete subtrees of its binary
// decomposition), and the group values are reduced the same way, level after
// level, until one value per ring is left.  Pixels are renumbered in ring
// order (`rank`, inverse `list`) so each level reads contiguous rows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "xs_internal.h"

namespace xs {
namespace {

constexpr int kBlock = 256;
constexpr int kPartChunk = 1024;  // pixels per partition block
constexpr int kLagBlock = 8;      // lags per thread in the g2 lag kernel
constexpr int kGroup = 32;        // elements per pairwise-tree group
constexpr int kLvTile = 64;       // XSVS: base windows per block
constexpr int kLvDepth = 6;       // XSVS: levels per launch (base and 5 coarser)
constexpr int kLvRows = kGroup;   // XSVS: ring rows per staged chunk (one tree group)
constexpr int kLvStride = 2 * kLvTile + 1;  // LDS row: 127 windows of 7 levels, odd stride
constexpr int kLvHalf = 2 * kLvTile;        // windows per tile over its 7 levels (126 used)
constexpr int kLvCols = 2 * kLvHalf;        // chunk-sum columns per tile: sums of J, then of J^2
constexpr int kLvLoads = kLvRows * kLvTile / kBlock;
constexpr int kLvChunksPerBlock = 4;        // consecutive chunks of one ring per block
static_assert(kLvRows * 8 == kBlock && kLvTile == 64 && (1 << kLvDepth) == kLvTile,
              "XSVS level kernel: thread (row, group of 8 windows) covers one chunk");
static_assert(kLvChunksPerBlock == 4, "XSVS level kernel: a block adds its chunk trees as two pairs");

unsigned blocks_for(int64_t n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }

// ---------------------------------------------------------------- pairwise tree

// Complete tree over 2^K values v(st), v(st + 1), ...  Above 16 values the
// two halves are summed one after the other (the same tree, half the registers).
template <int K, typename Load>
__device__ __forceinline__ double complete_tree(int st, const Load &v) {
    if constexpr (K > 4) {
        const double lo = complete_tree<K - 1>(st, v);
        return lo + complete_tree<K - 1>(st + (1 << (K - 1)), v);
    }
    double x[1 << K];
#pragma unroll
    for (int i = 0; i < (1 << K); ++i) x[i] = v(st + i);
#pragma unroll
    for (int w = (1 << K) / 2; w >= 1; w >>= 1)
#pragma unroll
        for (int i = 0; i < w; ++i) x[i] = x[2 * i] + x[2 * i + 1];
    return x[0];
}

// Pairwise tree of v(0) .. v(n - 1), 1 <= n <= 32: the complete subtrees of the
// binary decomposition of n, left to right by decreasing size, folded from the
// right (the bottom-up tree with the odd element carried up).
template <typename Load>
__device__ __forceinline__ double tree_upto32(int n, const Load &v) {
    double s = 0.0;
    int end = n;
    bool have = false;
    auto part = [&](double t, int size) {
        s = have ? t + s : t;
        have = true;
        end -= size;
    };
    if (n & 1) part(complete_tree<0>(end - 1, v), 1);
    if (n & 2) part(complete_tree<1>(end - 2, v), 2);
    if (n & 4) part(complete_tree<2>(end - 4, v), 4);
    if (n & 8) part(complete_tree<3>(end - 8, v), 8);
    if (n & 16) part(complete_tree<4>(end - 16, v), 16);
    if (n & 32) part(complete_tree<5>(end - 32, v), 32);
    return s;
}

// Complete trees over 2^K values x = v(st + i) and over their rounded squares x * x.
template <int K, typename Load>
__device__ __forceinline__ void complete_tree2(int st, const Load &v, double &s1, double &s2) {
    if constexpr (K > 4) {
        double a1, a2, b1, b2;
        complete_tree2<K - 1>(st, v, a1, a2);
        complete_tree2<K - 1>(st + (1 << (K - 1)), v, b1, b2);
        s1 = a1 + b1;
        s2 = a2 + b2;
    } else {
        double x[1 << K], y[1 << K];
#pragma unroll
        for (int i = 0; i < (1 << K); ++i) {
            x[i] = v(st + i);
            y[i] = x[i] * x[i];
        }
#pragma unroll
        for (int w = (1 << K) / 2; w >= 1; w >>= 1)
#pragma unroll
            for (int i = 0; i < w; ++i) {
                x[i] = x[2 * i] + x[2 * i + 1];
                y[i] = y[2 * i] + y[2 * i + 1];
            }
        s1 = x[0];
        s2 = y[0];
    }
}

// tree_upto32 of the values and of their rounded squares, in one read.
template <typename Load>
__device__ __forceinline__ void tree2_upto32(int n, const Load &v, double &s1, double &s2) {
    int end = n;
    bool have = false;
    auto part = [&](double t1, double t2, int size) {
        s1 = have ? t1 + s1 : t1;
        s2 = have ? t2 + s2 : t2;
        have = true;
        end -= size;
    };
    double t1, t2;
    s1 = s2 = 0.0;
    if (n & 1) { complete_tree2<0>(end - 1, v, t1, t2); part(t1, t2, 1); }
    if (n & 2) { complete_tree2<1>(end - 2, v, t1, t2); part(t1, t2, 2); }
    if (n & 4) { complete_tree2<2>(end - 4, v, t1, t2); part(t1, t2, 4); }
    if (n & 8) { complete_tree2<3>(end - 8, v, t1, t2); part(t1, t2, 8); }
    if (n & 16) { complete_tree2<4>(end - 16, v, t1, t2); part(t1, t2, 16); }
    if (n & 32) { complete_tree2<5>(end - 32, v, t1, t2); part(t1, t2, 32); }
}

// Ring of element e from the offsets off[0..R] (off non-decreasing, e < off[R]).
__device__ __forceinline__ int ring_of(const int32_t *off, int R, int64_t e) {
    int lo = 0, hi = R;  // off[lo] <= e < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

// G tree levels at once (G = 2^k <= 32): out[e][c] = tree over in's elements
// [s, s + cnt) of the element's ring, s = in_off[r] + (e - out_off[r]) * G.
// Rows of ncol columns.
template <int G>
__global__ __launch_bounds__(kBlock) void k_group_tree(const double *__restrict__ in,
                                                       double *__restrict__ out, int64_t ncol,
                                                       const int32_t *__restrict__ in_off,
                                                       const int32_t *__restrict__ out_off, int32_t R) {
    __shared__ int32_t o_s[kMaxRings + 1], i_s[kMaxRings + 1];
    for (int r = threadIdx.x; r <= R; r += kBlock) {
        o_s[r] = out_off[r];
        i_s[r] = in_off[r];
    }
    __syncthreads();
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t e = gid / ncol, c = gid - (gid / ncol) * ncol;
    if (e >= o_s[R]) return;
    const int r = ring_of(o_s, R, e);
    const int64_t s = i_s[r] + (e - o_s[r]) * G;
    const int cnt = static_cast<int>(std::min<int64_t>(G, i_s[r + 1] - s));
    out[e * ncol + c] = tree_upto32(cnt, [&](int i) { return in[(s + i) * ncol + c]; });
}

// ---------------------------------------------------------------- partition

// Ring of pixel p: r with e_r <= |q| < e_{r+1}, |q| = sqrt(fma(qz,qz,fma(qy,qy,qx*qx))),
// else -1.
__device__ __forceinline__ int32_t ring_index(const double *__restrict__ q, int64_t p, const RingEdges &edges) {
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
    return r;
}

__global__ __launch_bounds__(kBlock) void k_ring_key(const double *__restrict__ q, int64_t n_q,
                                                     RingEdges edges, int32_t *__restrict__ key) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (p >= n_q) return;
    key[p] = ring_index(q, p, edges);
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

// Offsets of the ring tree, one block (counts in LDS, one thread per ring for
// the per-ring counts, thread 0 for the running sums):
//   lev[l][r], l = 0..levels, r = 0..R: first element of ring r at tree level l
//   (level 0: the ring's pixels, the ring starts; level l + 1 has ceil(n / 32)
//   of level l's n elements per ring);
//   grp[r], r = 0..R: first block group (chunk_groups level-1 chunks) of ring r.
__global__ __launch_bounds__(kBlock) void k_tree_offsets(const int32_t *__restrict__ tot, int32_t R,
                                                         int32_t levels, int32_t chunk_groups,
                                                         int32_t *__restrict__ lev, int32_t *__restrict__ grp) {
    __shared__ int32_t n_s[kMaxRings], c1_s[kMaxRings], o_s[kMaxRings + 1];
    for (int r = threadIdx.x; r < R; r += kBlock) n_s[r] = tot[r];
    // step l <= levels: tree level l; step levels + 1: block groups of level 1
    for (int l = 0; l <= levels + 1; ++l) {
        __syncthreads();
        if (l > 0)
            for (int r = threadIdx.x; r < R; r += kBlock) {
                if (l <= levels) {
                    n_s[r] = (n_s[r] + kGroup - 1) / kGroup;
                    if (l == 1) c1_s[r] = n_s[r];
                } else {
                    n_s[r] = (c1_s[r] + chunk_groups - 1) / chunk_groups;
                }
            }
        __syncthreads();
        if (threadIdx.x == 0) {
            int32_t acc = 0;
            for (int r = 0; r < R; ++r) {
                o_s[r] = acc;
                acc += n_s[r];
            }
            o_s[R] = acc;
        }
        __syncthreads();
        int32_t *dst = l <= levels ? lev + static_cast<int64_t>(l) * (R + 1) : grp;
        for (int r = threadIdx.x; r <= R; r += kBlock) dst[r] = o_s[r];
    }
}

// Stable ranks: the pixels of ring r get ranks ring_start[r], ring_start[r] + 1, ...
// in ascending pixel index, and list[rank[p]] = p; a pixel of key -1 gets rank -1.
// Wave w of the block takes pixels [256 w, 256 w + 256) of the block's 1024 in four
// steps of 64: lanes of one key are found with a ballot per distinct key, ranked by
// their position in the ballot, and the wave's per-ring running counts kept in LDS;
// the counts of the earlier waves then give each wave's starting offsets.
__global__ __launch_bounds__(kBlock) void k_part_rank(const int32_t *__restrict__ key, int64_t n_q,
                                                      int32_t R, const int32_t *__restrict__ off,
                                                      const int32_t *__restrict__ ring_start,
                                                      int32_t *__restrict__ rank, int32_t *__restrict__ list) {
    constexpr int kWaves = kBlock / 64, kSteps = kPartChunk / kBlock;
    __shared__ int32_t run[kWaves][kMaxRings];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int r = lane; r < R; r += 64) run[wave][r] = 0;
    __syncthreads();
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kPartChunk + static_cast<int64_t>(wave) * (64 * kSteps);
    int32_t k[kSteps], within[kSteps];
    for (int st = 0; st < kSteps; ++st) {
        const int64_t p = base + st * 64 + lane;
        k[st] = p < n_q ? key[p] : -1;
        within[st] = 0;
        uint64_t todo = __ballot(k[st] >= 0);
        while (todo) {
            const int leader = __builtin_ctzll(todo);
            const int kk = __shfl(k[st], leader);
            const uint64_t same = __ballot(k[st] == kk);
            if (k[st] == kk)
                within[st] = run[wave][kk] + __builtin_popcountll(same & ((uint64_t(1) << lane) - 1));
            __builtin_amdgcn_wave_barrier();
            if (lane == leader) run[wave][kk] += __builtin_popcountll(same);
            __builtin_amdgcn_wave_barrier();
            todo &= ~same;
        }
    }
    __syncthreads();
    for (int st = 0; st < kSteps; ++st) {
        const int64_t p = base + st * 64 + lane;
        if (k[st] < 0) {
            if (p < n_q) rank[p] = -1;  // outside every ring
            continue;
        }
        int32_t o = ring_start[k[st]] + off[static_cast<int64_t>(blockIdx.x) * R + k[st]] + within[st];
        for (int w = 0; w < wave; ++w) o += run[w][k[st]];
        rank[p] = o;
        list[o] = static_cast<int32_t>(p);
    }
}

// ---------------------------------------------------------------- g2

// Stage the time series of pixels p0 .. p0 + 2^lpw - 1 in LDS:
// lds[t * 2^lpw + pp] = src[t * n_q + p0 + pp] (zero past n_q).  Each thread
// issues U loads before it writes, so a block waits for ceil(F 2^lpw / (256 U))
// memory round trips rather than one per element.
template <int U, typename T, int NT = kBlock>
__device__ __forceinline__ void stage_series(T *lds, const T *__restrict__ src, int F, int lpw, int64_t n_q,
                                             int64_t p0) {
    const int n = F << lpw, pmask = (1 << lpw) - 1;
    for (int base = 0; base < n; base += NT * U) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = base + u * NT + static_cast<int>(threadIdx.x);
            const int t = i >> lpw;
            const int64_t p = p0 + (i & pmask);
            v[u] = (i < n && p < n_q) ? src[static_cast<int64_t>(t) * n_q + p] : T{};
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = base + u * NT + static_cast<int>(threadIdx.x);
            if (i < n) lds[i] = v[u];
        }
    }
}

// Per pixel: S = sum_t I_t (sequential), mean = S / F, den = mean^2, and the
// pixel's ring key (-1 outside the rings or for den = 0: such a pixel leaves the
// ring partition).
__global__ __launch_bounds__(kBlock) void k_pixel_mean(const double *__restrict__ I, int64_t F,
                                                       int64_t n_q, const double *__restrict__ q,
                                                       RingEdges edges, int32_t *__restrict__ key,
                                                       double *__restrict__ den) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (p >= n_q) return;
    double S = 0.0;
#pragma unroll 8
    for (int64_t t = 0; t < F; ++t) S = S + I[t * n_q + p];
    const double mean = S / static_cast<double>(F);
    const double d = mean * mean;
    den[p] = d;
    key[p] = d == 0.0 ? -1 : ring_index(q, p, edges);
}

// G[rank[p]][tau] = (sum_{t < F - tau} fma-accumulated I_t I_{t+tau} / (F - tau)) / den_p.
// A block stages 2^lpw consecutive pixels' series in LDS (lds[t * pw + pp]); a
// thread owns one pixel and kLagBlock consecutive lags, sliding a window of
// the kLagBlock later values along t, so each lag's sum runs t = 0, 1, ... in
// order.  The main loop covers the t where every lag of the block is in range.
// Lag products of the staged series: thread (pixel pp, slot) owns lag blocks of L
// consecutive lags, lb = slot, slot + n_slots, ...; for lag block tau0 it keeps a window
// y[j] = x[t + tau0 + j] in registers that slides by one element per step, so each
// step reads two values from LDS (x[t] and the window's new end) for L fused
// multiply-adds.  The series is followed by L rows of zeros in LDS, so every lag of the
// block runs the F - tau0 steps of its smallest lag: the extra terms are x[t] * 0, which
// leave a finite sum unchanged bit for bit, and every G_p(tau) stays the sequential sum
// over t of x[t] x[t + tau].  L is chosen per call so that the lag blocks spread evenly
// over the slots.
template <int L>
__global__ __launch_bounds__(kBlock) void k_g2_lags(const double *__restrict__ I, int32_t F,
                                                    int64_t n_q, int32_t n_tau, int32_t lpw,
                                                    const int32_t *__restrict__ rank,
                                                    const double *__restrict__ den,
                                                    double *__restrict__ G) {
    extern __shared__ double lds[];
    const int pw = 1 << lpw;
    const int64_t p0 = static_cast<int64_t>(blockIdx.x) * pw;
    stage_series<16>(lds, I, F, lpw, n_q, p0);
    for (int i = (F << lpw) + static_cast<int>(threadIdx.x); i < ((F + L) << lpw); i += kBlock) lds[i] = 0.0;
    __syncthreads();
    const int pp = threadIdx.x & (pw - 1);
    const int slot = threadIdx.x >> lpw, n_slots = kBlock >> lpw;
    const int64_t p = p0 + pp;
    if (p >= n_q) return;
    const int32_t row = rank[p];
    if (row < 0) return;
    const double dn = den[p];
    const int n_lb = (n_tau + L - 1) / L;
    for (int lb = slot; lb < n_lb; lb += n_slots) {
        const int tau0 = lb * L;
        double acc[L], y[L];
#pragma unroll
        for (int j = 0; j < L; ++j) {
            acc[j] = 0.0;
            y[j] = lds[(tau0 + j) * pw + pp];  // tau0 + j < F + L: staged or zero
        }
        const int steps = F - tau0;
#pragma unroll 8
        for (int t = 0; t < steps; ++t) {
            const double x = lds[t * pw + pp];
#pragma unroll
            for (int j = 0; j < L; ++j) acc[j] = __builtin_fma(x, y[j], acc[j]);
#pragma unroll
            for (int j = 0; j + 1 < L; ++j) y[j] = y[j + 1];
            y[L - 1] = lds[(t + tau0 + L) * pw + pp];  // row < F + L
        }
#pragma unroll
        for (int j = 0; j < L; ++j) {
            const int tau = tau0 + j;
            if (tau < n_tau)
                G[static_cast<int64_t>(row) * n_tau + tau] = (acc[j] / static_cast<double>(F - tau)) / dn;
        }
    }
}

// The same sums with the block's pixel count 2^LPW fixed at compile time and the step
// loop unrolled by L: the window lives in a ring of L registers, y[(t + j) mod L] =
// x[t + tau0 + j], whose oldest slot takes the next value after each step, so no value
// moves between registers, and while every row read lies inside the series each LDS
// address is a constant offset from two per-thread bases.  The last steps (rounded up to
// a multiple of L) read rows clamped to one zero row after the series, so the extra
// steps, as above, add x * 0 to every sum; the series plus that row, (F + 1) 2^LPW
// doubles, is all the LDS a block takes.  Lag block lb runs F - lb L steps, so the
// wavefronts holding the first blocks work longest; the slots rotate by a quarter per
// block (blockIdx.x mod 4), so that the long blocks of neighbouring workgroups land on
// different wavefronts.
template <int L, int LPW, int NT>
__global__ __launch_bounds__(NT) void k_g2_lags_ring(const double *__restrict__ I, int32_t F, int64_t n_q,
                                                     int32_t n_tau, const int32_t *__restrict__ rank,
                                                     const double *__restrict__ den, double *__restrict__ G) {
    constexpr int PW = 1 << LPW, kSlots = NT >> LPW;
    extern __shared__ double lds[];
    const int64_t p0 = static_cast<int64_t>(blockIdx.x) * PW;
    stage_series<16, double, NT>(lds, I, F, LPW, n_q, p0);
    if (static_cast<int>(threadIdx.x) < PW) lds[(F << LPW) + threadIdx.x] = 0.0;
    __syncthreads();
    const int pp = threadIdx.x & (PW - 1);
    const int slot = ((threadIdx.x >> LPW) + (blockIdx.x & 3) * (kSlots / 4)) & (kSlots - 1);
    const int64_t p = p0 + pp;
    if (p >= n_q) return;
    const int32_t row = rank[p];
    if (row < 0) return;
    const double dn = den[p];
    const double *col = lds + pp;  // x[t] at col[t * PW], t <= F (row F is zero)
    const int n_lb = (n_tau + L - 1) / L;
    for (int lb = slot; lb < n_lb; lb += kSlots) {
        const int tau0 = lb * L;
        const double *ys = col + tau0 * PW;  // x[tau0 + i] at ys[i * PW]
        double acc[L], y[L];
#pragma unroll
        for (int j = 0; j < L; ++j) {
            acc[j] = 0.0;
            y[j] = col[min(tau0 + j, F) * PW];
        }
        const int steps = F - tau0;
        int t = 0;
        // rows t + s and t + s + tau0 + L stay below F
        for (; t + 2 * L <= steps; t += L) {
            const double *xt = col + t * PW, *yt = ys + (t + L) * PW;
#pragma unroll
            for (int s = 0; s < L; ++s) {
                const double x = xt[s * PW];
#pragma unroll
                for (int j = 0; j < L; ++j) acc[j] = __builtin_fma(x, y[(s + j) % L], acc[j]);
                y[s] = yt[s * PW];
            }
        }
        for (; t < steps; t += L) {
#pragma unroll
            for (int s = 0; s < L; ++s) {
                const double x = col[min(t + s, F) * PW];
#pragma unroll
                for (int j = 0; j < L; ++j) acc[j] = __builtin_fma(x, y[(s + j) % L], acc[j]);
                y[s] = col[min(t + s + tau0 + L, F) * PW];
            }
        }
#pragma unroll
        for (int j = 0; j < L; ++j) {
            const int tau = tau0 + j;
            if (tau < n_tau)
                G[static_cast<int64_t>(row) * n_tau + tau] = (acc[j] / static_cast<double>(F - tau)) / dn;
        }
    }
}

template <int LPW, int NT>
void launch_g2_ring(int L, dim3 grid, size_t lds, hipStream_t s, const double *I, int32_t F, int64_t n_q,
                    int32_t n_tau, const int32_t *rank, const double *den, double *G) {
    switch (L) {
    case 7: hipLaunchKernelGGL((k_g2_lags_ring<7, LPW, NT>), grid, dim3(NT), lds, s, I, F, n_q, n_tau, rank, den, G); break;
    case 8: hipLaunchKernelGGL((k_g2_lags_ring<8, LPW, NT>), grid, dim3(NT), lds, s, I, F, n_q, n_tau, rank, den, G); break;
    case 13: hipLaunchKernelGGL((k_g2_lags_ring<13, LPW, NT>), grid, dim3(NT), lds, s, I, F, n_q, n_tau, rank, den, G); break;
    case 16: hipLaunchKernelGGL((k_g2_lags_ring<16, LPW, NT>), grid, dim3(NT), lds, s, I, F, n_q, n_tau, rank, den, G); break;
    case 24: hipLaunchKernelGGL((k_g2_lags_ring<24, LPW, NT>), grid, dim3(NT), lds, s, I, F, n_q, n_tau, rank, den, G); break;
    default: hipLaunchKernelGGL((k_g2_lags_ring<32, LPW, NT>), grid, dim3(NT), lds, s, I, F, n_q, n_tau, rank, den, G); break;
    }
}

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

// Ring means from the tree's top level (rows of ncol columns): out[r][c] =
// total / n (NaN for an empty ring), count[r] = n.
__global__ __launch_bounds__(kBlock) void k_ring_mean_finish(const double *__restrict__ top, int64_t ncol,
                                                             int32_t R, const int32_t *__restrict__ ring_start,
                                                             const int32_t *__restrict__ top_off,
                                                             double *__restrict__ out, int32_t *__restrict__ count) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= static_cast<int64_t>(R) * ncol) return;
    const int r = static_cast<int>(i / ncol);
    const int64_t c = i - static_cast<int64_t>(r) * ncol;
    const int32_t n = ring_start[r + 1] - ring_start[r];
    out[i] = n > 0 ? top[static_cast<int64_t>(top_off[r]) * ncol + c] / static_cast<double>(n)
                   : __builtin_nan("");
    if (count && c == 0) count[r] = n;
}

// ---------------------------------------------------------------- F(q, tau)

// Rows of the per-pixel intermediate scattering function, Eq. (Fq_pq):
// G[rank[p]][tau] = (re, im) of [sum_{t < F - tau} p_t conj(p_{t+tau}) / (F - tau)] / f2,
// p_t = a_t + i b_t, accumulated for t = 0, 1, ... as
//   re = fma(a_t, a_{t+tau}, re), re = fma(b_t, b_{t+tau}, re),
//   im = fma(b_t, a_{t+tau}, im), im = fma(-a_t, b_{t+tau}, im).
// Staging and lag blocking as in k_g2_lags, with the complex series in LDS.
__device__ __forceinline__ void isf_step(double2 x, double2 y, double &re, double &im) {
    re = __builtin_fma(x.x, y.x, re);
    re = __builtin_fma(x.y, y.y, re);
    im = __builtin_fma(x.y, y.x, im);
    im = __builtin_fma(-x.x, y.y, im);
}

__device__ __forceinline__ void isf_store(double *G, int32_t row, int32_t n_tau, int tau, int F, double f2,
                                          double re, double im) {
    const double nt = static_cast<double>(F - tau);
    double *g = G + (static_cast<int64_t>(row) * n_tau + tau) * 2;
    g[0] = (re / nt) / f2;
    g[1] = (im / nt) / f2;
}

__global__ __launch_bounds__(kBlock) void k_isf_lags(const double2 *__restrict__ amp, int32_t F, int64_t n_q,
                                                     int32_t n_tau, int32_t lpw, const int32_t *__restrict__ rank,
                                                     double f2, double *__restrict__ G) {
    extern __shared__ double2 lds2[];
    const int pw = 1 << lpw;
    const int64_t p0 = static_cast<int64_t>(blockIdx.x) * pw;
    stage_series<8>(lds2, amp, F, lpw, n_q, p0);
    __syncthreads();
    const int pp = threadIdx.x & (pw - 1);
    const int slot = threadIdx.x >> lpw, n_slots = kBlock >> lpw;
    const int64_t p = p0 + pp;
    if (p >= n_q) return;
    const int32_t row = rank[p];
    if (row < 0) return;
    const int n_lb = (n_tau + kLagBlock - 1) / kLagBlock;
    for (int lb = slot; lb < n_lb; lb += n_slots) {
        const int tau0 = lb * kLagBlock;
        double re[kLagBlock], im[kLagBlock];
        double2 y[kLagBlock];
#pragma unroll
        for (int j = 0; j < kLagBlock; ++j) {
            re[j] = 0.0;
            im[j] = 0.0;
            y[j] = tau0 + j < F ? lds2[(tau0 + j) * pw + pp] : make_double2(0.0, 0.0);
        }
        const int t_main = F - tau0 - kLagBlock;  // t < t_main: lags and the next load in range
        int t = 0;
#pragma unroll 4
        for (; t < t_main; ++t) {
            const double2 x = lds2[t * pw + pp];
#pragma unroll
            for (int j = 0; j < kLagBlock; ++j) isf_step(x, y[j], re[j], im[j]);
#pragma unroll
            for (int j = 0; j + 1 < kLagBlock; ++j) y[j] = y[j + 1];
            y[kLagBlock - 1] = lds2[(t + tau0 + kLagBlock) * pw + pp];
        }
        for (; t + tau0 < F; ++t) {
            const double2 x = lds2[t * pw + pp];
#pragma unroll
            for (int j = 0; j < kLagBlock; ++j)
                if (t + tau0 + j < F) isf_step(x, y[j], re[j], im[j]);
#pragma unroll
            for (int j = 0; j + 1 < kLagBlock; ++j) y[j] = y[j + 1];
            const int nt = t + tau0 + kLagBlock;
            y[kLagBlock - 1] = nt < F ? lds2[nt * pw + pp] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int j = 0; j < kLagBlock; ++j)
            if (tau0 + j < n_tau) isf_store(G, row, n_tau, tau0 + j, F, f2, re[j], im[j]);
    }
}

// The register-ring form of k_isf_lags (as k_g2_lags_ring): blocks of L lags, the window
// of the L next amplitudes in a ring of registers, the step loop unrolled by L, rows past
// the series read from one zero row (the extra steps add products with 0, which leave
// every sum unchanged bit for bit), slots rotated by a quarter per block.  L is picked
// per call so that the lag blocks spread over the slots (7 for 100 lags over 16 slots).
template <int L, int LPW>
__global__ __launch_bounds__(kBlock) void k_isf_lags_ring(const double2 *__restrict__ amp, int32_t F, int64_t n_q,
                                                          int32_t n_tau, const int32_t *__restrict__ rank,
                                                          double f2, double *__restrict__ G) {
    constexpr int PW = 1 << LPW, kSlots = kBlock >> LPW;
    extern __shared__ double2 lds2[];
    const int64_t p0 = static_cast<int64_t>(blockIdx.x) * PW;
    stage_series<8>(lds2, amp, F, LPW, n_q, p0);
    if (static_cast<int>(threadIdx.x) < PW) lds2[(F << LPW) + threadIdx.x] = make_double2(0.0, 0.0);
    __syncthreads();
    const int pp = threadIdx.x & (PW - 1);
    const int slot = ((threadIdx.x >> LPW) + (blockIdx.x & 3) * (kSlots / 4)) & (kSlots - 1);
    const int64_t p = p0 + pp;
    if (p >= n_q) return;
    const int32_t row = rank[p];
    if (row < 0) return;
    const double2 *col = lds2 + pp;  // p_t at col[t * PW], t <= F (row F is zero)
    const int n_lb = (n_tau + L - 1) / L;
    for (int lb = slot; lb < n_lb; lb += kSlots) {
        const int tau0 = lb * L;
        const double2 *ys = col + tau0 * PW;
        double re[L], im[L];
        double2 y[L];
#pragma unroll
        for (int j = 0; j < L; ++j) {
            re[j] = 0.0;
            im[j] = 0.0;
            y[j] = col[min(tau0 + j, F) * PW];
        }
        const int steps = F - tau0;
        int t = 0;
        for (; t + 2 * L <= steps; t += L) {  // rows t + s and t + s + tau0 + L below F
            const double2 *xt = col + t * PW, *yt = ys + (t + L) * PW;
#pragma unroll
            for (int s = 0; s < L; ++s) {
                const double2 x = xt[s * PW];
#pragma unroll
                for (int j = 0; j < L; ++j) isf_step(x, y[(s + j) % L], re[j], im[j]);
                y[s] = yt[s * PW];
            }
        }
        for (; t < steps; t += L) {
#pragma unroll
            for (int s = 0; s < L; ++s) {
                const double2 x = col[min(t + s, F) * PW];
#pragma unroll
                for (int j = 0; j < L; ++j) isf_step(x, y[(s + j) % L], re[j], im[j]);
                y[s] = col[min(t + s + tau0 + L, F) * PW];
            }
        }
#pragma unroll
        for (int j = 0; j < L; ++j)
            if (tau0 + j < n_tau) isf_store(G, row, n_tau, tau0 + j, F, f2, re[j], im[j]);
    }
}

template <int LPW>
void launch_isf_ring(int L, dim3 grid, size_t lds, hipStream_t s, const double2 *amp, int32_t F, int64_t n_q,
                     int32_t n_tau, const int32_t *rank, double f2, double *G) {
    switch (L) {
    case 4: hipLaunchKernelGGL((k_isf_lags_ring<4, LPW>), grid, dim3(kBlock), lds, s, amp, F, n_q, n_tau, rank, f2, G); break;
    case 7: hipLaunchKernelGGL((k_isf_lags_ring<7, LPW>), grid, dim3(kBlock), lds, s, amp, F, n_q, n_tau, rank, f2, G); break;
    default: hipLaunchKernelGGL((k_isf_lags_ring<kLagBlock, LPW>), grid, dim3(kBlock), lds, s, amp, F, n_q, n_tau, rank, f2, G); break;
    }
}

// Same lag step reading global memory (series too long for LDS): one thread
// per (pixel, lag block).
__global__ __launch_bounds__(kBlock) void k_isf_lags_global(const double2 *__restrict__ amp, int64_t F,
                                                            int64_t n_q, int32_t n_tau,
                                                            const int32_t *__restrict__ rank, double f2,
                                                            double *__restrict__ G) {
    const int n_lb = (n_tau + kLagBlock - 1) / kLagBlock;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n_q * n_lb) return;
    const int64_t p = i % n_q;
    const int lb = static_cast<int>(i / n_q);
    const int32_t row = rank[p];
    if (row < 0) return;
    const int tau0 = lb * kLagBlock;
    double re[kLagBlock], im[kLagBlock];
#pragma unroll
    for (int j = 0; j < kLagBlock; ++j) re[j] = im[j] = 0.0;
    for (int64_t t = 0; t + tau0 < F; ++t) {
        const double2 x = amp[t * n_q + p];
#pragma unroll
        for (int j = 0; j < kLagBlock; ++j)
            if (t + tau0 + j < F) isf_step(x, amp[(t + tau0 + j) * n_q + p], re[j], im[j]);
    }
#pragma unroll
    for (int j = 0; j < kLagBlock; ++j)
        if (tau0 + j < n_tau) isf_store(G, row, n_tau, tau0 + j, static_cast<int>(F), f2, re[j], im[j]);
}

// Siegert relation and the contrast it predicts (Eqs. (bq_g2), (norm_Fq),
// (g2_from_fq), (beta_alt_int)), per ring r:
//   beta0 = g2[r][0] - 1,  lhs[r][tau] = (g2[r][tau] - 1) / beta0,
//   fhat2[r][tau] = |F[r][tau]|^2 / |F[r][0]|^2,  |z|^2 = fma(re, re, im * im),
//   beta[l][r] = beta0 * fma(2, s, 1) / W,  W = 2^l,
//   s = sum over k = 1 .. W-1 in order of fma(1 - k / W, fhat2[r][k], s).
// Threads [0, R n_tau) form lhs and fhat2, the next R n_levels form beta.
__global__ __launch_bounds__(kBlock) void k_siegert(const double *__restrict__ g2, const double *__restrict__ F,
                                                    int32_t R, int32_t n_tau, int32_t n_levels,
                                                    double *__restrict__ lhs, double *__restrict__ fhat2,
                                                    double *__restrict__ beta) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t n1 = static_cast<int64_t>(R) * n_tau;
    if (i < n1) {
        const int r = static_cast<int>(i / n_tau);
        const double *Fr = F + static_cast<int64_t>(r) * n_tau * 2;
        const int64_t k = i - static_cast<int64_t>(r) * n_tau;
        const double beta0 = g2[static_cast<int64_t>(r) * n_tau] - 1.0;
        if (lhs) lhs[i] = (g2[i] - 1.0) / beta0;
        if (fhat2) {
            const double f0 = __builtin_fma(Fr[0], Fr[0], Fr[1] * Fr[1]);
            fhat2[i] = __builtin_fma(Fr[2 * k], Fr[2 * k], Fr[2 * k + 1] * Fr[2 * k + 1]) / f0;
        }
    } else if (beta && i < n1 + static_cast<int64_t>(n_levels) * R) {
        const int64_t j = i - n1;
        const int l = static_cast<int>(j / R), r = static_cast<int>(j - static_cast<int64_t>(l) * R);
        const double *Fr = F + static_cast<int64_t>(r) * n_tau * 2;
        const double beta0 = g2[static_cast<int64_t>(r) * n_tau] - 1.0;
        const double f0 = __builtin_fma(Fr[0], Fr[0], Fr[1] * Fr[1]);
        const int64_t W = int64_t(1) << l;
        const double w = static_cast<double>(W);
        double acc = 0.0;
        for (int64_t k = 1; k < W; ++k) {
            const double fh = __builtin_fma(Fr[2 * k], Fr[2 * k], Fr[2 * k + 1] * Fr[2 * k + 1]) / f0;
            acc = __builtin_fma(1.0 - static_cast<double>(k) / w, fh, acc);
        }
        beta[static_cast<int64_t>(l) * R + r] = beta0 * __builtin_fma(2.0, acc, 1.0) / w;
    }
}

// ---------------------------------------------------------------- XSVS

// Launch order of the gathering XSVS blocks.  A block group (kLvChunksPerBlock
// chunks of one ring, kLvSpan ring rows) starts at the pixel whose position in
// its ring's list is a multiple of kLvSpan; order[] lists the groups by that
// pixel's index, so that the groups of neighbouring rings over the same detector
// rows come next to each other (their rows share cache lines).
constexpr int32_t kLvSpan = kLvChunksPerBlock * kLvRows;

__device__ __forceinline__ int32_t group_started_at(int64_t p, const int32_t *__restrict__ key,
                                                    const int32_t *__restrict__ rank, const int32_t *start_s,
                                                    const int32_t *grp_s) {
    const int32_t r = key[p];
    if (r < 0) return -1;
    const int32_t j = rank[p] - start_s[r];
    return j % kLvSpan == 0 ? grp_s[r] + j / kLvSpan : -1;
}

// cnt[b] = groups starting in pixel block b (kPartChunk pixels).
__global__ __launch_bounds__(kBlock) void k_group_count(const int32_t *__restrict__ key,
                                                        const int32_t *__restrict__ rank, int64_t n_q, int32_t R,
                                                        const int32_t *__restrict__ ring_start,
                                                        const int32_t *__restrict__ grp_off,
                                                        int32_t *__restrict__ cnt) {
    __shared__ int32_t start_s[kMaxRings + 1], grp_s[kMaxRings + 1], wsum[kBlock / 64];
    for (int i = threadIdx.x; i <= R; i += kBlock) {
        start_s[i] = ring_start[i];
        grp_s[i] = grp_off[i];
    }
    __syncthreads();
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kPartChunk;
    int32_t c = 0;
    for (int i = threadIdx.x; i < kPartChunk; i += kBlock)
        if (base + i < n_q && group_started_at(base + i, key, rank, start_s, grp_s) >= 0) ++c;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int w = 0; w < kBlock / 64; ++w) t += wsum[w];
        cnt[blockIdx.x] = t;
    }
}

// order[k] = the k-th group in ascending index of its first pixel: block b
// starts at off[b] (the exclusive scan of the counts) and places its groups in
// pixel order (one ballot per wave and step).
__global__ __launch_bounds__(kBlock) void k_group_scatter(const int32_t *__restrict__ key,
                                                          const int32_t *__restrict__ rank, int64_t n_q, int32_t R,
                                                          const int32_t *__restrict__ ring_start,
                                                          const int32_t *__restrict__ grp_off,
                                                          const int32_t *__restrict__ off_b,
                                                          int32_t *__restrict__ order) {
    constexpr int kWaves = kBlock / 64;
    __shared__ int32_t start_s[kMaxRings + 1], grp_s[kMaxRings + 1], wsum[kWaves];
    for (int i = threadIdx.x; i <= R; i += kBlock) {
        start_s[i] = ring_start[i];
        grp_s[i] = grp_off[i];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t run = off_b[blockIdx.x];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kPartChunk;
    for (int st = 0; st < kPartChunk / kBlock; ++st) {
        const int64_t p = base + st * kBlock + threadIdx.x;
        const int32_t g = p < n_q ? group_started_at(p, key, rank, start_s, grp_s) : -1;
        const uint64_t m = __ballot(g >= 0);
        __syncthreads();  // wsum of the previous step read
        if (lane == 0) wsum[wave] = __builtin_popcountll(m);
        __syncthreads();
        int32_t off = run;
        for (int w = 0; w < wave; ++w) off += wsum[w];
        if (g >= 0) order[off + __builtin_popcountll(m & ((uint64_t(1) << lane) - 1))] = g;
        for (int w = 0; w < kWaves; ++w) run += wsum[w];
    }
}

// Windows of base level L (K per row) and the next kLvDepth - 1 levels.
// Block (block group of kLvChunksPerBlock consecutive 32-row chunks of one
// ring, 64-window tile k0..).  Each chunk of the ring's rows of the tile's 64
// base windows is staged in LDS (row stride kLvStride):
//   columns [0, 64)    level L windows,
//   [64, 96) L+1,  [96, 112) L+2,  [112, 120) L+3,  [120, 124) L+4,
//   [124, 126) L+5, [126] L+6,
// the coarser levels formed by pairwise sums J_{l+1}[j] = J_l[2j] + J_l[2j+1].
// Thread t < 126 owns column t (one window of one level): it forms each
// chunk's pairwise trees of its values J and of their squares J*J (the two
// moments of Eq. (bq_Iq)) and adds the chunk trees of the block as the ring
// tree does (chunks 0 + 1, 2 + 3, then the two), writing that node over the
// block's 128 ring rows to csum[group][tile * 256 + t] and [tile * 256 + 128 + t].
// Level L+6 (one window per full tile) also goes to `next` [K >> 6][ld] (ring
// rows m contiguous, as in a frame) for the launch that continues from it.
// kGather: rows gathered from the frames X[k][list[m]], on a one-dimensional
// grid: the (tile, group) work items, tile-major with the groups in the order
// of `order`, are split into eight equal consecutive runs, run x taken by
// blocks x, x + 8, x + 16, ... (consecutive blocks go to different XCDs, so
// each XCD walks its run in order and its L2 sees the rows of neighbouring
// rings together).  Otherwise rows m read from the ring-ordered table
// X[k][m] that the previous launch wrote, grid (group, tile).  Both have ld
// elements per frame or table column.
template <bool kGather>
__global__ __launch_bounds__(kBlock) void k_xsvs_chunks(const double *__restrict__ X, int64_t K, int64_t ld,
                                                        const int32_t *__restrict__ list, int32_t R,
                                                        const int32_t *__restrict__ ring_start,
                                                        const int32_t *__restrict__ grp_off,
                                                        const int32_t *__restrict__ order, int64_t n_tiles,
                                                        int64_t ncol, double *__restrict__ csum,
                                                        double *__restrict__ next) {
    __shared__ double tile[kLvRows * kLvStride];
    __shared__ int32_t g_s[kMaxRings + 1];
    for (int i = threadIdx.x; i <= R; i += kBlock) g_s[i] = grp_off[i];
    __syncthreads();
    int64_t gb, tile_idx;
    if (kGather) {
        const int64_t G = g_s[R], work = G * n_tiles, per = (work + 7) >> 3;
        const int64_t j = blockIdx.x >> 3;
        if (j >= per) return;  // block-uniform, as below
        const int64_t w = static_cast<int64_t>(blockIdx.x & 7) * per + j;
        if (w >= work) return;
        tile_idx = w / G;
        gb = order[w - tile_idx * G];
    } else {
        gb = blockIdx.x;
        tile_idx = blockIdx.y;
        if (gb >= g_s[R]) return;
    }
    const int r = ring_of(g_s, R, gb);
    const int64_t k0 = tile_idx * kLvTile;
    const int W = static_cast<int>(std::min<int64_t>(kLvTile, K - k0));
    const int32_t a = ring_start[r], b = ring_start[r + 1];
    const int32_t c_first = static_cast<int32_t>((gb - g_s[r]) * kLvChunksPerBlock);
    const int32_t n_chunks_ring = (b - a + kLvRows - 1) / kLvRows;
    const int t = threadIdx.x;
    const int64_t col = tile_idx * kLvCols + t;
    const bool owner = t < kLvHalf - 2;
    const bool want_next = next != nullptr && k0 + kLvTile <= K;

    // staging map: element i of thread t is (row q_t, column c_t + i * dci):
    // lanes along the ring (kLvRows rows), 8 windows per step; the thread's row,
    // hence its pixel list[m0 + q_t] (gather) or table row m0 + q_t, is fixed
    const int q_t = t & (kLvRows - 1);
    const int c_t = t / kLvRows;
    constexpr int dci = kBlock / kLvRows;
    auto load_chunk = [&](double (&val)[kLvLoads], int32_t m0, int rows) {
        const bool ok = q_t < rows;
        const int64_t p = ok ? (kGather ? list[m0 + q_t] : m0 + q_t) : 0;
#pragma unroll
        for (int i = 0; i < kLvLoads; ++i) {
            const int c = c_t + i * dci;
            val[i] = ok && c < W ? X[(k0 + c) * ld + p] : 0.0;
        }
    };

    const int32_t c_end = std::min<int32_t>(n_chunks_ring, c_first + kLvChunksPerBlock);
    auto chunk_rows = [&](int32_t ch) { return std::min<int32_t>(kLvRows, b - (a + ch * kLvRows)); };
    // two chunks in flight: buffer A carries the even steps, B the odd ones; a
    // buffer is refilled with the chunk two steps ahead as soon as it is in LDS
    double bufA[kLvLoads], bufB[kLvLoads];
    // the owner's node sums: chunks 0 + 1 in (p1, p2), chunks 2 + 3 in (u1, u2)
    double p1 = 0.0, p2 = 0.0, u1 = 0.0, u2 = 0.0;
    load_chunk(bufA, a + c_first * kLvRows, chunk_rows(c_first));
    if (c_first + 1 < c_end) load_chunk(bufB, a + (c_first + 1) * kLvRows, chunk_rows(c_first + 1));
    auto process = [&](double (&buf)[kLvLoads], int32_t ch) {
        const int32_t mrow = a + ch * kLvRows;
        const int crow = chunk_rows(ch);
        __syncthreads();  // previous chunk consumed
#pragma unroll
        for (int i = 0; i < kLvLoads; ++i) tile[q_t * kLvStride + c_t + i * dci] = buf[i];
        if (ch + 2 < c_end) load_chunk(buf, a + (ch + 2) * kLvRows, chunk_rows(ch + 2));
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
                if (want_next && q < crow)
                    next[(k0 >> kLvDepth) * ld + mrow + q] = y6;
            }
        }
        __syncthreads();
        if (owner) {
            const double *colp = tile + t;
            double s1, s2;
            tree2_upto32(crow, [&](int i) { return colp[i * kLvStride]; }, s1, s2);
            switch (ch - c_first) {
            case 0: p1 = s1; p2 = s2; break;
            case 1: p1 += s1; p2 += s2; break;
            case 2: u1 = s1; u2 = s2; break;
            default: u1 += s1; u2 += s2; break;
            }
        }
    };
    for (int32_t ch = c_first; ch < c_end; ch += 2) {
        process(bufA, ch);
        if (ch + 1 < c_end) process(bufB, ch + 1);
    }
    if (owner) {
        if (c_end - c_first > 2) {
            p1 += u1;
            p2 += u2;
        }
        double *out = csum + gb * ncol + col;
        out[0] = p1;
        out[kLvHalf] = p2;
    }
}

// Exposure levels handled by one launch group: level base + d for d < depths,
// bwin[d] = [R][K_d] per-window contrast, K_d = K_base >> d.
struct LevelOut {
    double *bwin[kLvDepth];
    int64_t K[kLvDepth];
};

// beta per (ring, window column) from the tree top of the two moments:
// m1 = S1 / n, m2 = S2 / n, beta = (m2 - m1^2) / m1^2 (NaN for an empty ring),
// to the column's level and window.  Threads cover R x (ncol / 2) columns of J sums.
__global__ __launch_bounds__(kBlock) void k_xsvs_beta(const double *__restrict__ top, int64_t ncol, int64_t K,
                                                      int32_t depths, int32_t R,
                                                      const int32_t *__restrict__ ring_start,
                                                      const int32_t *__restrict__ top_off, LevelOut lo) {
    const int64_t half = ncol / 2;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= static_cast<int64_t>(R) * half) return;
    const int r = static_cast<int>(i / half);
    const int64_t h = i - static_cast<int64_t>(r) * half;
    const int64_t tile = h / kLvHalf;
    const int t = static_cast<int>(h % kLvHalf);
    const int64_t k0 = tile * kLvTile;
    const int64_t c = tile * kLvCols + t;
    int d = -1, j = 0;
#pragma unroll
    for (int dd = 0; dd < kLvDepth; ++dd) {
        const int o = 2 * kLvTile - ((2 * kLvTile) >> dd), w = kLvTile >> dd;
        if (dd < depths && t >= o && t < o + w) {
            d = dd;
            j = t - o;
        }
    }
    if (d < 0 || k0 + (static_cast<int64_t>(j) + 1) * (int64_t(1) << d) > K) return;
    const int32_t n = ring_start[r + 1] - ring_start[r];
    double beta = __builtin_nan("");
    if (n > 0) {
        const double *row = top + static_cast<int64_t>(top_off[r]) * ncol;
        const double m1 = row[c] / static_cast<double>(n);
        const double m2 = row[c + kLvHalf] / static_cast<double>(n);
        const double sq = m1 * m1;
        beta = (m2 - sq) / sq;
    }
    lo.bwin[d][static_cast<int64_t>(r) * lo.K[d] + (k0 >> d) + j] = beta;
}

// Mean over windows, block per (ring r, level d of the group): beta_out[d][r] =
// (sum_k bwin_d[r][k] in order) / K_d; optional per-window output beta_win[d][k][r]
// (rows k >= K_d filled with NaN).
__global__ __launch_bounds__(kBlock) void k_xsvs_mean(LevelOut lo, int64_t F, int32_t R,
                                                      double *__restrict__ beta_out,
                                                      double *__restrict__ beta_win) {
    __shared__ double buf[kBlock];
    // block (ring r, level d of the launch group): level L + d has K windows per ring
    const int r = blockIdx.x, d = blockIdx.y;
    const int64_t K = lo.K[d];
    const double *row = lo.bwin[d] + static_cast<int64_t>(r) * K;
    beta_out += static_cast<int64_t>(d) * R;
    double *beta_win_level = beta_win ? beta_win + static_cast<int64_t>(d) * F * R : nullptr;
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

// ---------------------------------------------------------------- frame sums, histogram

constexpr int kSumMaxLog = 24;  // frame sums of up to 2^24 terms

// J[k][p] = scale * pairwise tree over i < n_sum of I[k s_out + i s_sum][p]: a binary
// counter holds the complete subtrees (st[l]: 2^l terms while bit l of n_done
// is set; a new term merges left + right up the set bits), then the fold from
// the right, which is the bottom-up tree with the odd element carried up.  The
// counter is the same in every lane, so its branches are uniform.  LV levels hold
// any n_sum < 2^LV (the host picks the smallest built LV, so the counter takes
// few registers and more waves fit a SIMD).  A thread owns PX consecutive pixels
// (one 16-byte load per term for PX = 2, when n_q is even) and reads AHEAD terms
// at a time, so that several loads are in flight.
template <int PX> struct SumVec;
template <> struct SumVec<1> {
    using T = double;
    static __device__ double at(const T &v, int) { return v; }
};
template <> struct SumVec<2> {
    using T = double2;
    static __device__ double at(const T &v, int i) { return i ? v.y : v.x; }
};

template <int PX, int LV, int AHEAD>
__global__ __launch_bounds__(kBlock) void k_frame_sums(const double *__restrict__ I, int64_t n_q, int64_t n_out,
                                                       int64_t s_out, int64_t n_sum, int64_t s_sum, double scale,
                                                       double *__restrict__ J) {
    using V = SumVec<PX>;
    using T = typename V::T;
    const int64_t nv = n_q / PX;  // n_q is a multiple of PX
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (idx >= n_out * nv) return;
    const int64_t k = idx / nv, pv = idx - k * nv;
    double st[PX][LV];
    int64_t n_done = 0;
    const T *src = reinterpret_cast<const T *>(I + k * s_out * n_q) + pv;
    const int64_t stride = s_sum * nv;
    for (int64_t i0 = 0; i0 < n_sum; i0 += AHEAD) {
        T vv[AHEAD];
#pragma unroll
        for (int u = 0; u < AHEAD; ++u) vv[u] = i0 + u < n_sum ? src[(i0 + u) * stride] : T{};
#pragma unroll
        for (int u = 0; u < AHEAD; ++u) {
            if (i0 + u >= n_sum) break;  // uniform
#pragma unroll
            for (int x = 0; x < PX; ++x) {
                double v = V::at(vv[u], x);
                bool carry = true;
#pragma unroll
                for (int l = 0; l < LV; ++l) {
                    if (carry) {
                        if ((n_done >> l) & 1) {
                            v = st[x][l] + v;
                        } else {
                            st[x][l] = v;
                            carry = false;
                        }
                    }
                }
            }
            ++n_done;
        }
    }
#pragma unroll
    for (int x = 0; x < PX; ++x) {
        double sum = 0.0;
        bool have = false;
#pragma unroll
        for (int l = 0; l < LV; ++l)
            if ((n_done >> l) & 1) {
                sum = have ? st[x][l] + sum : st[x][l];
                have = true;
            }
        J[k * n_q + pv * PX + x] = sum * scale;
    }
}

// Ring-ordered rows of the frames: X[m][t] = I[t][list[m]] for the in-ring pixels
// m < ring_start[R] (list holds no pixel beyond them).  A block moves a tile of
// kRowTile ring rows x kRowTile frames through LDS: it reads each frame's run of
// ring pixels (neighbouring ring pixels share cache lines) and writes whole rows.
constexpr int kRowTile = 64;
__global__ __launch_bounds__(kBlock) void k_ring_rows(const double *__restrict__ I, int64_t F, int64_t n_q,
                                                      const int32_t *__restrict__ list,
                                                      const int32_t *__restrict__ ring_start, int32_t R,
                                                      double *__restrict__ X) {
    __shared__ double tile[kRowTile][kRowTile + 1];
    const int64_t m0 = static_cast<int64_t>(blockIdx.x) * kRowTile, t0 = static_cast<int64_t>(blockIdx.y) * kRowTile;
    const int64_t rows = ring_start[R];
    if (m0 >= rows) return;  // block-uniform
    const int i = threadIdx.x & (kRowTile - 1), g = threadIdx.x / kRowTile;
    constexpr int kGroups = kBlock / kRowTile;
    const int64_t m = m0 + i;
    const int64_t p = m < rows ? list[m] : 0;
    for (int j = g; j < kRowTile; j += kGroups) {
        const int64_t t = t0 + j;
        tile[i][j] = (m < rows && t < F) ? I[t * n_q + p] : 0.0;
    }
    __syncthreads();
    for (int r = g; r < kRowTile; r += kGroups) {
        const int64_t mr = m0 + r, t = t0 + i;
        if (mr < rows && t < F) X[mr * F + t] = tile[r][i];
    }
}

// Histogram of u = (I / <I>_ring) * scale per (frame, ring): bin floor(u) for
// 0 <= u < n_bins (u <= 0: bin 0), else the overflow bin n_bins (NaN too).
// Block = (kHistSpan pixels of one frame, so that clearing and flushing the LDS
// histogram is paid once per 4096 pixels); counts gathered in LDS, then added to
// counts[(t R + r)(n_bins + 1) + b] with global atomics.
constexpr int64_t kHistSpan = 16 * kBlock;
__global__ __launch_bounds__(kBlock) void k_ring_hist(const double *__restrict__ I, int64_t n_q,
                                                      const int32_t *__restrict__ key, int32_t R,
                                                      const double *__restrict__ mean, int32_t n_bins,
                                                      double scale, unsigned long long *__restrict__ counts) {
    extern __shared__ unsigned int h[];
    const int nb1 = n_bins + 1, nh = R * nb1;
    for (int i = threadIdx.x; i < nh; i += kBlock) h[i] = 0u;
    __syncthreads();
    const int64_t t = blockIdx.y;
    const int64_t p_end = std::min<int64_t>(n_q, static_cast<int64_t>(blockIdx.x + 1) * kHistSpan);
    for (int64_t p = static_cast<int64_t>(blockIdx.x) * kHistSpan + threadIdx.x; p < p_end; p += kBlock) {
        const int r = key[p];
        if (r >= 0) {
            const double u = (I[t * n_q + p] / mean[t * R + r]) * scale;
            int b = n_bins;
            if (u < static_cast<double>(n_bins)) b = u > 0.0 ? static_cast<int>(floor(u)) : 0;
            atomicAdd(&h[r * nb1 + b], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nh; i += kBlock)
        if (h[i]) atomicAdd(&counts[t * nh + i], static_cast<unsigned long long>(h[i]));
}

__global__ __launch_bounds__(kBlock) void k_fill_u64(unsigned long long *__restrict__ p, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kBlock)
        p[i] = 0ull;
}

// out[c][r] = in[r][c] for an R x C table.
__global__ __launch_bounds__(kBlock) void k_transpose_rt(const double *__restrict__ in, int64_t R, int64_t C,
                                                         double *__restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= R * C) return;
    const int64_t r = i / C, c = i - r * C;
    out[c * R + r] = in[i];
}

// ---------------------------------------------------------------- host side

// Tree levels above the leaves so that every ring of up to n_q leaves ends with one value.
int tree_levels(int64_t n_q) {
    int levels = 0;
    int64_t e = std::max<int64_t>(n_q, 1);
    while (e > 1) {
        e = (e + kGroup - 1) / kGroup;
        ++levels;
    }
    return std::max(levels, 1);
}

// Elements of tree level l over all R rings, at most (level 0: n_q).
int64_t level_bound(int64_t n_q, int32_t R, int l) {
    int64_t e = std::max<int64_t>(n_q, 1);
    for (int i = 0; i < l; ++i) e = (e + kGroup - 1) / kGroup + R;
    return e;
}

// Where a reduction's working buffers come from: the library's per-stream cached
// scratch (base == nullptr), or consecutive 256-byte-aligned pieces of one fixed
// device buffer of cap bytes (the no-allocation entry point).
struct Arena {
    hipStream_t s;
    char *base = nullptr;
    size_t cap = 0, used = 0;
    xs_status get(Slot slot, size_t bytes, void **p) {
        if (!base) return scratch(s, slot, bytes, p);
        const size_t need = (std::max<size_t>(bytes, 1) + 255) & ~size_t(255);
        if (need > cap - used)
            return set_error(XS_EINVAL, "working buffers need more than the %zu-byte fixed scratch", cap);
        *p = base + used;
        used += need;
        return XS_OK;
    }
};

struct Partition {
    int32_t *start = nullptr;  // ring starts [R + 1] = tree level 0 offsets
    int32_t *rank = nullptr;
    int32_t *list = nullptr;
    int32_t *lev = nullptr;    // [(levels + 1)][R + 1]
    int32_t *grp = nullptr;    // [R + 1] block groups of level-1 chunks
    int levels = 0;
};

// Ring starts, ring-order ranks (-1 for pixels with key -1), the inverse list
// and the tree offsets.
xs_status partition(Arena &A, const int32_t *key, int64_t n_q, int32_t R, Partition *P) {
    hipStream_t s = A.s;
    const int64_t nb = (n_q + kPartChunk - 1) / kPartChunk;
    const int levels = tree_levels(n_q);
    void *cnt = nullptr, *rk = nullptr;
    XS_TRY(A.get(SLOT_RING_CNT, sizeof(int32_t) * (nb * R + R + (levels + 1) * (R + 1) + (R + 1)), &cnt));
    XS_TRY(A.get(SLOT_RING_LIST, sizeof(int32_t) * 2 * std::max<int64_t>(n_q, 1), &rk));
    int32_t *c = static_cast<int32_t *>(cnt);
    int32_t *tot = c + nb * R;
    P->lev = tot + R;
    P->grp = P->lev + (levels + 1) * (R + 1);
    P->start = P->lev;
    P->rank = static_cast<int32_t *>(rk);
    P->list = P->rank + std::max<int64_t>(n_q, 1);
    P->levels = levels;
    if (n_q > 0)
        hipLaunchKernelGGL(k_part_count, dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, key, n_q, R, c);
    hipLaunchKernelGGL(k_part_scan_ring, dim3(static_cast<unsigned>(R)), dim3(kBlock), 0, s, c, nb, R, tot);
    hipLaunchKernelGGL(k_tree_offsets, dim3(1), dim3(kBlock), 0, s, tot, R, levels, kLvChunksPerBlock, P->lev,
                       P->grp);
    if (n_q > 0)
        hipLaunchKernelGGL(k_part_rank, dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, key, n_q, R, c,
                           P->start, P->rank, P->list);
    XS_HIP(hipGetLastError());
    return XS_OK;
}

// Reduce tree level `from` (rows of ncol in `a`) to the top level (one row per
// ring); `a` and `b` alternate as input and output.  Returns the top's buffer.
double *reduce_tree(hipStream_t s, const Partition &P, int32_t R, int from, int64_t n_q, int64_t ncol, double *a,
                    double *b) {
    double *in = a, *out = b;
    for (int l = from; l < P.levels; ++l) {
        const int64_t n_out = level_bound(n_q, R, l + 1);
        hipLaunchKernelGGL(k_group_tree<kGroup>, dim3(blocks_for(n_out * ncol)), dim3(kBlock), 0, s, in, out, ncol,
                           P.lev + static_cast<int64_t>(l) * (R + 1), P.lev + static_cast<int64_t>(l + 1) * (R + 1),
                           R);
        std::swap(in, out);
    }
    return in;
}

// g2 with its working buffers from `A`; timed (HIP events) only on the cached-scratch path.
xs_status g2_rings_in(Arena &A, const double *I, int64_t F, int64_t n_q, const double *q,
                      const RingEdges &edges, int32_t n_tau, double *g2_out, int32_t *ring_count) {
    hipStream_t s = A.s;
    const int32_t R = edges.n_rings;
    const bool timed = A.base == nullptr;
    TimerScope tm(s, TIMER_G2, timed);
    void *key = nullptr, *G = nullptr, *G2 = nullptr, *den = nullptr;
    XS_TRY(A.get(SLOT_RING_KEY, sizeof(int32_t) * std::max<int64_t>(n_q, 1), &key));
    XS_TRY(A.get(SLOT_PIXEL2, sizeof(double) * std::max<int64_t>(n_q, 1), &den));
    XS_TRY(A.get(SLOT_G, sizeof(double) * std::max<int64_t>(n_q * n_tau, 1), &G));
    XS_TRY(A.get(SLOT_LEVEL_B, sizeof(double) * level_bound(n_q, R, 1) * n_tau, &G2));
    int32_t *k = static_cast<int32_t *>(key);
    double *dn = static_cast<double *>(den);
    if (n_q > 0) {
        hipLaunchKernelGGL(k_pixel_mean, dim3(blocks_for(n_q)), dim3(kBlock), 0, s, I, F, n_q, q, edges, k, dn);
        XS_HIP(hipGetLastError());
    }
    Partition P;
    XS_TRY(partition(A, k, n_q, R, &P));
    if (n_q > 0) {
        // pixels per block for the LDS path: the largest power of two <= 64 whose series
        // (plus the zero rows after it) fit 64 KiB; the lag block L: the smallest built size
        // that leaves no slot with two blocks
        auto pick_l = [&](int lpw, int threads = kBlock) {
            const int n_slots = threads >> lpw;
            const int want = static_cast<int>((n_tau + n_slots - 1) / n_slots);
            return want <= 7 ? 7 : want <= 8 ? 8 : want <= 13 ? 13 : want <= 16 ? 16 : want <= 24 ? 24 : 32;
        };
        auto fits = [&](int lpw, int rows_after) {
            return ((F + rows_after) << lpw) * static_cast<int64_t>(sizeof(double)) <= 65536;
        };
        int lpw = 6;
        while (lpw > 0 && !fits(lpw, 32)) --lpw;
        constexpr int kRingThreads = kBlock;
        // register-ring kernel: one zero row after the series, 16 pixels per block (six
        // blocks per CU at 200 frames, so that the staging of some overlaps the sums of others)
        constexpr int kRingLpw = 4;
        const int32_t F32 = static_cast<int32_t>(F);
        double *Gd = static_cast<double *>(G);
        if (fits(kRingLpw, 1)) {
            const int L = pick_l(kRingLpw, kRingThreads);
            const size_t lds = sizeof(double) * ((F + 1) << kRingLpw);
            const dim3 grid(static_cast<unsigned>((n_q + (int64_t(1) << kRingLpw) - 1) >> kRingLpw));
            launch_g2_ring<kRingLpw, kRingThreads>(L, grid, lds, s, I, F32, n_q, n_tau, P.rank, dn, Gd);
        } else if (fits(lpw, 32)) {
            const size_t lds = sizeof(double) * ((F + 32) << lpw);
            const int64_t pw = int64_t(1) << lpw;
            const int want = pick_l(lpw);
            const dim3 grid(static_cast<unsigned>((n_q + pw - 1) / pw));
            const int32_t lpw32 = static_cast<int32_t>(lpw);
            if (want <= 8)
                hipLaunchKernelGGL(k_g2_lags<8>, grid, dim3(kBlock), lds, s, I, F32, n_q, n_tau, lpw32, P.rank, dn, Gd);
            else if (want <= 13)
                hipLaunchKernelGGL(k_g2_lags<13>, grid, dim3(kBlock), lds, s, I, F32, n_q, n_tau, lpw32, P.rank, dn, Gd);
            else if (want <= 16)
                hipLaunchKernelGGL(k_g2_lags<16>, grid, dim3(kBlock), lds, s, I, F32, n_q, n_tau, lpw32, P.rank, dn, Gd);
            else if (want <= 24)
                hipLaunchKernelGGL(k_g2_lags<24>, grid, dim3(kBlock), lds, s, I, F32, n_q, n_tau, lpw32, P.rank, dn, Gd);
            else
                hipLaunchKernelGGL(k_g2_lags<32>, grid, dim3(kBlock), lds, s, I, F32, n_q, n_tau, lpw32, P.rank, dn, Gd);
        } else {
            const int64_t n_lb = (n_tau + kLagBlock - 1) / kLagBlock;
            hipLaunchKernelGGL(k_g2_lags_global, dim3(blocks_for(n_q * n_lb)), dim3(kBlock), 0, s, I, F, n_q,
                               n_tau, P.rank, dn, static_cast<double *>(G));
        }
        XS_HIP(hipGetLastError());
    }
    // ring sums: pairwise tree over the rank-ordered rows of G
    const double *top = reduce_tree(s, P, R, 0, n_q, n_tau, static_cast<double *>(G), static_cast<double *>(G2));
    hipLaunchKernelGGL(k_ring_mean_finish, dim3(blocks_for(static_cast<int64_t>(R) * n_tau)), dim3(kBlock), 0, s,
                       top, static_cast<int64_t>(n_tau), R, P.start,
                       P.lev + static_cast<int64_t>(P.levels) * (R + 1), g2_out, ring_count);
    tm.end(static_cast<double>(F) * n_q * sizeof(double));
    XS_HIP(hipGetLastError());
    return XS_OK;
}

// Fixed working memory of the no-allocation g2 call: one array per device, mapped
// when the code object is loaded.  Host code must never pass `g2_fixed_scratch`
// itself to a kernel (in host code the name is a host-side stand-in); its device
// address comes from hipGetSymbolAddress, once per device.
constexpr size_t kFixedScratchBytes = size_t(64) << 20;
__device__ __align__(256) char g2_fixed_scratch[kFixedScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_fixed_mu;
char *g_fixed_ptr[kMaxDevices] = {};

xs_status fixed_scratch(char **out) {
    int dev = 0;
    XS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return set_error(XS_ENOTSUP, "device index %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_fixed_mu);
    if (!g_fixed_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(g2_fixed_scratch));
        if (e != hipSuccess || !p) return hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
        g_fixed_ptr[dev] = static_cast<char *>(p);
    }
    *out = g_fixed_ptr[dev];
    return XS_OK;
}

}  // namespace

xs_status g2_rings(hipStream_t s, const double *I, int64_t F, int64_t n_q, const double *q,
                   const RingEdges &edges, int32_t n_tau, double *g2_out, int32_t *ring_count) {
    Arena A{s};
    return g2_rings_in(A, I, F, n_q, q, edges, n_tau, g2_out, ring_count);
}

xs_status g2_rings_fixed(hipStream_t s, const double *I, int64_t F, int64_t n_q, const double *q,
                         const RingEdges &edges, int32_t n_tau, double *g2_out, int32_t *ring_count) {
    char *base = nullptr;
    XS_TRY(fixed_scratch(&base));
    Arena A{s, base, kFixedScratchBytes, 0};
    return g2_rings_in(A, I, F, n_q, q, edges, n_tau, g2_out, ring_count);
}

size_t g2_fixed_scratch_bytes() { return kFixedScratchBytes; }

xs_status isf_rings(hipStream_t s, const double *amp, int64_t F, int64_t n_q, const double *q,
                    const RingEdges &edges, int32_t n_tau, double f2, double *F_out, int32_t *ring_count) {
    const int32_t R = edges.n_rings;
    const int64_t ncol = 2 * static_cast<int64_t>(n_tau);
    TimerScope tm(s, TIMER_ISF);
    void *key = nullptr, *G = nullptr, *G2 = nullptr;
    XS_TRY(scratch(s, SLOT_RING_KEY, sizeof(int32_t) * std::max<int64_t>(n_q, 1), &key));
    XS_TRY(scratch(s, SLOT_G, sizeof(double) * std::max<int64_t>(n_q * ncol, 1), &G));
    XS_TRY(scratch(s, SLOT_LEVEL_B, sizeof(double) * level_bound(n_q, R, 1) * ncol, &G2));
    int32_t *k = static_cast<int32_t *>(key);
    if (n_q > 0) {
        hipLaunchKernelGGL(k_ring_key, dim3(blocks_for(n_q)), dim3(kBlock), 0, s, q, n_q, edges, k);
        XS_HIP(hipGetLastError());
    }
    Partition P;
    Arena cached{s};
    XS_TRY(partition(cached, k, n_q, R, &P));
    const double2 *a2 = reinterpret_cast<const double2 *>(amp);
    if (n_q > 0) {
        // pixels per block for the LDS path: largest power of two <= 64 with the
        // complex series (and, for the register-ring kernel, one zero row) in at most 64 KiB
        int lpw = 6;
        while (lpw > 0 && (F << lpw) * static_cast<int64_t>(sizeof(double2)) > 65536) --lpw;
        int rlpw = 5;
        while (rlpw > 3 && ((F + 1) << rlpw) * static_cast<int64_t>(sizeof(double2)) > 65536) --rlpw;
        if (((F + 1) << rlpw) * static_cast<int64_t>(sizeof(double2)) <= 65536) {
            const size_t lds = sizeof(double2) * ((F + 1) << rlpw);
            const dim3 grid(static_cast<unsigned>((n_q + (int64_t(1) << rlpw) - 1) >> rlpw));
            const int32_t F32 = static_cast<int32_t>(F);
            double *Gd = static_cast<double *>(G);
            // lag block L: the smallest built size that leaves no slot with two blocks
            const int want = static_cast<int>((n_tau + (kBlock >> rlpw) - 1) / (kBlock >> rlpw));
            const int L = want <= 4 ? 4 : want <= 7 ? 7 : kLagBlock;
            if (rlpw == 5) launch_isf_ring<5>(L, grid, lds, s, a2, F32, n_q, n_tau, P.rank, f2, Gd);
            else if (rlpw == 4) launch_isf_ring<4>(L, grid, lds, s, a2, F32, n_q, n_tau, P.rank, f2, Gd);
            else launch_isf_ring<3>(L, grid, lds, s, a2, F32, n_q, n_tau, P.rank, f2, Gd);
        } else if ((F << lpw) * static_cast<int64_t>(sizeof(double2)) <= 65536) {
            const size_t lds = sizeof(double2) * (F << lpw);
            const int64_t pw = int64_t(1) << lpw;
            hipLaunchKernelGGL(k_isf_lags, dim3(static_cast<unsigned>((n_q + pw - 1) / pw)), dim3(kBlock), lds, s,
                               a2, static_cast<int32_t>(F), n_q, n_tau, static_cast<int32_t>(lpw), P.rank, f2,
                               static_cast<double *>(G));
        } else {
            const int64_t n_lb = (n_tau + kLagBlock - 1) / kLagBlock;
            hipLaunchKernelGGL(k_isf_lags_global, dim3(blocks_for(n_q * n_lb)), dim3(kBlock), 0, s, a2, F, n_q,
                               n_tau, P.rank, f2, static_cast<double *>(G));
        }
        XS_HIP(hipGetLastError());
    }
    const double *top = reduce_tree(s, P, R, 0, n_q, ncol, static_cast<double *>(G), static_cast<double *>(G2));
    hipLaunchKernelGGL(k_ring_mean_finish, dim3(blocks_for(static_cast<int64_t>(R) * ncol)), dim3(kBlock), 0, s,
                       top, ncol, R, P.start, P.lev + static_cast<int64_t>(P.levels) * (R + 1), F_out, ring_count);
    tm.end(static_cast<double>(F) * n_q * sizeof(double2));
    XS_HIP(hipGetLastError());
    return XS_OK;
}

xs_status siegert(hipStream_t s, const double *g2, const double *F, int32_t R, int32_t n_tau, int32_t n_levels,
                  double *lhs, double *fhat2, double *beta) {
    const int64_t n = static_cast<int64_t>(R) * n_tau + static_cast<int64_t>(R) * n_levels;
    hipLaunchKernelGGL(k_siegert, dim3(blocks_for(n)), dim3(kBlock), 0, s, g2, F, R, n_tau, n_levels, lhs, fhat2,
                       beta);
    XS_HIP(hipGetLastError());
    return XS_OK;
}

xs_status xsvs_contrast(hipStream_t s, const double *I, int64_t F, int64_t n_q, const double *q,
                        const RingEdges &edges, int32_t n_levels, double *beta_out,
                        double *beta_win) {
    const int32_t R = edges.n_rings;
    TimerScope tm(s, TIMER_XSVS);
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
    Partition P;
    Arena cached{s};
    XS_TRY(partition(cached, k, n_q, R, &P));
    const int64_t rows = std::max<int64_t>(n_q, 1);  // bounds the pixels in rings
    const int64_t groups_bound = level_bound(n_q, R, 1) / kLvChunksPerBlock + R + 1;
    // launch order of the gathering blocks (groups by first pixel)
    const int64_t nb = (n_q + kPartChunk - 1) / kPartChunk;
    void *ord = nullptr;
    XS_TRY(scratch(s, SLOT_XSVS_ORDER, sizeof(int32_t) * (groups_bound + nb + 1), &ord));
    int32_t *order = static_cast<int32_t *>(ord), *gcnt = order + groups_bound;
    if (nb > 0) {
        hipLaunchKernelGGL(k_group_count, dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, k, P.rank, n_q, R,
                           P.start, P.grp, gcnt);
        hipLaunchKernelGGL(k_part_scan_ring, dim3(1), dim3(kBlock), 0, s, gcnt, nb, 1, gcnt + nb);
        hipLaunchKernelGGL(k_group_scatter, dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, k, P.rank, n_q,
                           R, P.start, P.grp, gcnt, order);
        XS_HIP(hipGetLastError());
    }
    const double *src = nullptr;
    // launch groups of kLvDepth levels; a group that does not reach the last
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
        const int64_t tiles = (K + kLvTile - 1) / kLvTile;
        const int64_t ncol = tiles * kLvCols;
        void *t1 = nullptr, *t2 = nullptr;
        // c1: the group nodes, later tree level 3; c2: level 2
        XS_TRY(scratch(s, SLOT_G, sizeof(double) * std::max(groups_bound, level_bound(n_q, R, 3)) * ncol, &t1));
        XS_TRY(scratch(s, SLOT_PIXEL2, sizeof(double) * level_bound(n_q, R, 2) * ncol, &t2));
        double *c1 = static_cast<double *>(t1), *c2 = static_cast<double *>(t2);
        LevelOut lo{};
        for (int32_t d = 0; d < depths; ++d) {
            lo.bwin[d] = bw + off[L + d];
            lo.K[d] = K >> d;
        }
        const dim3 grid(static_cast<unsigned>(groups_bound), static_cast<unsigned>(tiles));
        // one ring tree node per block group: then tree level 2 (1024 ring rows,
        // 8 group nodes) and on; with one level (rings of <= 32 pixels) the
        // group nodes are the tops
        const int32_t *top_off = P.levels >= 2 ? P.lev + static_cast<int64_t>(P.levels) * (R + 1) : P.grp;
        // one read of the windows: chunk trees of J and J*J, then the ring trees
        if (L == 0) {
            const int64_t blocks = 8 * ((groups_bound * tiles + 7) / 8);
            if (blocks > 0x7fffffff) return set_error(XS_EINVAL, "XSVS: %lld gathering blocks exceed one grid",
                                                     static_cast<long long>(blocks));
            hipLaunchKernelGGL(k_xsvs_chunks<true>, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s, I, K,
                               n_q, static_cast<const int32_t *>(P.list), R, P.start, P.grp,
                               static_cast<const int32_t *>(order), tiles, ncol, c1, dst);
        } else {
            hipLaunchKernelGGL(k_xsvs_chunks<false>, grid, dim3(kBlock), 0, s, src, K, n_q,
                               static_cast<const int32_t *>(nullptr), R, P.start, P.grp,
                               static_cast<const int32_t *>(nullptr), tiles, ncol, c1, dst);
        }
        XS_HIP(hipGetLastError());
        const double *top = c1;
        if (P.levels >= 2) {
            constexpr int kNodes = kGroup / kLvChunksPerBlock;
            hipLaunchKernelGGL(k_group_tree<kNodes>, dim3(blocks_for(level_bound(n_q, R, 2) * ncol)), dim3(kBlock),
                               0, s, c1, c2, ncol, P.grp, P.lev + static_cast<int64_t>(2) * (R + 1), R);
            top = reduce_tree(s, P, R, 2, n_q, ncol, c2, c1);
        }
        hipLaunchKernelGGL(k_xsvs_beta, dim3(blocks_for(static_cast<int64_t>(R) * (ncol / 2))), dim3(kBlock), 0, s,
                           top, ncol, K, depths, R, P.start, top_off, lo);
        XS_HIP(hipGetLastError());
        // mean over the windows of every level of the group, one launch
        if (R > 0)
            hipLaunchKernelGGL(k_xsvs_mean, dim3(static_cast<unsigned>(R), static_cast<unsigned>(depths)), dim3(kBlock),
                               0, s, lo, F, R, beta_out + static_cast<int64_t>(L) * R,
                               beta_win ? beta_win + static_cast<int64_t>(L) * F * R : nullptr);
        XS_HIP(hipGetLastError());
        src = dst;
        K >>= kLvDepth;
    }
    tm.end(static_cast<double>(F) * n_q * sizeof(double));
    return XS_OK;
}

xs_status frame_sums(hipStream_t s, const double *I, int64_t n_q, int64_t n_out, int64_t s_out, int64_t n_sum,
                     int64_t s_sum, double scale, double *J) {
    if (n_sum > (int64_t(1) << kSumMaxLog)) return set_error(XS_EINVAL, "n_sum must be <= 2^%d", kSumMaxLog);
    if (n_out * n_q > 0) {
        // counter levels: n_sum < 2^LV
        const int lv = n_sum < 64 ? 6 : n_sum < 4096 ? 12 : kSumMaxLog + 1;
        const bool pair = n_q % 2 == 0 && reinterpret_cast<uintptr_t>(I) % 16 == 0;
        const dim3 grid(blocks_for(n_out * (pair ? n_q / 2 : n_q)));
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, grid, dim3(kBlock), 0, s, I, n_q, n_out, s_out, n_sum, s_sum, scale, J);
        };
        if (pair) {
            if (lv == 6) go(k_frame_sums<2, 6, 2>);
            else if (lv == 12) go(k_frame_sums<2, 12, 2>);
            else go(k_frame_sums<2, kSumMaxLog + 1, 2>);
        } else {
            if (lv == 6) go(k_frame_sums<1, 6, 4>);
            else if (lv == 12) go(k_frame_sums<1, 12, 4>);
            else go(k_frame_sums<1, kSumMaxLog + 1, 4>);
        }
    }
    XS_HIP(hipGetLastError());
    return XS_OK;
}

xs_status ring_histogram(hipStream_t s, const double *I, int64_t F, int64_t n_q, const double *q,
                         const RingEdges &edges, int32_t n_bins, double kappa_max, int64_t *counts, double *mean) {
    const int32_t R = edges.n_rings;
    const int64_t nh = static_cast<int64_t>(R) * (n_bins + 1);
    if (nh * static_cast<int64_t>(sizeof(unsigned int)) > 65536)
        return set_error(XS_EINVAL, "n_rings * (n_bins + 1) must be <= 16384");
    void *key = nullptr, *X = nullptr, *X2 = nullptr, *mu = nullptr;
    XS_TRY(scratch(s, SLOT_RING_KEY, sizeof(int32_t) * std::max<int64_t>(n_q, 1), &key));
    XS_TRY(scratch(s, SLOT_G, sizeof(double) * std::max<int64_t>(n_q * F, 1), &X));
    XS_TRY(scratch(s, SLOT_LEVEL_B, sizeof(double) * level_bound(n_q, R, 1) * F, &X2));
    XS_TRY(scratch(s, SLOT_BWIN, sizeof(double) * 2 * std::max<int64_t>(F * R, 1), &mu));
    if (!mean) mean = static_cast<double *>(mu) + std::max<int64_t>(F * R, 1);  // [F][R] kept internally
    int32_t *k = static_cast<int32_t *>(key);
    if (n_q > 0) hipLaunchKernelGGL(k_ring_key, dim3(blocks_for(n_q)), dim3(kBlock), 0, s, q, n_q, edges, k);
    Partition P;
    Arena cached{s};
    XS_TRY(partition(cached, k, n_q, R, &P));
    if (n_q > 0)
        hipLaunchKernelGGL(k_ring_rows, dim3(static_cast<unsigned>((n_q + kRowTile - 1) / kRowTile),
                                             static_cast<unsigned>((F + kRowTile - 1) / kRowTile)),
                           dim3(kBlock), 0, s, I, F, n_q,
                           static_cast<const int32_t *>(P.list), static_cast<const int32_t *>(P.start), R,
                           static_cast<double *>(X));
    // ring means per frame: pairwise tree over the ring-ordered rows (columns = frames)
    const double *top = reduce_tree(s, P, R, 0, n_q, F, static_cast<double *>(X), static_cast<double *>(X2));
    double *m_rt = static_cast<double *>(mu);  // [R][F]
    hipLaunchKernelGGL(k_ring_mean_finish, dim3(blocks_for(static_cast<int64_t>(R) * F)), dim3(kBlock), 0, s, top,
                       F, R, P.start, P.lev + static_cast<int64_t>(P.levels) * (R + 1), m_rt,
                       static_cast<int32_t *>(nullptr));
    hipLaunchKernelGGL(k_transpose_rt, dim3(blocks_for(static_cast<int64_t>(R) * F)), dim3(kBlock), 0, s,
                       static_cast<const double *>(m_rt), static_cast<int64_t>(R), F, mean);
    hipLaunchKernelGGL(k_fill_u64, dim3(std::min<unsigned>(blocks_for(nh * F), 4096u)), dim3(kBlock), 0, s,
                       reinterpret_cast<unsigned long long *>(counts), nh * F);
    if (n_q > 0)
        hipLaunchKernelGGL(k_ring_hist, dim3(static_cast<unsigned>((n_q + kHistSpan - 1) / kHistSpan),
                                             static_cast<unsigned>(F)), dim3(kBlock),
                           sizeof(unsigned int) * nh, s, I, n_q, static_cast<const int32_t *>(k), R,
                           static_cast<const double *>(mean), n_bins, static_cast<double>(n_bins) / kappa_max,
                           reinterpret_cast<unsigned long long *>(counts));
    XS_HIP(hipGetLastError());
    return XS_OK;
}

}  // namespace xs
