// FP32 compensated (FP32C) form of the direct method and of its position
// gradient, for batches of systems and frames in one persistent launch.
//
// Sec. 3.1 (Algorithm 1): every pixel's amplitude is an independent sum over
// atoms, p^e(q) = sum_j f_j exp(-i q.r_j) (Eq. (pe_ri)), I = |p^e|^2 (Eq. (Iq_pq)).
// FP32 cannot hold the phase q.r/(2 pi) of a large box (hundreds of
// revolutions) to 1e-7 revolution, so the phase is split.  Atoms are sorted
// along a Hilbert curve and cut into tiles of 64 with FP64 origin o_k; pixels
// are sorted the same way in q-space and cut into compact groups with FP64
// centre q_c.  With d_j = r_j - o_k and dq_p = q_p - q_c (revolutions per
// Angstrom):
//   q_p.r_j = q_p.o_k + q_c.d_j + dq_p.d_j
//   theta(p,k) = frac(q_p.o_k)  FP64, once per (pixel, tile)
//   beta(j)    = frac(q_c.d_j)  FP64 from the exact offset, once per (atom, group)
//   dq_p.d_j   FP32, |.| < ~0.6 revolution
// so the FP32 part of every phase stays below ~2 revolutions and rounds at
// ~1e-7 revolution.  v_sin_f32 / v_cos_f32 take revolutions.  Tile partial
// sums run in FP32 and fold into FP64; chunk partials combine in fixed order.
//
// Pipeline of a call:
//   sort      atoms of every segment (system x frame) and pixels of every
//             system by 30-bit Hilbert index (deterministic radix sort);
//   tiles     64 consecutive sorted atoms, bounding-box centre as FP64
//             origin, FP32 offsets split hi + lo, FP32 form factor;
//   pair sum  persistent work queue over items, largest first;
//   combine   chunk partials summed in order, written in input pixel order.
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "xs_internal.h"

namespace xs {
namespace {

constexpr int kTile = 64;        // atoms per spatial tile (one wavefront)
constexpr int kBlock = 256;      // threads per workgroup (4 wavefronts)
constexpr int kWaves = kBlock / 64;
constexpr int kHilbertBits = 10;  // per dimension
constexpr double kInvTwoPi = 0x1.45f306dc9c883p-3;  // RN(1/(2 pi))
constexpr int kLatRuns = 8;                         // lattice item: runs across a row per lane row
constexpr int kLatRows = kBlock / kLatRuns;         // lattice item: rows (32)
constexpr double kLatTol = 1e-11;                   // lattice test: |q_p - model| bound, 1 / Angstrom
constexpr int kFwdCounters = 3;                     // work-queue counters of the forward forms
constexpr int kRotTiles = 2;                        // tiles sharing one origin and one rotation (forward)
// Items with a wavevector of |q| / (2 pi) below this (revolutions per Angstrom, i.e. |q| < 0.5
// per Angstrom) fold their FP32 sums into FP64 after every tile instead of every pair of
// tiles.  At small |q| the phases inside a tile vary little, so a tile's FP32 sum is nearly
// coherent (a sizable fraction of its atom count) while the amplitude left after the tiles
// cancel is small; the rounding of those long coherent FP32 sums then dominates the error.
constexpr double kSmallQRev = 0.08;

// ---------------------------------------------------------------- tables

struct BinSeg {            // tiling view of one segment (system x frame)
    int64_t pos;           // atom offset of the frame in pos
    int64_t f;             // offset into f
    int64_t atom0;         // offset of this segment's atoms in the key / index arrays
    int64_t cell0;         // offset of this segment's cells in the cell histogram
    int64_t tile0;         // first tile of this segment
    int32_t bits;          // Hilbert bits per dimension (2^bits cells per edge of the bounding box)
    int32_t n_atoms;
    int32_t n_tiles;
    int32_t pad;
};

struct PixSet {            // one distinct pixel set (a system's q)
    int64_t q;             // pixel offset into q
    int64_t slot0;         // offset of its pixels in the sorted order
    int32_t n_q;
    int32_t lattice;       // 1: row lattice with rows of whole 64-pixel groups, kept in input order
};

struct FwdSeg {            // pair-sum view of one segment
    int64_t q;             // pixel offset into q
    int64_t slot0;         // offset of the segment's pixel set in the sorted order
    int64_t out;           // pixel offset into outputs
    int64_t part;          // offset (pixels) of partials: chunk c at part + c*n_q
    int64_t tile0;
    int32_t n_q;
    int32_t n_tiles;
    int32_t n_chunks;
    int32_t n2;            // lattice form: pixels per row (0: general form)
    double a[3];           // lattice form: step between neighbours of a row (revolutions / A)
    int32_t n_jb;          // lattice and row forms: item rectangles across a row
    int32_t form;          // 0 general (sorted pixels), 1 lattice, 2 rows
};

struct LatSet {            // a pixel set that passed the row-lattice test
    int64_t q;
    int32_t n_q;
    int32_t n2;
    double a[3];           // row step, 1 / Angstrom
    int32_t flat;          // 1: every q_z of the set is 0
    int32_t pad;
};

struct RowSet {            // a pixel set stored as rows of n2 pixels sharing q_y exactly
    int64_t q;
    int32_t n_q;
    int32_t n2;
};

struct FwdItem {
    int32_t seg;
    int32_t p0;            // first sorted pixel slot of the item
    int32_t t0;            // first tile (relative to the segment)
    int32_t nt;            // tiles in this chunk
    int32_t chunk;
    int32_t pad;
};

struct GradSeg {
    int64_t q;             // pixel offset into q
    int64_t slot0;         // offset of the pixel set in the sorted order / prepared data
    int64_t out;           // pixel offset into amp / dL_dI
    int64_t pos;           // atom offset in pos (for outputs)
    int64_t f;             // offset into f
    int64_t tile0;
    int64_t part;          // offset (atom slots) of partials: chunk c at part + c*n_tiles*64
    int64_t grp0;          // first 64-pixel group of the pixel set in the centre table
    int32_t n_q;
    int32_t n_tiles;
    int32_t n_chunks;
    int32_t lat;           // 1: every 64-pixel group is a run along a lattice row
    double a[3];           // lattice row step (revolutions / A)
    int32_t mf;            // matrix-core lattice form: components (2 if every q_z is 0, else 3); 0: off
    int32_t n2;            // matrix-core form: pixels per row
    int32_t n_jb;          // matrix-core form: rectangles across a row
    int32_t pad;
};

struct GradItem {
    int32_t seg;
    int32_t t0;            // first tile of this group
    int32_t nt;            // tiles in the group (<= kWaves * AL)
    int32_t p0;            // first sorted pixel slot of the chunk (multiple of 64)
    int32_t np;            // pixels in the chunk
    int32_t chunk;
};

// ---------------------------------------------------------------- Hilbert index
// Skilling's transpose form of the Hilbert curve (J. Skilling, "Programming the
// Hilbert curve", AIP Conf. Proc. 707, 2004): undo excess work on the axes,
// Gray-encode, then interleave the transposed bits.  Consecutive indices are
// always face-adjacent cells, so a run of consecutive points is compact.
// bits in [1, 10].
__device__ __forceinline__ uint32_t hilbert3(uint32_t x0, uint32_t x1, uint32_t x2, int bits) {
    uint32_t X[3] = {x0, x1, x2};
    const uint32_t M = 1u << (bits - 1);
    for (uint32_t Q = M; Q > 1; Q >>= 1) {
        const uint32_t P = Q - 1;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                const uint32_t t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    X[1] ^= X[0];
    X[2] ^= X[1];
    uint32_t t = 0;
    for (uint32_t Q = M; Q > 1; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1;
    X[0] ^= t;
    X[1] ^= t;
    X[2] ^= t;
    uint32_t h = 0;
    for (int b = bits - 1; b >= 0; --b)
        h = (h << 3) | (((X[0] >> b) & 1u) << 2) | (((X[1] >> b) & 1u) << 1) | ((X[2] >> b) & 1u);
    return h;
}

__device__ __forceinline__ uint32_t cell_of(double x, double scale, int bits) {
    const double top = double((1 << bits) - 1);
    double c = __builtin_floor(x * scale);
    c = c < 0.0 ? 0.0 : (c > top ? top : c);
    if (!(c == c)) c = 0.0;  // NaN positions land in cell 0
    return static_cast<uint32_t>(c);
}

// ---------------------------------------------------------------- atom tiling
// Deterministic counting sort of every segment's atoms by Hilbert cell, built
// from plain kernels only (no memset or copy), so a captured graph can replay
// it: zero -> cell key + histogram -> exclusive scan (3 phases) -> scatter ->
// per-cell ascending index order -> tiles.

__global__ __launch_bounds__(kBlock) void k_zero_i32(int32_t *__restrict__ p, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kBlock)
        p[i] = 0;
}

// Bounding box of every segment's positions (and of every pixel set's q-vectors), in
// two passes: kBoxParts blocks per set reduce strided chunks (NaN coordinates are
// skipped by fmin / fmax), then one block per set folds their partials: box[6 s + c] =
// lo_c, box[6 s + 3 + c] = hi_c.  The cell grid spans this box, so positions anywhere
// (wrapped into the simulation cell or not) give compact cells and tiles.
constexpr int kBoxParts = 64;
__device__ __forceinline__ int64_t points_of(const BinSeg &s, int64_t &n) {
    n = s.n_atoms;
    return s.pos;
}
__device__ __forceinline__ int64_t points_of(const PixSet &s, int64_t &n) {
    n = s.n_q;
    return s.q;
}

template <typename Set>
__global__ __launch_bounds__(kBlock) void k_bbox_part(const Set *__restrict__ sets, const double *__restrict__ xyz,
                                                      double *__restrict__ part) {
    int64_t n = 0;
    const int64_t first = points_of(sets[blockIdx.y], n);
    __shared__ double s_lo[3][kBlock], s_hi[3][kBlock];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t j = blockIdx.x * kBlock + threadIdx.x; j < n; j += kBoxParts * kBlock) {
        const double *r = xyz + (first + j) * 3;
        for (int c = 0; c < 3; ++c) {
            lo[c] = fmin(lo[c], r[c]);
            hi[c] = fmax(hi[c], r[c]);
        }
    }
    for (int c = 0; c < 3; ++c) {
        s_lo[c][threadIdx.x] = lo[c];
        s_hi[c][threadIdx.x] = hi[c];
    }
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < static_cast<unsigned>(off))
            for (int c = 0; c < 3; ++c) {
                s_lo[c][threadIdx.x] = fmin(s_lo[c][threadIdx.x], s_lo[c][threadIdx.x + off]);
                s_hi[c][threadIdx.x] = fmax(s_hi[c][threadIdx.x], s_hi[c][threadIdx.x + off]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 3) {
        double *o = part + (static_cast<int64_t>(blockIdx.y) * kBoxParts + blockIdx.x) * 6;
        o[threadIdx.x] = s_lo[threadIdx.x][0];
        o[3 + threadIdx.x] = s_hi[threadIdx.x][0];
    }
}

__global__ __launch_bounds__(64) void k_bbox_fold(const double *__restrict__ part, double *__restrict__ box) {
    if (threadIdx.x >= 3) return;
    const int c = threadIdx.x;
    double l = INFINITY, h = -INFINITY;
    for (int b = 0; b < kBoxParts; ++b) {
        const double *o = part + (static_cast<int64_t>(blockIdx.x) * kBoxParts + b) * 6;
        l = fmin(l, o[c]);
        h = fmax(h, o[3 + c]);
    }
    const bool ok = l <= h;  // false for a set without finite coordinates
    box[6 * blockIdx.x + c] = ok ? l : 0.0;
    box[6 * blockIdx.x + 3 + c] = ok ? h : 0.0;
}

__global__ __launch_bounds__(kBlock) void k_cell_keys(const BinSeg *__restrict__ segs,
                                                      const double *__restrict__ pos,
                                                      const double *__restrict__ box,
                                                      uint32_t *__restrict__ keys,
                                                      int32_t *__restrict__ hist) {
    const BinSeg sg = segs[blockIdx.y];
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= sg.n_atoms) return;
    const double *r = pos + (sg.pos + j) * 3;
    const double *bx = box + 6 * blockIdx.y;
    double sc[3];
    for (int c = 0; c < 3; ++c) {
        const double span = bx[3 + c] - bx[c];
        sc[c] = span > 0.0 ? double(1 << sg.bits) / span : 0.0;
    }
    const uint32_t h = hilbert3(cell_of(r[0] - bx[0], sc[0], sg.bits), cell_of(r[1] - bx[1], sc[1], sg.bits),
                                cell_of(r[2] - bx[2], sc[2], sg.bits), sg.bits);
    keys[sg.atom0 + j] = h;
    atomicAdd(&hist[sg.cell0 + h], 1);
}

constexpr int kScanBlock = 1024;  // elements per scan block (256 threads x 4)

__global__ __launch_bounds__(kBlock) void k_scan_reduce(const int32_t *__restrict__ v, int64_t n,
                                                        int32_t *__restrict__ sums) {
    __shared__ int32_t s[kBlock];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanBlock;
    int32_t a = 0;
    for (int i = threadIdx.x; i < kScanBlock; i += kBlock)
        if (base + i < n) a += v[base + i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = s[0];
}

// Exclusive scan of the block sums in place (one block).
__global__ __launch_bounds__(1024) void k_scan_top(int32_t *__restrict__ sums, int64_t nb) {
    __shared__ int32_t s[1024];
    const int64_t per = (nb + 1023) / 1024;
    const int64_t a = threadIdx.x * per, b = a + per < nb ? a + per : nb;
    int32_t t = 0;
    for (int64_t i = a; i < b; ++i) t += sums[i];
    s[threadIdx.x] = t;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // inclusive Hillis-Steele
        const int32_t x = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += x;
        __syncthreads();
    }
    int32_t run = threadIdx.x > 0 ? s[threadIdx.x - 1] : 0;
    for (int64_t i = a; i < b; ++i) {
        const int32_t x = sums[i];
        sums[i] = run;
        run += x;
    }
}

// start[i] = exclusive prefix of v; cursor[i] = start[i].
__global__ __launch_bounds__(kBlock) void k_scan_down(const int32_t *__restrict__ v, int64_t n,
                                                      const int32_t *__restrict__ sums,
                                                      int32_t *__restrict__ start,
                                                      int32_t *__restrict__ cursor) {
    __shared__ int32_t s[kBlock];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanBlock + threadIdx.x * 4;
    int32_t x[4], t = 0;
    for (int k = 0; k < 4; ++k) {
        x[k] = base + k < n ? v[base + k] : 0;
        t += x[k];
    }
    s[threadIdx.x] = t;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        const int32_t y = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += y;
        __syncthreads();
    }
    int32_t run = sums[blockIdx.x] + (threadIdx.x > 0 ? s[threadIdx.x - 1] : 0);
    for (int k = 0; k < 4; ++k)
        if (base + k < n) {
            start[base + k] = run;
            cursor[base + k] = run;
            run += x[k];
        }
}

__global__ __launch_bounds__(kBlock) void k_cell_scatter(const BinSeg *__restrict__ segs,
                                                         const uint32_t *__restrict__ keys,
                                                         int32_t *__restrict__ cursor,
                                                         int32_t *__restrict__ sorted) {
    const BinSeg sg = segs[blockIdx.y];
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= sg.n_atoms) return;
    const int32_t slot = atomicAdd(&cursor[sg.cell0 + keys[sg.atom0 + j]], 1);
    sorted[slot] = j;
}

// Each cell's atoms in ascending index order (after the scatter, cursor[c]
// is the end of cell c): one thread per cell sorts a cell of up to kOrderSmall
// atoms by insertion; a larger cell (strongly clustered positions) is appended to
// big[1 ..] (big[0] counts them) for k_cell_order_big.
constexpr int kOrderSmall = 64;

__global__ __launch_bounds__(kBlock) void k_cell_order(const int32_t *__restrict__ start,
                                                       const int32_t *__restrict__ end, int64_t n,
                                                       int32_t *__restrict__ sorted, int32_t *__restrict__ big) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (c >= n) return;
    const int32_t a = start[c], b = end[c];
    if (b - a > kOrderSmall) {
        big[1 + atomicAdd(&big[0], 1)] = static_cast<int32_t>(c);
        return;
    }
    for (int32_t i = a + 1; i < b; ++i) {
        const int32_t x = sorted[i];
        int32_t k = i - 1;
        while (k >= a && sorted[k] > x) {
            sorted[k + 1] = sorted[k];
            --k;
        }
        sorted[k + 1] = x;
    }
}

// The large cells listed in big[]: a block per cell ranks the cell's atom indices
// with a bitmap over its segment's index range, in windows of kRankWords * 32
// indices.  Per window: bit x - w0 set for each atom x of the cell in the window,
// an exclusive scan of the words' popcounts, then atom x goes to the cell start +
// the cell's atoms in earlier windows + the set bits below it.  Linear in the
// cell's atoms times the windows plus the segment's atom count; the cell's
// unordered atoms are first copied to tmp (sorted[] is overwritten as they move).
constexpr int kRankWords = 4096;

__global__ __launch_bounds__(kBlock) void k_cell_order_big(const BinSeg *__restrict__ segs, int32_t n_seg,
                                                           const int32_t *__restrict__ start,
                                                           const int32_t *__restrict__ end,
                                                           const int32_t *__restrict__ big,
                                                           int32_t *__restrict__ tmp, int32_t *__restrict__ sorted) {
    constexpr int kPer = kRankWords / kBlock;
    constexpr int kSpan = kRankWords * 32;
    __shared__ uint32_t bits[kRankWords];
    __shared__ int32_t pre[kRankWords];
    __shared__ int32_t wsum[kBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t n_big = big[0];
    for (int32_t e = blockIdx.x; e < n_big; e += gridDim.x) {
        const int32_t c = big[1 + e];
        const int32_t a = start[c], b = end[c];
        int lo = 0, hi = n_seg;  // the segment of cell c: the last with cell0 <= c
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (segs[mid].cell0 <= c) lo = mid; else hi = mid;
        }
        const int32_t n_atoms = segs[lo].n_atoms;
        for (int32_t i = a + static_cast<int32_t>(threadIdx.x); i < b; i += kBlock) tmp[i] = sorted[i];
        __syncthreads();
        int32_t below = 0;  // the cell's atoms in earlier windows
        for (int32_t w0 = 0; w0 < n_atoms; w0 += kSpan) {
            for (int k = threadIdx.x; k < kRankWords; k += kBlock) bits[k] = 0u;
            __syncthreads();
            for (int32_t i = a + static_cast<int32_t>(threadIdx.x); i < b; i += kBlock) {
                const int32_t x = tmp[i] - w0;
                if (x >= 0 && x < kSpan) atomicOr(&bits[x >> 5], 1u << (x & 31));
            }
            __syncthreads();
            // exclusive scan of the popcounts: thread t takes words [kPer t, kPer t + kPer)
            int32_t own = 0;
            for (int k = 0; k < kPer; ++k) own += __builtin_popcount(bits[threadIdx.x * kPer + k]);
            int32_t inc = own;
            for (int off = 1; off < 64; off <<= 1) {
                const int32_t y = __shfl_up(inc, off);
                if (lane >= off) inc += y;
            }
            if (lane == 63) wsum[wave] = inc;
            __syncthreads();
            int32_t run = inc - own, total = 0;
            for (int w = 0; w < kBlock / 64; ++w) {
                if (w < wave) run += wsum[w];
                total += wsum[w];
            }
            for (int k = 0; k < kPer; ++k) {
                pre[threadIdx.x * kPer + k] = run;
                run += __builtin_popcount(bits[threadIdx.x * kPer + k]);
            }
            __syncthreads();
            for (int32_t i = a + static_cast<int32_t>(threadIdx.x); i < b; i += kBlock) {
                const int32_t x = tmp[i] - w0;
                if (x >= 0 && x < kSpan) {
                    const uint32_t below_x = bits[x >> 5] & ((1u << (x & 31)) - 1u);
                    sorted[a + below + pre[x >> 5] + __builtin_popcount(below_x)] = tmp[i];
                }
            }
            below += total;
            __syncthreads();  // bits, pre and wsum are rewritten by the next window
        }
    }
}

// Pixel sets: bounding box (one block per set), then 64-bit keys
// (set << 30 | Hilbert index of the q cell) for a radix sort.
__global__ __launch_bounds__(kBlock) void k_pix_keys(const PixSet *__restrict__ sets,
                                                     const double *__restrict__ q,
                                                     const double *__restrict__ bbox,
                                                     uint64_t *__restrict__ keys,
                                                     int32_t *__restrict__ vals) {
    const PixSet ps = sets[blockIdx.y];
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= ps.n_q) return;
    uint32_t c[3];
    for (int d = 0; d < 3; ++d) {
        const double lo = bbox[6 * blockIdx.y + d], hi = bbox[6 * blockIdx.y + 3 + d];
        const double span = hi - lo;
        const double scale = span > 0.0 ? double(1 << kHilbertBits) / (span * 1.000001) : 0.0;
        c[d] = cell_of(q[(ps.q + p) * 3 + d] - lo, scale, kHilbertBits);
    }
    const uint64_t h = ps.lattice ? static_cast<uint64_t>(p) : hilbert3(c[0], c[1], c[2], kHilbertBits);
    keys[ps.slot0 + p] = (static_cast<uint64_t>(blockIdx.y) << (3 * kHilbertBits)) | h;
    vals[ps.slot0 + p] = p;
}

// One wavefront per tile: bounding-box centre as FP64 origin; offsets in FP32
// as hi + lo (lo = residual of the FP64 offset); FP32 form factor; zero padding.
__global__ __launch_bounds__(kBlock) void k_make_tiles(const BinSeg *__restrict__ segs,
                                                       const double *__restrict__ pos,
                                                       const double *__restrict__ f,
                                                       const int32_t *__restrict__ sorted,
                                                       float4 *__restrict__ t_hi,
                                                       float4 *__restrict__ t_lo,
                                                       double4 *__restrict__ origins,
                                                       int32_t *__restrict__ tile_atom) {
    const BinSeg sg = segs[blockIdx.y];
    const int t = blockIdx.x * kWaves + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (t >= sg.n_tiles) return;
    const int slot = t * kTile + lane;
    const bool real = slot < sg.n_atoms;
    double r[3] = {0.0, 0.0, 0.0};
    int32_t j = -1;
    if (real) {
        j = sorted[sg.atom0 + slot];
        const double *rp = pos + (sg.pos + j) * 3;
        r[0] = rp[0];
        r[1] = rp[1];
        r[2] = rp[2];
    }
    double o[3];
    for (int d = 0; d < 3; ++d) {
        double lo = real ? r[d] : INFINITY, hi = real ? r[d] : -INFINITY;
        for (int off = 32; off > 0; off >>= 1) {
            lo = fmin(lo, __shfl_xor(lo, off));
            hi = fmax(hi, __shfl_xor(hi, off));
        }
        o[d] = 0.5 * (lo + hi);
    }
    const int64_t ti = sg.tile0 + t;
    float4 vh = make_float4(0.f, 0.f, 0.f, 0.f), vl = make_float4(0.f, 0.f, 0.f, 0.f);
    if (real) {
        const double d0 = r[0] - o[0], d1 = r[1] - o[1], d2 = r[2] - o[2];
        const float h0 = static_cast<float>(d0), h1 = static_cast<float>(d1), h2 = static_cast<float>(d2);
        vh = make_float4(h0, h1, h2, static_cast<float>(f[sg.f + j]));
        vl = make_float4(static_cast<float>(d0 - h0), static_cast<float>(d1 - h1),
                         static_cast<float>(d2 - h2), 0.f);
    }
    t_hi[ti * kTile + lane] = vh;
    t_lo[ti * kTile + lane] = vl;
    tile_atom[ti * kTile + lane] = j;
    // largest |f| of the tile (the scale of the matrix-core form's FP16 factors)
    float fmax = fabsf(vh.w);
    for (int off = 32; off > 0; off >>= 1) fmax = fmaxf(fmax, __shfl_xor(fmax, off));
    if (lane == 0) origins[ti] = make_double4(o[0], o[1], o[2], static_cast<double>(fmax));
}

__global__ void k_reset_counters(int32_t *counter, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) counter[i] = 0;
}

__device__ __forceinline__ float frac_f32(double t) { return static_cast<float>(t - __builtin_rint(t)); }

// ---------------------------------------------------------------- forward pair sum
//
// Workgroup = 4 wavefronts; the item's 256*QL pixels (consecutive in Hilbert
// order, so compact in q) share one centre q_c.  Lane owns QL pixels.  Atom
// tiles of the item's chunk are staged 4 at a time into LDS (double buffered)
// with their beta(j) = frac(q_c.d_j), and read back as broadcasts.
// Per pair the in-tile phase xi = beta + dq.d (2 FMA, or 3 when the item has
// dq_z != 0) feeds v_sin/v_cos and 2 FMA into the group sums
// (C, S) = sum_j f_j (cos, sin)(2 pi xi), over the 4 tiles of a staged group,
// whose offsets d are taken from one group origin O.  The base phase
// theta = frac(q_p.O) (FP64) enters once per (pixel, group) as a rotation,
// sum_j f_j e^{2 pi i (theta + xi)} = e^{2 pi i theta} (C + i S), whose result
// folds into FP64.
template <int QL, bool PLANAR>
__device__ __forceinline__ void tile_pairs(const float4 *__restrict__ at, const float *__restrict__ bt,
                                           const float (&dqx)[QL], const float (&dqy)[QL],
                                           const float (&dqz)[QL], float (&cs)[QL], float (&sn)[QL]) {
    // two atoms at a time: phases, then sines and cosines, then sums (atom j before
    // atom j + 1), the transcendentals back to back
    constexpr int kA = 2;
#pragma unroll 2
    for (int j = 0; j < kTile; j += kA) {
        float4 a[kA];
        float ph[kA][QL], c[kA][QL], s[kA][QL];
#pragma unroll
        for (int u = 0; u < kA; ++u) {
            a[u] = at[j + u];
            const float b = bt[j + u];
#pragma unroll
            for (int k = 0; k < QL; ++k) {
                ph[u][k] = __builtin_fmaf(dqx[k], a[u].x, b);
                ph[u][k] = __builtin_fmaf(dqy[k], a[u].y, ph[u][k]);
                if (!PLANAR) ph[u][k] = __builtin_fmaf(dqz[k], a[u].z, ph[u][k]);
            }
        }
#pragma unroll
        for (int u = 0; u < kA; ++u)
#pragma unroll
            for (int k = 0; k < QL; ++k) {
                c[u][k] = __builtin_amdgcn_cosf(ph[u][k]);
                s[u][k] = __builtin_amdgcn_sinf(ph[u][k]);
            }
#pragma unroll
        for (int u = 0; u < kA; ++u)
#pragma unroll
            for (int k = 0; k < QL; ++k) {
                cs[k] = __builtin_fmaf(a[u].w, c[u][k], cs[k]);
                sn[k] = __builtin_fmaf(a[u].w, s[u][k], sn[k]);
            }
    }
}

template <int QL, int OCC>
__global__ __launch_bounds__(kBlock, OCC) void k_forward_fp32c(
    const FwdItem *__restrict__ items, int32_t n_items, int32_t *__restrict__ counter,
    const FwdSeg *__restrict__ segs, const double *__restrict__ q,
    const int32_t *__restrict__ pix_order, const float4 *__restrict__ t_hi,
    const float4 *__restrict__ t_lo, const double4 *__restrict__ origins,
    double2 *__restrict__ partial) {
    __shared__ float4 s_atoms[2][kWaves * kTile];
    __shared__ float s_beta[2][kWaves * kTile];
    __shared__ double4 s_orig[2][kWaves];
    __shared__ double s_q[3][QL][kBlock];  // item pixels, revolutions per Angstrom (FP64)
    __shared__ double s_red[6][kWaves];
    __shared__ int32_t s_item;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int32_t it = s_item;
        __syncthreads();  // everyone has read s_item before it is rewritten
        if (it >= n_items) break;
        const FwdItem item = items[it];
        const FwdSeg sg = segs[item.seg];
        // lane pixels: sorted slots p0 + k*256 + tid
        int32_t orig[QL];
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
#pragma unroll
        for (int k = 0; k < QL; ++k) {
            const int sp = item.p0 + k * kBlock + tid;
            const bool real = sp < sg.n_q;
            const int p = pix_order[sg.slot0 + (real ? sp : sg.n_q - 1)];
            orig[k] = real ? p : -1;
            const double *qp = q + (sg.q + p) * 3;
            for (int c = 0; c < 3; ++c) {
                const double v = qp[c] * kInvTwoPi;
                s_q[c][k][tid] = v;
                if (real) {
                    lo[c] = fmin(lo[c], v);
                    hi[c] = fmax(hi[c], v);
                }
            }
        }
        // item centre q_c: bounding-box centre (wavefront then block reduction)
        for (int c = 0; c < 3; ++c)
            for (int off = 32; off > 0; off >>= 1) {
                lo[c] = fmin(lo[c], __shfl_xor(lo[c], off));
                hi[c] = fmax(hi[c], __shfl_xor(hi[c], off));
            }
        if (lane == 0)
            for (int c = 0; c < 3; ++c) {
                s_red[c][wave] = lo[c];
                s_red[3 + c][wave] = hi[c];
            }
        __syncthreads();
        double cen[3];
        bool planar;
        bool fold_each;  // fold the FP32 sums after every tile (small |q|)
        {
            double l3[3], h3[3];
            for (int c = 0; c < 3; ++c) {
                l3[c] = s_red[c][0];
                h3[c] = s_red[3 + c][0];
                for (int w = 1; w < kWaves; ++w) {
                    l3[c] = fmin(l3[c], s_red[c][w]);
                    h3[c] = fmax(h3[c], s_red[3 + c][w]);
                }
                cen[c] = 0.5 * (l3[c] + h3[c]);
            }
            planar = l3[2] == h3[2];  // dq_z = 0 for every pixel of the item
            double qn2 = 0.0;  // squared distance of the item's q box from q = 0
            for (int c = 0; c < 3; ++c) {
                const double m = (l3[c] <= 0.0 && h3[c] >= 0.0) ? 0.0 : fmin(fabs(l3[c]), fabs(h3[c]));
                qn2 = __builtin_fma(m, m, qn2);
            }
            fold_each = qn2 < kSmallQRev * kSmallQRev;
        }
        float dqx[QL], dqy[QL], dqz[QL];
        double re64[QL], im64[QL];
#pragma unroll
        for (int k = 0; k < QL; ++k) {
            dqx[k] = static_cast<float>(s_q[0][k][tid] - cen[0]);
            dqy[k] = static_cast<float>(s_q[1][k][tid] - cen[1]);
            dqz[k] = static_cast<float>(s_q[2][k][tid] - cen[2]);
            re64[k] = 0.0;
            im64[k] = 0.0;
        }
        const int64_t tbase = sg.tile0 + item.t0;
        const int n_groups = (item.nt + kWaves - 1) / kWaves;
        // The kWaves tiles of a staged group share one origin O (the midpoint of their
        // origins' bounding box): atom offsets are re-expressed as d' = (r - o_k) + (o_k - O)
        // in FP64, and one rotation by theta = frac(q_p.O) per (pixel, group) replaces one
        // per (pixel, tile).
        auto group_origin = [&](int g) {  // shared origin of the pair of tiles g (item-relative)
            double lo3[3] = {INFINITY, INFINITY, INFINITY}, hi3[3] = {-INFINITY, -INFINITY, -INFINITY};
            const int n_here = min(kRotTiles, item.nt - g * kRotTiles);
            for (int w = 0; w < n_here; ++w) {
                const double4 o = origins[tbase + g * kRotTiles + w];
                lo3[0] = fmin(lo3[0], o.x); hi3[0] = fmax(hi3[0], o.x);
                lo3[1] = fmin(lo3[1], o.y); hi3[1] = fmax(hi3[1], o.y);
                lo3[2] = fmin(lo3[2], o.z); hi3[2] = fmax(hi3[2], o.z);
            }
            return make_double4(0.5 * (lo3[0] + hi3[0]), 0.5 * (lo3[1] + hi3[1]), 0.5 * (lo3[2] + hi3[2]), 0.0);
        };
        // atom of tile tt (relative to the item), offset from the group origin O
        auto stage = [&](const float4 h, const float4 l, const double4 ot, const double4 O, int buf) {
            const double dx = (double(h.x) + double(l.x)) + (ot.x - O.x);
            const double dy = (double(h.y) + double(l.y)) + (ot.y - O.y);
            const double dz = (double(h.z) + double(l.z)) + (ot.z - O.z);
            const double b = __builtin_fma(cen[2], dz, __builtin_fma(cen[1], dy, cen[0] * dx));
            s_atoms[buf][tid] = make_float4(static_cast<float>(dx), static_cast<float>(dy), static_cast<float>(dz), h.w);
            s_beta[buf][tid] = frac_f32(b);
        };
        // stage group 0
        {
            const int tt = tid / kTile;
            const double4 O = group_origin(tt / kRotTiles);
            if (tt < item.nt) {
                const int64_t ai = (tbase + tt) * kTile + (tid & (kTile - 1));
                stage(t_hi[ai], t_lo[ai], origins[tbase + tt], O, 0);
            }
            if ((tid & (kRotTiles * kTile - 1)) == 0) s_orig[0][tid / (kRotTiles * kTile)] = O;
        }
        __syncthreads();
        for (int g = 0; g < n_groups; ++g) {
            const int buf = g & 1;
            // fetch the next group into registers; stored after this group's work
            float4 nh = make_float4(0.f, 0.f, 0.f, 0.f), nl = nh;
            double4 no = make_double4(0.0, 0.0, 0.0, 0.0), nO = no;
            const int ng = g + 1;
            const bool have_next = ng < n_groups;
            bool next_real = false;
            if (have_next) {
                const int tt = ng * kWaves + tid / kTile;
                next_real = tt < item.nt;
                if (next_real) {
                    const int64_t ai = (tbase + tt) * kTile + (tid & (kTile - 1));
                    nh = t_hi[ai];
                    nl = t_lo[ai];
                    no = origins[tbase + tt];
                }
                nO = group_origin(tt / kRotTiles);
            }
            const int tiles_here = min(kWaves, item.nt - g * kWaves);
            for (int w0 = 0; w0 < tiles_here; w0 += kRotTiles) {
                const int w1 = min(w0 + kRotTiles, tiles_here);
                const double4 o = s_orig[buf][w0 / kRotTiles];
                float cs[QL], sn[QL];
                for (int w = w0; w < w1; ++w) {
                    if (w == w0 || fold_each) {
#pragma unroll
                        for (int k = 0; k < QL; ++k) cs[k] = sn[k] = 0.f;
                    }
                    const float4 *at = &s_atoms[buf][w * kTile];
                    const float *bt = &s_beta[buf][w * kTile];
                    if (planar) tile_pairs<QL, true>(at, bt, dqx, dqy, dqz, cs, sn);
                    else tile_pairs<QL, false>(at, bt, dqx, dqy, dqz, cs, sn);
                    if (w + 1 < w1 && !fold_each) continue;
#pragma unroll
                    for (int k = 0; k < QL; ++k) {
                        const float th = frac_f32(__builtin_fma(s_q[2][k][tid], o.z,
                                                  __builtin_fma(s_q[1][k][tid], o.y, s_q[0][k][tid] * o.x)));
                        const float ct = __builtin_amdgcn_cosf(th), st = __builtin_amdgcn_sinf(th);
                        re64[k] += static_cast<double>(__builtin_fmaf(ct, cs[k], -st * sn[k]));
                        im64[k] += static_cast<double>(__builtin_fmaf(st, cs[k], ct * sn[k]));
                    }
                }
            }
            if (have_next) {
                if (next_real) stage(nh, nl, no, nO, buf ^ 1);
                if ((tid & (kRotTiles * kTile - 1)) == 0) s_orig[buf ^ 1][tid / (kRotTiles * kTile)] = nO;
            }
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < QL; ++k)
            if (orig[k] >= 0)
                partial[sg.part + static_cast<int64_t>(item.chunk) * sg.n_q + orig[k]] =
                    make_double2(re64[k], im64[k]);
    }
}

// ---------------------------------------------------------------- forward, row form
//
// Pixels of a detector stored row by row: every run of n2 consecutive pixels
// shares q_y exactly (planar grids and the Ewald-sphere detectors alike).  An
// item is a rectangle of kRowRows rows x kRowRuns runs of QL pixels; lane
// (row, run) owns QL consecutive pixels of one row, so its dq_y is one value
// and the part of the in-tile phase common to its pixels is formed once per
// (lane, atom):
//   Y_j = beta_j + dq_y d_y,j,    xi_pj = Y_j + dq_x,p d_x,j (+ dq_z,p d_z,j).
// Every pair still takes v_sin and v_cos of its own phase xi_pj (1 FMA of phase
// per pair on a q_z = 0 grid, 2 on a curved detector, 2 FMA of sums).  Atom
// offsets, group origins and the rotation by frac(q_p.O) per (pixel, group)
// are those of the general form.
constexpr int kRowRuns = 8;                  // runs across a row per lane row
constexpr int kRowRows = kBlock / kRowRuns;  // rows per item (32)

template <int QL, bool FLAT>
__device__ __forceinline__ void row_pairs(const float4 *__restrict__ at, const float *__restrict__ bt,
                                          const float dqy, const float (&dqx)[QL], const float (&dqz)[QL],
                                          float (&cs)[QL], float (&sn)[QL]) {
    // two atoms at a time: both atoms' phases, then their sines and cosines, then the
    // sums (atom j before atom j + 1, as one at a time): the transcendentals run back to
    // back instead of each feeding the next FMA
    constexpr int kA = 2;
#pragma unroll 2
    for (int j = 0; j < kTile; j += kA) {
        float4 a[kA];
        float ph[kA][QL], c[kA][QL], s[kA][QL];
#pragma unroll
        for (int u = 0; u < kA; ++u) {
            a[u] = at[j + u];
            const float y = __builtin_fmaf(dqy, a[u].y, bt[j + u]);
#pragma unroll
            for (int k = 0; k < QL; ++k) {
                ph[u][k] = __builtin_fmaf(dqx[k], a[u].x, y);
                if (!FLAT) ph[u][k] = __builtin_fmaf(dqz[k], a[u].z, ph[u][k]);
            }
        }
#pragma unroll
        for (int u = 0; u < kA; ++u)
#pragma unroll
            for (int k = 0; k < QL; ++k) {
                c[u][k] = __builtin_amdgcn_cosf(ph[u][k]);
                s[u][k] = __builtin_amdgcn_sinf(ph[u][k]);
            }
#pragma unroll
        for (int u = 0; u < kA; ++u)
#pragma unroll
            for (int k = 0; k < QL; ++k) {
                cs[k] = __builtin_fmaf(a[u].w, c[u][k], cs[k]);
                sn[k] = __builtin_fmaf(a[u].w, s[u][k], sn[k]);
            }
    }
}

template <int QL, int OCC>
__global__ __launch_bounds__(kBlock, OCC) void k_forward_rows(
    const FwdItem *__restrict__ items, int32_t n_items, int32_t *__restrict__ counter,
    const FwdSeg *__restrict__ segs, const double *__restrict__ q, const float4 *__restrict__ t_hi,
    const float4 *__restrict__ t_lo, const double4 *__restrict__ origins, double2 *__restrict__ partial) {
    __shared__ float4 s_atoms[2][kWaves * kTile];
    __shared__ float s_beta[2][kWaves * kTile];
    __shared__ double4 s_orig[2][kWaves / kRotTiles];
    __shared__ double s_q[2][QL][kBlock];  // q_x and q_z of the lane's pixels, revolutions per Angstrom
    __shared__ double s_red[6][kWaves];
    __shared__ int32_t s_item;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int32_t it = s_item;
        __syncthreads();  // everyone has read s_item before it is rewritten
        if (it >= n_items) break;
        const FwdItem item = items[it];
        const FwdSeg sg = segs[item.seg];
        const int n1 = sg.n_q / sg.n2;
        const int ib = item.p0 / sg.n_jb, jb = item.p0 - ib * sg.n_jb;
        const int row = ib * kRowRows + tid / kRowRuns;
        const int col0 = jb * kRowRuns * QL + (tid % kRowRuns) * QL;
        const bool active = row < n1 && col0 < sg.n2;
        const int nk = active ? min(QL, sg.n2 - col0) : 0;
        const int64_t p0 = active ? static_cast<int64_t>(row) * sg.n2 + col0 : 0;
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        double qy = 0.0;
#pragma unroll
        for (int k = 0; k < QL; ++k) {
            const bool real = k < nk;
            const double *qp = q + (sg.q + p0 + (real ? k : 0)) * 3;
            const double vx = qp[0] * kInvTwoPi, vy = qp[1] * kInvTwoPi, vz = qp[2] * kInvTwoPi;
            s_q[0][k][tid] = vx;
            s_q[1][k][tid] = vz;
            if (k == 0) qy = vy;
            if (real) {
                lo[0] = fmin(lo[0], vx); hi[0] = fmax(hi[0], vx);
                lo[1] = fmin(lo[1], vy); hi[1] = fmax(hi[1], vy);
                lo[2] = fmin(lo[2], vz); hi[2] = fmax(hi[2], vz);
            }
        }
        // item centre q_c: bounding-box centre (wavefront then block reduction)
        for (int c = 0; c < 3; ++c)
            for (int off = 32; off > 0; off >>= 1) {
                lo[c] = fmin(lo[c], __shfl_xor(lo[c], off));
                hi[c] = fmax(hi[c], __shfl_xor(hi[c], off));
            }
        if (lane == 0)
            for (int c = 0; c < 3; ++c) {
                s_red[c][wave] = lo[c];
                s_red[3 + c][wave] = hi[c];
            }
        __syncthreads();
        double cen[3];
        bool flat;
        bool fold_each;  // fold the FP32 sums after every tile (small |q|)
        {
            double l3[3], h3[3];
            for (int c = 0; c < 3; ++c) {
                l3[c] = s_red[c][0];
                h3[c] = s_red[3 + c][0];
                for (int w = 1; w < kWaves; ++w) {
                    l3[c] = fmin(l3[c], s_red[c][w]);
                    h3[c] = fmax(h3[c], s_red[3 + c][w]);
                }
                cen[c] = 0.5 * (l3[c] + h3[c]);
            }
            flat = l3[2] == h3[2];  // dq_z = 0 for every pixel of the item
            double qn2 = 0.0;  // squared distance of the item's q box from q = 0
            for (int c = 0; c < 3; ++c) {
                const double m = (l3[c] <= 0.0 && h3[c] >= 0.0) ? 0.0 : fmin(fabs(l3[c]), fabs(h3[c]));
                qn2 = __builtin_fma(m, m, qn2);
            }
            fold_each = qn2 < kSmallQRev * kSmallQRev;
        }
        const float dqy = static_cast<float>(qy - cen[1]);
        float dqx[QL], dqz[QL];
        double re64[QL], im64[QL];
#pragma unroll
        for (int k = 0; k < QL; ++k) {
            dqx[k] = static_cast<float>(s_q[0][k][tid] - cen[0]);
            dqz[k] = static_cast<float>(s_q[1][k][tid] - cen[2]);
            re64[k] = 0.0;
            im64[k] = 0.0;
        }
        const int64_t tbase = sg.tile0 + item.t0;
        const int n_groups = (item.nt + kWaves - 1) / kWaves;
        auto group_origin = [&](int g) {  // shared origin of the pair of tiles g (item-relative)
            double lo3[3] = {INFINITY, INFINITY, INFINITY}, hi3[3] = {-INFINITY, -INFINITY, -INFINITY};
            const int n_here = min(kRotTiles, item.nt - g * kRotTiles);
            for (int w = 0; w < n_here; ++w) {
                const double4 o = origins[tbase + g * kRotTiles + w];
                lo3[0] = fmin(lo3[0], o.x); hi3[0] = fmax(hi3[0], o.x);
                lo3[1] = fmin(lo3[1], o.y); hi3[1] = fmax(hi3[1], o.y);
                lo3[2] = fmin(lo3[2], o.z); hi3[2] = fmax(hi3[2], o.z);
            }
            return make_double4(0.5 * (lo3[0] + hi3[0]), 0.5 * (lo3[1] + hi3[1]), 0.5 * (lo3[2] + hi3[2]), 0.0);
        };
        auto stage = [&](const float4 h, const float4 l, const double4 ot, const double4 O, int buf) {
            const double dx = (double(h.x) + double(l.x)) + (ot.x - O.x);
            const double dy = (double(h.y) + double(l.y)) + (ot.y - O.y);
            const double dz = (double(h.z) + double(l.z)) + (ot.z - O.z);
            const double b = __builtin_fma(cen[2], dz, __builtin_fma(cen[1], dy, cen[0] * dx));
            s_atoms[buf][tid] = make_float4(static_cast<float>(dx), static_cast<float>(dy), static_cast<float>(dz), h.w);
            s_beta[buf][tid] = frac_f32(b);
        };
        {
            const int tt = tid / kTile;
            const double4 O = group_origin(tt / kRotTiles);
            if (tt < item.nt) {
                const int64_t ai = (tbase + tt) * kTile + (tid & (kTile - 1));
                stage(t_hi[ai], t_lo[ai], origins[tbase + tt], O, 0);
            }
            if ((tid & (kRotTiles * kTile - 1)) == 0) s_orig[0][tid / (kRotTiles * kTile)] = O;
        }
        __syncthreads();
        for (int g = 0; g < n_groups; ++g) {
            const int buf = g & 1;
            float4 nh = make_float4(0.f, 0.f, 0.f, 0.f), nl = nh;
            double4 no = make_double4(0.0, 0.0, 0.0, 0.0), nO = no;
            const int ng = g + 1;
            const bool have_next = ng < n_groups;
            bool next_real = false;
            if (have_next) {
                const int tt = ng * kWaves + tid / kTile;
                next_real = tt < item.nt;
                if (next_real) {
                    const int64_t ai = (tbase + tt) * kTile + (tid & (kTile - 1));
                    nh = t_hi[ai];
                    nl = t_lo[ai];
                    no = origins[tbase + tt];
                }
                nO = group_origin(tt / kRotTiles);
            }
            const int tiles_here = min(kWaves, item.nt - g * kWaves);
            for (int w0 = 0; w0 < tiles_here; w0 += kRotTiles) {
                const int w1 = min(w0 + kRotTiles, tiles_here);
                const double4 o = s_orig[buf][w0 / kRotTiles];
                float cs[QL], sn[QL];
                for (int w = w0; w < w1; ++w) {
                    if (w == w0 || fold_each) {
#pragma unroll
                        for (int k = 0; k < QL; ++k) cs[k] = sn[k] = 0.f;
                    }
                    const float4 *at = &s_atoms[buf][w * kTile];
                    const float *bt = &s_beta[buf][w * kTile];
                    if (flat) row_pairs<QL, true>(at, bt, dqy, dqx, dqz, cs, sn);
                    else row_pairs<QL, false>(at, bt, dqy, dqx, dqz, cs, sn);
                    if (w + 1 < w1 && !fold_each) continue;
                    const double yo = qy * o.y;
#pragma unroll
                    for (int k = 0; k < QL; ++k) {
                        const float th =
                            frac_f32(__builtin_fma(s_q[1][k][tid], o.z, __builtin_fma(s_q[0][k][tid], o.x, yo)));
                        const float ct = __builtin_amdgcn_cosf(th), st = __builtin_amdgcn_sinf(th);
                        re64[k] += static_cast<double>(__builtin_fmaf(ct, cs[k], -st * sn[k]));
                        im64[k] += static_cast<double>(__builtin_fmaf(st, cs[k], ct * sn[k]));
                    }
                }
            }
            if (have_next) {
                if (next_real) stage(nh, nl, no, nO, buf ^ 1);
                if ((tid & (kRotTiles * kTile - 1)) == 0) s_orig[buf ^ 1][tid / (kRotTiles * kTile)] = nO;
            }
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < QL; ++k)
            if (k < nk)
                partial[sg.part + static_cast<int64_t>(item.chunk) * sg.n_q + p0 + k] = make_double2(re64[k], im64[k]);
    }
}

// ---------------------------------------------------------------- forward, lattice form
//
// Pixels of the segment come in rows of n2 consecutive q-vectors stepping by a
// common vector a.  An item is a rectangle of kLatRows rows x kLatRuns runs;
// lane (row, run) owns the QL pixels p0 + k (k < QL) of its run, with
// q_{p0+k} = q_{p0} + k a.  The in-tile phase of pixel k is
// beta_j + dq_0.d_j + k a.d_j, so
//   sum_j f_j e^{2 pi i (beta_j + dq_0.d_j + k a.d_j)} = sum_j z_j g_jk,
//   z_j = e^{2 pi i (beta_j + dq_0.d_j)}  (one v_sin + v_cos per lane and atom),
//   g_jk = f_j e^{2 pi i k a.d_j}          (per atom, formed once per staged tile).
// Per pair (k >= 1) that is 4 FMA of a complex multiply-add instead of a
// v_sin/v_cos pair; every g_jk comes from its own sincos, so the error does not
// grow with k.  Base phases theta_k = frac(q_{p0}.o + k a.o) (FP64) rotate the
// tile sums as in the general form.
// LDS per staged atom: float2 (d_x, d_y), float d_z and QL/2 float4 holding
// g_1 .. g_{QL-1} (re, im), beta and f in the last slot (40 KB per block at
// QL = 8 with two buffers, so four blocks share a CU).
template <int QL>
__device__ __forceinline__ void lattice_atom_factors(const float4 &h, float e, float beta, float4 *dst) {
    float g[2 * QL];
#pragma unroll
    for (int k = 1; k < QL; ++k) {
        const float ang = static_cast<float>(k) * e;
        g[2 * k] = h.w * __builtin_amdgcn_cosf(ang);
        g[2 * k + 1] = h.w * __builtin_amdgcn_sinf(ang);
    }
    g[0] = beta;
    g[1] = 0.f;
#pragma unroll
    for (int v = 0; v < QL / 2; ++v) {
        // slot v: g_{2v+1}, g_{2v+2}; the last slot: g_{QL-1}, beta, f
        const int k1 = 2 * v + 1, k2 = 2 * v + 2;
        if (k2 < QL) dst[v] = make_float4(g[2 * k1], g[2 * k1 + 1], g[2 * k2], g[2 * k2 + 1]);
        else dst[v] = make_float4(g[2 * k1], g[2 * k1 + 1], g[0], h.w);
    }
}

template <int QL, bool PLANAR>
__device__ __forceinline__ void lattice_tile(const float2 *__restrict__ axy, const float *__restrict__ az,
                                             const float4 *__restrict__ gt, float dqx, float dqy, float dqz,
                                             float (&cs)[QL], float (&sn)[QL]) {
    constexpr int NV = QL / 2;
#pragma unroll 2
    for (int j = 0; j < kTile; ++j) {
        const float2 a = axy[j];
        float4 g[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) g[v] = gt[j * NV + v];
        const float beta = g[NV - 1].z, fw = g[NV - 1].w;
        float ph = __builtin_fmaf(dqx, a.x, beta);
        ph = __builtin_fmaf(dqy, a.y, ph);
        if (!PLANAR) ph = __builtin_fmaf(dqz, az[j], ph);
        const float zc = __builtin_amdgcn_cosf(ph), zs = __builtin_amdgcn_sinf(ph);
        cs[0] = __builtin_fmaf(fw, zc, cs[0]);
        sn[0] = __builtin_fmaf(fw, zs, sn[0]);
#pragma unroll
        for (int k = 1; k < QL; ++k) {
            const float4 &gv = g[(k - 1) / 2];
            const float gr = ((k - 1) & 1) ? gv.z : gv.x;
            const float gi = ((k - 1) & 1) ? gv.w : gv.y;
            cs[k] = __builtin_fmaf(zc, gr, cs[k]);
            cs[k] = __builtin_fmaf(-zs, gi, cs[k]);
            sn[k] = __builtin_fmaf(zc, gi, sn[k]);
            sn[k] = __builtin_fmaf(zs, gr, sn[k]);
        }
    }
}

template <int QL, int OCC>
__global__ __launch_bounds__(kBlock, OCC) void k_forward_lattice(
    const FwdItem *__restrict__ items, int32_t n_items, int32_t *__restrict__ counter,
    const FwdSeg *__restrict__ segs, const double *__restrict__ q, const float4 *__restrict__ t_hi,
    const float4 *__restrict__ t_lo, const double4 *__restrict__ origins, double2 *__restrict__ partial) {
    static_assert(QL % 2 == 0, "runs of an even number of pixels");
    constexpr int NV = QL / 2;
    __shared__ float2 s_xy[2][kWaves * kTile];
    __shared__ float s_z[2][kWaves * kTile];
    __shared__ float4 s_g[2][kWaves * kTile * NV];
    __shared__ double4 s_orig[2][kWaves];
    __shared__ double s_red[6][kWaves];
    __shared__ int32_t s_item;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int32_t it = s_item;
        __syncthreads();
        if (it >= n_items) break;
        const FwdItem item = items[it];
        const FwdSeg sg = segs[item.seg];
        const int n1 = sg.n_q / sg.n2;
        const int ib = item.p0 / sg.n_jb, jb = item.p0 - ib * sg.n_jb;
        const int row = ib * kLatRows + tid / kLatRuns;
        const int col0 = jb * kLatRuns * QL + (tid % kLatRuns) * QL;
        const bool active = row < n1 && col0 < sg.n2;
        const int nk = active ? min(QL, sg.n2 - col0) : 0;
        const int p0 = active ? row * sg.n2 + col0 : 0;
        const double ax = sg.a[0], ay = sg.a[1], az = sg.a[2];
        double q0[3];
        for (int c = 0; c < 3; ++c) q0[c] = q[(sg.q + p0) * 3 + c] * kInvTwoPi;
        // item centre: bounding box of the run ends (wavefront then block reduction)
        double lo[3], hi[3];
        {
            const double e[3] = {ax, ay, az};
            for (int c = 0; c < 3; ++c) {
                const double v0 = q0[c], v1 = __builtin_fma(static_cast<double>(nk > 0 ? nk - 1 : 0), e[c], q0[c]);
                lo[c] = active ? fmin(v0, v1) : INFINITY;
                hi[c] = active ? fmax(v0, v1) : -INFINITY;
            }
        }
        for (int c = 0; c < 3; ++c)
            for (int off = 32; off > 0; off >>= 1) {
                lo[c] = fmin(lo[c], __shfl_xor(lo[c], off));
                hi[c] = fmax(hi[c], __shfl_xor(hi[c], off));
            }
        if (lane == 0)
            for (int c = 0; c < 3; ++c) {
                s_red[c][wave] = lo[c];
                s_red[3 + c][wave] = hi[c];
            }
        __syncthreads();
        double cen[3];
        bool planar;
        {
            double l3[3], h3[3];
            for (int c = 0; c < 3; ++c) {
                l3[c] = s_red[c][0];
                h3[c] = s_red[3 + c][0];
                for (int w = 1; w < kWaves; ++w) {
                    l3[c] = fmin(l3[c], s_red[c][w]);
                    h3[c] = fmax(h3[c], s_red[3 + c][w]);
                }
                cen[c] = 0.5 * (l3[c] + h3[c]);
            }
            planar = l3[2] == h3[2];
        }
        const float dqx = static_cast<float>(q0[0] - cen[0]);
        const float dqy = static_cast<float>(q0[1] - cen[1]);
        const float dqz = static_cast<float>(q0[2] - cen[2]);
        const float afx = static_cast<float>(ax), afy = static_cast<float>(ay), afz = static_cast<float>(az);
        double re64[QL], im64[QL];
#pragma unroll
        for (int k = 0; k < QL; ++k) re64[k] = im64[k] = 0.0;
        const int64_t tbase = sg.tile0 + item.t0;
        const int n_groups = (item.nt + kWaves - 1) / kWaves;
        auto stage = [&](int buf, const float4 &h, const float4 &l) {
            const double b = __builtin_fma(cen[2], double(h.z) + double(l.z),
                             __builtin_fma(cen[1], double(h.y) + double(l.y), cen[0] * (double(h.x) + double(l.x))));
            const float e = __builtin_fmaf(afz, h.z, __builtin_fmaf(afy, h.y, afx * h.x));
            s_xy[buf][tid] = make_float2(h.x, h.y);
            s_z[buf][tid] = h.z;
            lattice_atom_factors<QL>(h, e, frac_f32(b), &s_g[buf][tid * NV]);
        };
        {
            const int tt = tid / kTile;
            if (tt < item.nt) {
                const int64_t ai = (tbase + tt) * kTile + (tid & (kTile - 1));
                stage(0, t_hi[ai], t_lo[ai]);
            }
            if (tid < kWaves && tid < item.nt) s_orig[0][tid] = origins[tbase + tid];
        }
        __syncthreads();
        for (int g = 0; g < n_groups; ++g) {
            const int buf = g & 1;
            float4 nh = make_float4(0.f, 0.f, 0.f, 0.f), nl = nh;
            double4 no = make_double4(0.0, 0.0, 0.0, 0.0);
            const int ng = g + 1;
            const bool have_next = ng < n_groups;
            bool next_real = false;
            if (have_next) {
                const int tt = ng * kWaves + tid / kTile;
                next_real = tt < item.nt;
                if (next_real) {
                    const int64_t ai = (tbase + tt) * kTile + (tid & (kTile - 1));
                    nh = t_hi[ai];
                    nl = t_lo[ai];
                }
                if (tid < kWaves && ng * kWaves + tid < item.nt) no = origins[tbase + ng * kWaves + tid];
            }
            const int tiles_here = min(kWaves, item.nt - g * kWaves);
            for (int w = 0; w < tiles_here; ++w) {
                float cs[QL], sn[QL];
#pragma unroll
                for (int k = 0; k < QL; ++k) cs[k] = sn[k] = 0.f;
                const float2 *axy = &s_xy[buf][w * kTile];
                const float *azp = &s_z[buf][w * kTile];
                const float4 *gt = &s_g[buf][w * kTile * NV];
                if (planar) lattice_tile<QL, true>(axy, azp, gt, dqx, dqy, dqz, cs, sn);
                else lattice_tile<QL, false>(axy, azp, gt, dqx, dqy, dqz, cs, sn);
                const double4 o = s_orig[buf][w];
                const double s0 = __builtin_fma(q0[2], o.z, __builtin_fma(q0[1], o.y, q0[0] * o.x));
                const double t1 = __builtin_fma(az, o.z, __builtin_fma(ay, o.y, ax * o.x));
#pragma unroll
                for (int k = 0; k < QL; ++k) {
                    const float th = frac_f32(__builtin_fma(static_cast<double>(k), t1, s0));
                    const float ct = __builtin_amdgcn_cosf(th), st = __builtin_amdgcn_sinf(th);
                    re64[k] += static_cast<double>(__builtin_fmaf(ct, cs[k], -st * sn[k]));
                    im64[k] += static_cast<double>(__builtin_fmaf(st, cs[k], ct * sn[k]));
                }
            }
            if (have_next) {
                if (next_real) stage(buf ^ 1, nh, nl);
                if (tid < kWaves) s_orig[buf ^ 1][tid] = no;
            }
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < QL; ++k)
            if (k < nk)
                partial[sg.part + static_cast<int64_t>(item.chunk) * sg.n_q + p0 + k] = make_double2(re64[k], im64[k]);
    }
}

// ---------------------------------------------------------------- forward, lattice form on matrix cores
//
// On a row lattice the sum over the atoms of one tile for a run of 32 pixels
// q_c + k' a (k' = k - 15.5, k < 32, q_c the run's midpoint) factorizes into a complex
// matrix product,
//   sum_j f_j e^{2 pi i q.r_j} = F * sum_j Z(run, j) G(j, k),
//   Z(run, j) = e^{2 pi i (theta_run + beta_j + dq_run.d_j)},   theta_run = frac(q_c.o)  (FP64)
//   G(j, k)   = (f_j / F) e^{2 pi i frac(k' a.r_j)},             a.r_j = a.o + a.d_j   (FP64)
// with o the tile origin, d_j = r_j - o, beta_j = frac(q_w.d_j) (FP64) for the centre q_w
// of the wavefront's pixels, dq_run = q_c - q_w and F the largest |f| of the tile (so
// every factor lies in the unit disk).  A wavefront owns 32 runs x 32 pixels (a 32 x 32
// square of the lattice), a block 64 x 64 pixels; per tile that is a 32x32x64 complex
// product.  Z and G come from FP32 sincos of phases reduced in FP64 (|phase| <= 0.5 for
// G; theta and beta in [-0.5, 0.5] plus the small in-square term for Z); each part is
// split into FP16 hi + lo (the exact FP32 residual rounded once) and the product keeps
// hi*hi + hi*lo + lo*hi (relative error ~2^-22) on v_mfma_f32_32x32x16_f16 with FP32
// accumulation: 12 matrix instructions per 16 atoms.  The tile sum times F is folded
// into the pixel's FP64 item sum, as in the other forms.
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef float float16_t __attribute__((ext_vector_type(16)));
constexpr int kMfEdge = 32;                  // wavefront square: 32 runs x 32 pixels
constexpr int kMfRows = 2 * kMfEdge;         // block rectangle: 64 rows
constexpr int kMfCols = 2 * kMfEdge;         //                  x 64 pixels per row

// x = hi + lo with hi the leading 11 significant bits of x (Veltkamp's split with the
// factor 2^13 + 1) and lo the exact FP32 remainder rounded once to FP16.  The hi part is
// formed in FP32, so its conversion to FP16 is exact (|x| >= 2^-14) and every use of it
// agrees; a hi rounded to FP16 directly can be rounded one way where it is packed into
// the matrix operand and the other way where the remainder is taken, at exact ties.
__device__ __forceinline__ void split_f16(float x, _Float16 &hi, _Float16 &lo) {
    const float c = x * 8193.0f;
    const float h = c - (c - x);
    hi = static_cast<_Float16>(h);
    lo = static_cast<_Float16>(x - h);
}

__device__ __forceinline__ half8_t neg8(half8_t v) {
    uint4 u = __builtin_bit_cast(uint4, v);
    u.x ^= 0x80008000u;
    u.y ^= 0x80008000u;
    u.z ^= 0x80008000u;
    u.w ^= 0x80008000u;
    return __builtin_bit_cast(half8_t, u);
}

template <int OCC>
__global__ __launch_bounds__(kBlock, OCC) void k_forward_lattice_mfma(
    const FwdItem *__restrict__ items, int32_t n_items, int32_t *__restrict__ counter,
    const FwdSeg *__restrict__ segs, const double *__restrict__ q, const float4 *__restrict__ t_hi,
    const float4 *__restrict__ t_lo, const double4 *__restrict__ origins, double2 *__restrict__ partial) {
    // G pieces: [buf][re_hi, re_lo, im_hi, im_lo][16-atom step][pixel k][8-atom half]
    __shared__ half8_t s_g[2][4][kTile / 16][kMfEdge][2];
    __shared__ float4 s_d[2][kTile];           // (d_x, d_y, d_z, 0)
    __shared__ float s_beta[2][kWaves][kTile];  // beta_j for each wavefront's centre
    __shared__ double4 s_orig[2];
    __shared__ double4 s_cen[kWaves];
    __shared__ int32_t s_item;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int run = lane & 31, hz = lane >> 5;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int32_t it = s_item;
        __syncthreads();
        if (it >= n_items) break;
        const FwdItem item = items[it];
        const FwdSeg sg = segs[item.seg];
        const int n1 = sg.n_q / sg.n2;
        const int ib = item.p0 / sg.n_jb, jb = item.p0 - ib * sg.n_jb;
        const int row0 = ib * kMfRows + (wave >> 1) * kMfEdge;
        const int col0 = jb * kMfCols + (wave & 1) * kMfEdge;
        const int row = row0 + run;
        const bool active = row < n1 && col0 < sg.n2;
        const int nk = active ? min(kMfEdge, sg.n2 - col0) : 0;
        const int p0 = active ? row * sg.n2 + col0 : 0;
        const double ax = sg.a[0], ay = sg.a[1], az = sg.a[2];
        // the run's midpoint q_{p0} + 15.5 a (revolutions / A), from the lattice model
        double qc[3];
        {
            const double e[3] = {ax, ay, az};
            for (int c = 0; c < 3; ++c)
                qc[c] = __builtin_fma(0.5 * (kMfEdge - 1), e[c], q[(sg.q + p0) * 3 + c] * kInvTwoPi);
        }
        // wavefront centre: bounding box of its active pixels
        double lo[3], hi[3];
        {
            const double e[3] = {ax, ay, az};
            for (int c = 0; c < 3; ++c) {
                const double v0 = __builtin_fma(-0.5 * (kMfEdge - 1), e[c], qc[c]);
                const double v1 = __builtin_fma(static_cast<double>(nk > 0 ? nk - 1 : 0), e[c], v0);
                lo[c] = active ? fmin(v0, v1) : INFINITY;
                hi[c] = active ? fmax(v0, v1) : -INFINITY;
            }
        }
        for (int c = 0; c < 3; ++c)
            for (int off = 32; off > 0; off >>= 1) {
                lo[c] = fmin(lo[c], __shfl_xor(lo[c], off));
                hi[c] = fmax(hi[c], __shfl_xor(hi[c], off));
            }
        // a wavefront without pixels (past the last row) keeps a finite centre
        double cw[3];
        for (int c = 0; c < 3; ++c) cw[c] = lo[c] <= hi[c] ? 0.5 * (lo[c] + hi[c]) : qc[c];
        const bool planar = !(lo[2] < hi[2]);
        if (lane == 0) s_cen[wave] = make_double4(cw[0], cw[1], cw[2], 0.0);
        __syncthreads();
        const float dqx = static_cast<float>(qc[0] - cw[0]);
        const float dqy = static_cast<float>(qc[1] - cw[1]);
        const float dqz = static_cast<float>(qc[2] - cw[2]);
        const int64_t tbase = sg.tile0 + item.t0;
        // staging of tile tt into buffer buf: atom offsets and the four wavefronts' beta
        // by the first wavefront; the G factors of pixel gk, 16-atom step gks and
        // 8-atom half ghh by every thread
        const int gk = tid & 31, gks = (tid >> 5) & 3, ghh = tid >> 7;
        const double kc = static_cast<double>(gk) - 0.5 * (kMfEdge - 1);
        auto stage = [&](int buf, int tt) {
            const int64_t ti = tbase + tt;
            const double4 o = origins[ti];
            if (tid < kTile) {
                const float4 h = t_hi[ti * kTile + tid], l = t_lo[ti * kTile + tid];
                const double dx = double(h.x) + double(l.x), dy = double(h.y) + double(l.y),
                             dz = double(h.z) + double(l.z);
                s_d[buf][tid] = make_float4(h.x, h.y, h.z, 0.f);
#pragma unroll
                for (int w = 0; w < kWaves; ++w) {
                    const double4 c = s_cen[w];
                    s_beta[buf][w][tid] = frac_f32(__builtin_fma(c.z, dz, __builtin_fma(c.y, dy, c.x * dx)));
                }
            }
            if (tid == 0) s_orig[buf] = o;
            const double t1 = __builtin_fma(az, o.z, __builtin_fma(ay, o.y, ax * o.x));
            const float sc = o.w > 0.0 ? static_cast<float>(1.0 / o.w) : 0.f;
            half8_t grh, grl, gih, gil;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t ai = ti * kTile + 16 * gks + 8 * ghh + u;
                const float4 h = t_hi[ai], l = t_lo[ai];
                const double ar = t1 + __builtin_fma(az, double(h.z) + double(l.z),
                                       __builtin_fma(ay, double(h.y) + double(l.y), ax * (double(h.x) + double(l.x))));
                const float ph = frac_f32(kc * ar);
                const float w = h.w * sc;
                const float gr = w * __builtin_amdgcn_cosf(ph), gi = w * __builtin_amdgcn_sinf(ph);
                _Float16 a, bb;
                split_f16(gr, a, bb);
                grh[u] = a;
                grl[u] = bb;
                split_f16(gi, a, bb);
                gih[u] = a;
                gil[u] = bb;
            }
            s_g[buf][0][gks][gk][ghh] = grh;
            s_g[buf][1][gks][gk][ghh] = grl;
            s_g[buf][2][gks][gk][ghh] = gih;
            s_g[buf][3][gks][gk][ghh] = gil;
        };
        double dre[16], dim[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) dre[i] = dim[i] = 0.0;
        if (item.nt > 0) stage(0, 0);
        __syncthreads();
        for (int tt = 0; tt < item.nt; ++tt) {
            const int buf = tt & 1;
            const double4 o = s_orig[buf];
            const float th = frac_f32(__builtin_fma(qc[2], o.z, __builtin_fma(qc[1], o.y, qc[0] * o.x)));
            float16_t are, aim;
#pragma unroll
            for (int i = 0; i < 16; ++i) are[i] = aim[i] = 0.f;
#pragma unroll
            for (int ks = 0; ks < kTile / 16; ++ks) {
                half8_t zrh, zrl, zih, zil;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int j = 16 * ks + 8 * hz + u;
                    const float4 d = s_d[buf][j];
                    float ph = th + s_beta[buf][wave][j];
                    ph = __builtin_fmaf(dqx, d.x, ph);
                    ph = __builtin_fmaf(dqy, d.y, ph);
                    if (!planar) ph = __builtin_fmaf(dqz, d.z, ph);
                    _Float16 a, bb;
                    split_f16(__builtin_amdgcn_cosf(ph), a, bb);
                    zrh[u] = a;
                    zrl[u] = bb;
                    split_f16(__builtin_amdgcn_sinf(ph), a, bb);
                    zih[u] = a;
                    zil[u] = bb;
                }
                const half8_t grh = s_g[buf][0][ks][run][hz], grl = s_g[buf][1][ks][run][hz];
                const half8_t gih = s_g[buf][2][ks][run][hz], gil = s_g[buf][3][ks][run][hz];
                const half8_t nzih = neg8(zih), nzil = neg8(zil);
                are = __builtin_amdgcn_mfma_f32_32x32x16_f16(zrh, grh, are, 0, 0, 0);
                aim = __builtin_amdgcn_mfma_f32_32x32x16_f16(zrh, gih, aim, 0, 0, 0);
                are = __builtin_amdgcn_mfma_f32_32x32x16_f16(zrh, grl, are, 0, 0, 0);
                aim = __builtin_amdgcn_mfma_f32_32x32x16_f16(zrh, gil, aim, 0, 0, 0);
                are = __builtin_amdgcn_mfma_f32_32x32x16_f16(zrl, grh, are, 0, 0, 0);
                aim = __builtin_amdgcn_mfma_f32_32x32x16_f16(zrl, gih, aim, 0, 0, 0);
                are = __builtin_amdgcn_mfma_f32_32x32x16_f16(nzih, gih, are, 0, 0, 0);
                aim = __builtin_amdgcn_mfma_f32_32x32x16_f16(zih, grh, aim, 0, 0, 0);
                are = __builtin_amdgcn_mfma_f32_32x32x16_f16(nzih, gil, are, 0, 0, 0);
                aim = __builtin_amdgcn_mfma_f32_32x32x16_f16(zih, grl, aim, 0, 0, 0);
                are = __builtin_amdgcn_mfma_f32_32x32x16_f16(nzil, gih, are, 0, 0, 0);
                aim = __builtin_amdgcn_mfma_f32_32x32x16_f16(zil, grh, aim, 0, 0, 0);
            }
            const float F = static_cast<float>(o.w);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                dre[i] += static_cast<double>(F * are[i]);
                dim[i] += static_cast<double>(F * aim[i]);
            }
            if (tt + 1 < item.nt) stage(buf ^ 1, tt + 1);
            __syncthreads();
        }
        // accumulator entry i: run (i/4)*8 + hz*4 + i%4, pixel k = lane % 32
        const int k = lane & 31;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int r = (i >> 2) * 8 + hz * 4 + (i & 3);
            const int prow = row0 + r, pcol = col0 + k;
            if (prow < n1 && pcol < sg.n2)
                partial[sg.part + static_cast<int64_t>(item.chunk) * sg.n_q + static_cast<int64_t>(prow) * sg.n2 + pcol] =
                    make_double2(dre[i], dim[i]);
        }
    }
}

// Largest deviation of a pixel set from the row lattice q_p = q_{row start} + j a
// (j = p mod n2), per block, and the largest |q_z| (after the gridDim.x deviations);
// NaN counts as infinite.
__global__ __launch_bounds__(kBlock) void k_lattice_check(const double *__restrict__ q, int32_t n_q, int32_t n2,
                                                          double ax, double ay, double az,
                                                          double *__restrict__ block_max) {
    __shared__ double red[kBlock], redz[kBlock];
    double m = 0.0, mz = 0.0;
    const double a[3] = {ax, ay, az};
    for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < n_q;
         p += static_cast<int64_t>(gridDim.x) * kBlock) {
        const int64_t j = p % n2, r0 = p - j;
        for (int c = 0; c < 3; ++c) {
            const double d = fabs(q[3 * p + c] - __builtin_fma(static_cast<double>(j), a[c], q[3 * r0 + c]));
            m = d == d ? fmax(m, d) : INFINITY;
        }
        const double z = fabs(q[3 * p + 2]);
        mz = z == z ? fmax(mz, z) : INFINITY;
    }
    red[threadIdx.x] = m;
    redz[threadIdx.x] = mz;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < static_cast<unsigned>(off)) {
            red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
            redz[threadIdx.x] = fmax(redz[threadIdx.x], redz[threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        block_max[blockIdx.x] = red[0];
        block_max[gridDim.x + blockIdx.x] = redz[0];
    }
}

// Rows of n2 pixels sharing q_y: per block, the number of pixels whose q_y differs
// from the first pixel of their row (NaN counts as a difference).
__global__ __launch_bounds__(kBlock) void k_row_check(const double *__restrict__ q, int32_t n_q, int32_t n2,
                                                      double *__restrict__ block_bad) {
    __shared__ double red[kBlock];
    double bad = 0.0;
    for (int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; p < n_q;
         p += static_cast<int64_t>(gridDim.x) * kBlock) {
        const int64_t r0 = p - p % n2;
        bad += q[3 * p + 1] == q[3 * r0 + 1] ? 0.0 : 1.0;
    }
    red[threadIdx.x] = bad;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < static_cast<unsigned>(off)) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) block_bad[blockIdx.x] = red[0];
}

// Sum the chunk partials of every pixel in chunk order; a = sum f cos,
// b = -sum f sin (the amplitude carries exp(-i q.r)), I = a*a + b*b.
__global__ __launch_bounds__(kBlock) void k_forward_combine(const FwdSeg *__restrict__ segs,
                                                            const double2 *__restrict__ partial,
                                                            double *__restrict__ I,
                                                            double *__restrict__ amp) {
    const FwdSeg sg = segs[blockIdx.y];
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= sg.n_q) return;
    // chunk partials added in chunk order, kAhead chunks loaded before they are added
    constexpr int kAhead = 8;
    const double2 *src = partial + sg.part + p;
    double a = 0.0, sb = 0.0;
    for (int c0 = 0; c0 < sg.n_chunks; c0 += kAhead) {
        double2 v[kAhead];
#pragma unroll
        for (int u = 0; u < kAhead; ++u)
            if (c0 + u < sg.n_chunks) v[u] = src[static_cast<int64_t>(c0 + u) * sg.n_q];
#pragma unroll
        for (int u = 0; u < kAhead; ++u)
            if (c0 + u < sg.n_chunks) {
                a += v[u].x;
                sb += v[u].y;
            }
    }
    const double b = -sb;
    const int64_t o = sg.out + p;
    I[o] = __builtin_fma(a, a, b * b);
    if (amp) {
        amp[2 * o] = a;
        amp[2 * o + 1] = b;
    }
}

// ---------------------------------------------------------------- gradient
//
// dL/dr_j = -2 f_j sum_p w_p q_p (a_p sin phi_pj + b_p cos phi_pj)
//         =    f_j sum_p W_p sin(phi_pj + psi_p),
// with W_p = -2 w_p |A_p| q_p and psi_p = arg(A_p) / (2 pi) (revolutions), since
// a sin(phi) + b cos(phi) = |A| sin(phi + arg A) for A = a + ib.
// Pixel prologue, in sorted order, groups of 64 consecutive sorted pixels
// sharing a centre q_c: FP32 (dq, 0), FP32 (W, 0), FP64 (q_rev, psi) and the
// group centre (FP64; w = flags of the components that vanish in the group).
constexpr int kPixStage = 64;
__global__ __launch_bounds__(kBlock) void k_grad_prep(const GradSeg *__restrict__ segs,
                                                      const double *__restrict__ q,
                                                      const int32_t *__restrict__ pix_order,
                                                      const double *__restrict__ amp,
                                                      const double *__restrict__ w,
                                                      float4 *__restrict__ pdq,
                                                      float4 *__restrict__ pw,
                                                      double4 *__restrict__ pq64,
                                                      double4 *__restrict__ centre) {
    const GradSeg sg = segs[blockIdx.y];
    const int sp = blockIdx.x * kBlock + threadIdx.x;  // sorted slot
    if (blockIdx.x * kBlock >= sg.n_q) return;          // block-uniform exit
    const bool real = sp < sg.n_q;
    const int p = pix_order[sg.slot0 + (real ? sp : sg.n_q - 1)];
    const double *qp = q + (sg.q + p) * 3;
    const double rx = qp[0] * kInvTwoPi, ry = qp[1] * kInvTwoPi, rz = qp[2] * kInvTwoPi;
    double lo[3] = {real ? rx : INFINITY, real ? ry : INFINITY, real ? rz : INFINITY};
    double hi[3] = {real ? rx : -INFINITY, real ? ry : -INFINITY, real ? rz : -INFINITY};
    for (int c = 0; c < 3; ++c)
        for (int off = 32; off > 0; off >>= 1) {
            lo[c] = fmin(lo[c], __shfl_xor(lo[c], off));
            hi[c] = fmax(hi[c], __shfl_xor(hi[c], off));
        }
    const double cx = 0.5 * (lo[0] + hi[0]), cy = 0.5 * (lo[1] + hi[1]), cz = 0.5 * (lo[2] + hi[2]);
    if (!real) return;
    const double a = amp[2 * (sg.out + p)], b = amp[2 * (sg.out + p) + 1];
    const double mag = __builtin_sqrt(a * a + b * b);
    const double psi = atan2(b, a) * kInvTwoPi;
    const double c = -2.0 * w[sg.out + p] * mag;
    const int64_t i = sg.slot0 + sp;
    pdq[i] = make_float4(static_cast<float>(rx - cx), static_cast<float>(ry - cy),
                         static_cast<float>(rz - cz), 0.f);
    pw[i] = make_float4(static_cast<float>(c * qp[0]), static_cast<float>(c * qp[1]),
                        static_cast<float>(c * qp[2]), 0.f);
    pq64[i] = make_double4(rx, ry, rz, psi);
    // group kind, a sum of flags: 1 all q_z equal (dq_z = 0), 2 all q_z = 0 (also W_z = 0),
    // 4 all q_y equal (dq_y = 0: a run along one detector row)
    if ((threadIdx.x & 63) == 0)
        centre[sg.grp0 + sp / kPixStage] =
            make_double4(cx, cy, cz, (lo[2] == hi[2] ? (lo[2] == 0.0 ? 3.0 : 1.0) : 0.0) + (lo[1] == hi[1] ? 4.0 : 0.0));
}

// Workgroup = 4 wavefronts; wavefront w owns tiles t0 + w*AL + a (a < AL),
// lane l owns atom l of each.  The item's sorted pixels are staged 64 at a
// time (one centre q_c per 64): per staged group each lane forms
// beta = frac(q_c.d) for its atoms (FP64, from the exact offset) and each
// wavefront the base phases theta'(p, tile) = frac(q_p.o + psi_p); the next
// group's pixel data is fetched from memory while this one is summed.  Per
// pair: add + 3 FMA (one fewer when the group has dq_z = 0, one fewer when it has
// dq_y = 0: a run along a detector row), one v_sin, 3 FMA (2 when every q_z of the
// group is 0, so W_z = 0).  Group partials fold into FP64.
template <int AL, bool PLANAR, bool NOZ, bool NOY>
__device__ __forceinline__ void pixel_pairs(const float4 *__restrict__ sq, const float4 *__restrict__ sw,
                                            const float (*__restrict__ sth)[kPixStage],
                                            const float (&dx)[AL], const float (&dy)[AL],
                                            const float (&dz)[AL], const float (&beta)[AL],
                                            float (&gx)[AL], float (&gy)[AL], float (&gz)[AL]) {
    constexpr int kRun = 4;  // pixels per block: phases, then sines, then sums
#pragma unroll 1
    for (int m0 = 0; m0 < kPixStage; m0 += kRun) {
        float sn[kRun][AL];
#pragma unroll
        for (int k = 0; k < kRun; ++k) {
            const float4 qv = sq[m0 + k];
#pragma unroll
            for (int a = 0; a < AL; ++a) {
                float ph = __builtin_fmaf(qv.x, dx[a], sth[a][m0 + k] + beta[a]);
                if (!NOY) ph = __builtin_fmaf(qv.y, dy[a], ph);
                if (!PLANAR) ph = __builtin_fmaf(qv.z, dz[a], ph);
                sn[k][a] = ph;
            }
        }
#pragma unroll
        for (int k = 0; k < kRun; ++k)
#pragma unroll
            for (int a = 0; a < AL; ++a) sn[k][a] = __builtin_amdgcn_sinf(sn[k][a]);
#pragma unroll
        for (int k = 0; k < kRun; ++k) {
            const float4 wv = sw[m0 + k];
#pragma unroll
            for (int a = 0; a < AL; ++a) {
                gx[a] = __builtin_fmaf(wv.x, sn[k][a], gx[a]);
                gy[a] = __builtin_fmaf(wv.y, sn[k][a], gy[a]);
                if (!NOZ) gz[a] = __builtin_fmaf(wv.z, sn[k][a], gz[a]);
            }
        }
    }
}

// Lattice rows: a 64-pixel group is the run q_{c} + (m - 31.5) a, m < 64, of one
// row (its centre q_c is the run's midpoint), so dq_m.d_j = (m - 31.5) e_j with
// e_j = a.d_j fixed per atom lane: phase = theta'(m, tile) + (beta_j + (m - 31.5) e_j),
// formed per block of 8 pixels as base = fma(m0 - 31.5, e, beta) and then
// fma(k, e, base): one FMA and one add per pair.
template <int AL, bool NOZ>
__device__ __forceinline__ void pixel_pairs_lattice(const float4 *__restrict__ sw,
                                                    const float (*__restrict__ sth)[kPixStage],
                                                    const float (&e)[AL], const float (&beta)[AL],
                                                    float (&gx)[AL], float (&gy)[AL], float (&gz)[AL]) {
    constexpr int kRun = 8;  // pixels per unrolled block: offset (m0 - 31.5 + k) e = base + k e
#pragma unroll 1
    for (int m0 = 0; m0 < kPixStage; m0 += kRun) {
        const float mcb = static_cast<float>(m0) - 0.5f * static_cast<float>(kPixStage - 1);
        // phases of the block first, then the sines, then the sums: independent
        // transcendentals back to back instead of one sine feeding the next FMA
        float sn[kRun][AL];
#pragma unroll
        for (int a = 0; a < AL; ++a) {
            const float base = __builtin_fmaf(mcb, e[a], beta[a]);
            sn[0][a] = sth[a][m0] + base;
#pragma unroll
            for (int k = 1; k < kRun; ++k)
                sn[k][a] = sth[a][m0 + k] + __builtin_fmaf(static_cast<float>(k), e[a], base);
        }
#pragma unroll
        for (int k = 0; k < kRun; ++k)
#pragma unroll
            for (int a = 0; a < AL; ++a) sn[k][a] = __builtin_amdgcn_sinf(sn[k][a]);
#pragma unroll
        for (int k = 0; k < kRun; ++k) {
            const float4 wv = sw[m0 + k];
#pragma unroll
            for (int a = 0; a < AL; ++a) {
                gx[a] = __builtin_fmaf(wv.x, sn[k][a], gx[a]);
                gy[a] = __builtin_fmaf(wv.y, sn[k][a], gy[a]);
                if (!NOZ) gz[a] = __builtin_fmaf(wv.z, sn[k][a], gz[a]);
            }
        }
    }
}

template <int AL, int OCC, bool LAT>
__global__ __launch_bounds__(kBlock, OCC) void k_grad_fp32c(
    const GradItem *__restrict__ items, int32_t n_items, int32_t *__restrict__ counter,
    const GradSeg *__restrict__ segs, const float4 *__restrict__ t_hi,
    const float4 *__restrict__ t_lo, const double4 *__restrict__ origins,
    const float4 *__restrict__ pdq, const float4 *__restrict__ pw,
    const double4 *__restrict__ pq64, const double4 *__restrict__ centre,
    double *__restrict__ gpart) {
    __shared__ float4 s_q[kPixStage];
    __shared__ float4 s_w[kPixStage];
    __shared__ float s_th[kWaves][AL][kPixStage];
    __shared__ double4 s_c;
    __shared__ int32_t s_item;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int32_t it = s_item;
        __syncthreads();
        if (it >= n_items) break;
        const GradItem item = items[it];
        const GradSeg sg = segs[item.seg];
        float dx[AL], dy[AL], dz[AL];
        float lx[AL], ly[AL], lz[AL];
        float e[AL];
        double ox[AL], oy[AL], oz[AL];
        double gx64[AL], gy64[AL], gz64[AL];
#pragma unroll
        for (int a = 0; a < AL; ++a) {
            int t = wave * AL + a;
            t = t < item.nt ? t : 0;
            const int64_t ti = sg.tile0 + item.t0 + t;
            const float4 h = t_hi[ti * kTile + lane], l = t_lo[ti * kTile + lane];
            const double4 o = origins[ti];
            dx[a] = h.x; dy[a] = h.y; dz[a] = h.z;
            lx[a] = l.x; ly[a] = l.y; lz[a] = l.z;
            ox[a] = o.x; oy[a] = o.y; oz[a] = o.z;
            e[a] = LAT ? static_cast<float>(__builtin_fma(sg.a[2], double(h.z) + double(l.z),
                                            __builtin_fma(sg.a[1], double(h.y) + double(l.y),
                                                          sg.a[0] * (double(h.x) + double(l.x)))))
                       : 0.f;
            gx64[a] = gy64[a] = gz64[a] = 0.0;
        }
        // pixel data of a staged group, loaded one group ahead
        float4 r_q = make_float4(0.f, 0.f, 0.f, 0.f), r_w = r_q;
        double4 r_d = make_double4(0.0, 0.0, 0.0, 0.0), r_c = r_d;
        auto fetch = [&](int s0) {
            const int n_here = min(kPixStage, item.np - s0);
            const int sp = item.p0 + s0 + (lane < n_here ? lane : 0);
            const int64_t i = sg.slot0 + sp;
            if (wave == 0) {
                if (!LAT) r_q = pdq[i];
                r_w = lane < n_here ? pw[i] : make_float4(0.f, 0.f, 0.f, 0.f);
                if (lane == 0) r_c = centre[sg.grp0 + (item.p0 + s0) / kPixStage];
            }
            r_d = pq64[i];
        };
        fetch(0);
        for (int s0 = 0; s0 < item.np; s0 += kPixStage) {
            if (wave == 0) {
                if (!LAT) s_q[lane] = r_q;
                s_w[lane] = r_w;
                if (lane == 0) s_c = r_c;
            }
#pragma unroll
            for (int a = 0; a < AL; ++a)
                s_th[wave][a][lane] =
                    frac_f32(__builtin_fma(r_d.z, oz[a], __builtin_fma(r_d.y, oy[a], r_d.x * ox[a])) + r_d.w);
            __syncthreads();
            if (s0 + kPixStage < item.np) fetch(s0 + kPixStage);
            const double4 c = s_c;
            float beta[AL];
#pragma unroll
            for (int a = 0; a < AL; ++a)
                beta[a] = frac_f32(__builtin_fma(c.z, double(dz[a]) + double(lz[a]),
                                   __builtin_fma(c.y, double(dy[a]) + double(ly[a]),
                                                 c.x * (double(dx[a]) + double(lx[a])))));
            float gx[AL], gy[AL], gz[AL];
#pragma unroll
            for (int a = 0; a < AL; ++a) gx[a] = gy[a] = gz[a] = 0.f;
            const int kind = static_cast<int>(c.w);
            const bool z0 = (kind & 2) != 0, dz0 = (kind & 1) != 0, dy0 = (kind & 4) != 0;
            if (LAT) {
                if (z0) pixel_pairs_lattice<AL, true>(s_w, s_th[wave], e, beta, gx, gy, gz);
                else pixel_pairs_lattice<AL, false>(s_w, s_th[wave], e, beta, gx, gy, gz);
            } else if (dy0) {
                if (z0) pixel_pairs<AL, true, true, true>(s_q, s_w, s_th[wave], dx, dy, dz, beta, gx, gy, gz);
                else if (dz0) pixel_pairs<AL, true, false, true>(s_q, s_w, s_th[wave], dx, dy, dz, beta, gx, gy, gz);
                else pixel_pairs<AL, false, false, true>(s_q, s_w, s_th[wave], dx, dy, dz, beta, gx, gy, gz);
            } else if (z0) {
                pixel_pairs<AL, true, true, false>(s_q, s_w, s_th[wave], dx, dy, dz, beta, gx, gy, gz);
            } else if (dz0) {
                pixel_pairs<AL, true, false, false>(s_q, s_w, s_th[wave], dx, dy, dz, beta, gx, gy, gz);
            } else {
                pixel_pairs<AL, false, false, false>(s_q, s_w, s_th[wave], dx, dy, dz, beta, gx, gy, gz);
            }
#pragma unroll
            for (int a = 0; a < AL; ++a) {
                gx64[a] += static_cast<double>(gx[a]);
                gy64[a] += static_cast<double>(gy[a]);
                gz64[a] += static_cast<double>(gz[a]);
            }
            __syncthreads();
        }
#pragma unroll
        for (int a = 0; a < AL; ++a) {
            const int t = wave * AL + a;
            if (t < item.nt) {
                const int64_t slot = sg.part + (static_cast<int64_t>(item.chunk) * sg.n_tiles + item.t0 + t) * kTile + lane;
                gpart[3 * slot] = gx64[a];
                gpart[3 * slot + 1] = gy64[a];
                gpart[3 * slot + 2] = gz64[a];
            }
        }
    }
}

// ---------------------------------------------------------------- adjoint, lattice form on matrix cores
//
// With A_p the amplitude, w_p = dL/dI_p and phi_pj = 2 pi q_p.r_j, the adjoint term of atom j
// is f_j sum_p (-2 w_p |A_p| q_p) sin(phi_pj + arg A_p) = f_j sum_p Im(V_p e^{i phi_pj}) with
// V_p = -2 w_p q_p A_p (a complex vector per pixel).  On a 32 x 32 square of a row lattice
// (pixel (run, k) at q_run + k' a, k' = k - 15.5) the exponential factorizes as in the
// forward, e^{i phi} = Z(run, j) G(k, j), so per component c
//   sum_p Im(V_pc e^{i phi_pj}) = sum_run Im( Z(run, j) H_c(run, j) ),
//   H_c(run, j) = sum_k V_c(run, k) G(k, j),     G(k, j) = e^{2 pi i frac(k' a.r_j)},
// a 32 x 32 x 64 complex product per tile and component on the matrix cores (V split into
// FP16 hi + lo after scaling by the wavefront's largest |part| per component, G split
// likewise; hi*hi + hi*lo + lo*hi), then an FP32 epilogue that forms Z for the
// accumulator's (run, atom) entries and sums Im(Z H) over the runs.  The four
// wavefronts' sums per atom are added in FP64 and written once per tile and 64 x 64
// pixel rectangle; the combine step adds the rectangles and multiplies by f_j.  NC is the
// number of components: 2 for pixel sets whose q_z are all 0 (found when a plan is
// created; the smaller register set then allows two wavefronts per SIMD), else 3.
struct MfGradLds {
    half8_t g[2][4][2][2][kTile];  // [buf][re_hi, re_lo, im_hi, im_lo][k step][k half][atom]
    float4 d[2][kTile];            // (d_x, d_y, d_z, 0)
    float beta[2][kWaves][kTile];  // beta_j for each wavefront's centre
    float4 tq[2][kWaves][kMfEdge]; // per run: (theta, dq_run) with dq_run = q_run - q_w
    double4 qc[kWaves][kMfEdge];   // run midpoints (revolutions / A)
    double4 orig[2];
    double4 cen[kWaves];
    float acc[2][kWaves][3][kTile];
    int32_t item;
};

template <int NC>
__device__ __forceinline__ void grad_lattice_item(MfGradLds &L, const FwdItem &item, const GradSeg &sg,
                                                  int nk, bool active, int64_t p0,
                                                  const double *__restrict__ q, const double *__restrict__ amp,
                                                  const double *__restrict__ w, const float4 *__restrict__ t_hi,
                                                  const float4 *__restrict__ t_lo,
                                                  const double4 *__restrict__ origins, double *__restrict__ gpart) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int hz = lane >> 5, col = lane & 31;
    // A operands: V_c(run = lane % 32, k = 16 s + 8 hz + u), scaled and split
    half8_t av[NC][2][4];
    float scale[NC];
    {
        float vr[NC][16], vi[NC][16];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int k = 16 * s + 8 * hz + u;
                const bool ok = active && k < nk;
                const int64_t p = ok ? p0 + k : 0;
                const double c0 = ok ? -2.0 * w[sg.out + p] : 0.0;
                const double re = c0 * amp[2 * (sg.out + p)], im = c0 * amp[2 * (sg.out + p) + 1];
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const double qv = q[(sg.q + p) * 3 + c];
                    vr[c][8 * s + u] = static_cast<float>(re * qv);
                    vi[c][8 * s + u] = static_cast<float>(im * qv);
                }
            }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            float m = 0.f;
#pragma unroll
            for (int i = 0; i < 16; ++i) m = fmaxf(m, fmaxf(fabsf(vr[c][i]), fabsf(vi[c][i])));
            for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
            scale[c] = m;
            const float inv = m > 0.f ? 1.0f / m : 0.f;
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    _Float16 a, bb;
                    split_f16(vr[c][8 * s + u] * inv, a, bb);
                    av[c][s][0][u] = a;
                    av[c][s][1][u] = bb;
                    split_f16(vi[c][8 * s + u] * inv, a, bb);
                    av[c][s][2][u] = a;
                    av[c][s][3][u] = bb;
                }
        }
    }
    const double ax = sg.a[0], ay = sg.a[1], az = sg.a[2];
    const int64_t tbase = sg.tile0 + item.t0;
    // staging of tile tt: atom offsets and beta (threads < 64), run phases theta and
    // offsets (threads 128..255), the G factors of atom gj, k step gs and k half gh (every thread)
    const int gj = tid & 63, gh = (tid >> 6) & 1, gs = tid >> 7;
    auto stage = [&](int buf, int tt) {
        const int64_t ti = tbase + tt;
        const double4 o = origins[ti];
        const float4 h = t_hi[ti * kTile + gj], l = t_lo[ti * kTile + gj];
        const double dx = double(h.x) + double(l.x), dy = double(h.y) + double(l.y), dz = double(h.z) + double(l.z);
        if (tid < kTile) {
            L.d[buf][tid] = make_float4(h.x, h.y, h.z, 0.f);
#pragma unroll
            for (int v = 0; v < kWaves; ++v) {
                const double4 c = L.cen[v];
                L.beta[buf][v][tid] = frac_f32(__builtin_fma(c.z, dz, __builtin_fma(c.y, dy, c.x * dx)));
            }
        } else if (tid >= 2 * kTile) {
            const int v = (tid - 2 * kTile) >> 5, r = tid & 31;
            const double4 c = L.qc[v][r], cw = L.cen[v];
            L.tq[buf][v][r] = make_float4(frac_f32(__builtin_fma(c.z, o.z, __builtin_fma(c.y, o.y, c.x * o.x))),
                                          static_cast<float>(c.x - cw.x), static_cast<float>(c.y - cw.y),
                                          static_cast<float>(c.z - cw.z));
        }
        if (tid == 0) L.orig[buf] = o;
        const double ar = __builtin_fma(az, o.z + dz, __builtin_fma(ay, o.y + dy, ax * (o.x + dx)));
        half8_t grh, grl, gih, gil;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double kc = static_cast<double>(16 * gs + 8 * gh + u) - 0.5 * (kMfEdge - 1);
            const float ph = frac_f32(kc * ar);
            _Float16 a, bb;
            split_f16(__builtin_amdgcn_cosf(ph), a, bb);
            grh[u] = a;
            grl[u] = bb;
            split_f16(__builtin_amdgcn_sinf(ph), a, bb);
            gih[u] = a;
            gil[u] = bb;
        }
        L.g[buf][0][gs][gh][gj] = grh;
        L.g[buf][1][gs][gh][gj] = grl;
        L.g[buf][2][gs][gh][gj] = gih;
        L.g[buf][3][gs][gh][gj] = gil;
    };
    if (item.nt > 0) stage(0, 0);
    __syncthreads();
    for (int tt = 0; tt < item.nt; ++tt) {
        const int buf = tt & 1;
        // the two 32-atom halves one after the other (one set of accumulators live)
        float gsum[2][NC];
#pragma unroll 1
        for (int nb = 0; nb < 2; ++nb) {
            float16_t hre[NC], him[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int i = 0; i < 16; ++i) hre[c][i] = him[c][i] = 0.f;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int j = 32 * nb + col;
                const half8_t grh = L.g[buf][0][s][hz][j], grl = L.g[buf][1][s][hz][j];
                const half8_t gih = L.g[buf][2][s][hz][j], gil = L.g[buf][3][s][hz][j];
                const half8_t ngih = neg8(gih), ngil = neg8(gil);
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const half8_t vrh = av[c][s][0], vrl = av[c][s][1], vih = av[c][s][2], vil = av[c][s][3];
                    hre[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(vrh, grh, hre[c], 0, 0, 0);
                    him[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(vrh, gih, him[c], 0, 0, 0);
                    hre[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(vrh, grl, hre[c], 0, 0, 0);
                    him[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(vrh, gil, him[c], 0, 0, 0);
                    hre[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(vrl, grh, hre[c], 0, 0, 0);
                    him[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(vrl, gih, him[c], 0, 0, 0);
                    hre[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(vih, ngih, hre[c], 0, 0, 0);
                    him[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(vih, grh, him[c], 0, 0, 0);
                    hre[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(vih, ngil, hre[c], 0, 0, 0);
                    him[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(vih, grl, him[c], 0, 0, 0);
                    hre[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(vil, ngih, hre[c], 0, 0, 0);
                    him[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(vil, grh, him[c], 0, 0, 0);
                }
            }
            // epilogue: atom 32 nb + lane % 32 and the lane's accumulator rows, runs
            // (i / 4) * 8 + 4 hz + i % 4 (one LDS address per half-wavefront)
            const int j = 32 * nb + col;
            const float4 d = L.d[buf][j];
            const float bj = L.beta[buf][wave][j];
            float g[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) g[c] = 0.f;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const float4 tq = L.tq[buf][wave][(i >> 2) * 8 + 4 * hz + (i & 3)];
                float ph = __builtin_fmaf(tq.y, d.x, tq.x + bj);
                ph = __builtin_fmaf(tq.z, d.y, ph);
                if (NC == 3) ph = __builtin_fmaf(tq.w, d.z, ph);
                const float zr = __builtin_amdgcn_cosf(ph), zi = __builtin_amdgcn_sinf(ph);
#pragma unroll
                for (int c = 0; c < NC; ++c) g[c] = __builtin_fmaf(zr, him[c][i], __builtin_fmaf(zi, hre[c][i], g[c]));
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if (nb == 0) gsum[0][c] = g[c];
                else gsum[1][c] = g[c];
            }
        }
        // lanes l and l ^ 32 hold the two halves of the runs: lane l keeps atom l
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const float send = hz ? gsum[0][c] : gsum[1][c];
            const float recv = __shfl_xor(send, 32);
            L.acc[buf][wave][c][lane] = ((hz ? gsum[1][c] : gsum[0][c]) + recv) * scale[c];
        }
        if (tt + 1 < item.nt) stage(buf ^ 1, tt + 1);
        __syncthreads();
        if (tid < 3 * kTile) {
            const int j = tid / 3, c = tid - 3 * j;
            double v = 0.0;
            if (c < NC)
#pragma unroll
                for (int u = 0; u < kWaves; ++u) v += static_cast<double>(L.acc[buf][u][c][j]);
            const int64_t slot = sg.part + (static_cast<int64_t>(item.chunk) * sg.n_tiles + item.t0 + tt) * kTile + j;
            gpart[3 * slot + c] = v;
        }
    }
}

template <int NC, int OCC>
__global__ __launch_bounds__(kBlock, OCC) void k_grad_lattice_mfma(
    const FwdItem *__restrict__ items, int32_t n_items, int32_t *__restrict__ counter,
    const GradSeg *__restrict__ segs, const double *__restrict__ q, const double *__restrict__ amp,
    const double *__restrict__ w, const float4 *__restrict__ t_hi, const float4 *__restrict__ t_lo,
    const double4 *__restrict__ origins, double *__restrict__ gpart) {
    __shared__ MfGradLds L;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int run = lane & 31, hz = lane >> 5;
    for (;;) {
        if (tid == 0) L.item = atomicAdd(counter, 1);
        __syncthreads();
        const int32_t it = L.item;
        __syncthreads();
        if (it >= n_items) break;
        const FwdItem item = items[it];
        const GradSeg sg = segs[item.seg];
        const int n1 = sg.n_q / sg.n2;
        const int ib = item.p0 / sg.n_jb, jb = item.p0 - ib * sg.n_jb;
        const int row0 = ib * kMfRows + (wave >> 1) * kMfEdge;
        const int col0 = jb * kMfCols + (wave & 1) * kMfEdge;
        const int row = row0 + run;
        const bool active = row < n1 && col0 < sg.n2;
        const int nk = active ? min(kMfEdge, sg.n2 - col0) : 0;
        const int64_t p0 = active ? static_cast<int64_t>(row) * sg.n2 + col0 : 0;
        const double e[3] = {sg.a[0], sg.a[1], sg.a[2]};
        double qc[3], lo[3], hi[3];
        for (int c = 0; c < 3; ++c) {
            qc[c] = __builtin_fma(0.5 * (kMfEdge - 1), e[c], q[(sg.q + p0) * 3 + c] * kInvTwoPi);
            const double v0 = __builtin_fma(-0.5 * (kMfEdge - 1), e[c], qc[c]);
            const double v1 = __builtin_fma(static_cast<double>(nk > 0 ? nk - 1 : 0), e[c], v0);
            lo[c] = active ? fmin(v0, v1) : INFINITY;
            hi[c] = active ? fmax(v0, v1) : -INFINITY;
        }
        for (int c = 0; c < 3; ++c)
            for (int off = 32; off > 0; off >>= 1) {
                lo[c] = fmin(lo[c], __shfl_xor(lo[c], off));
                hi[c] = fmax(hi[c], __shfl_xor(hi[c], off));
            }
        if (lane == 0) {
            double cw[3];
            for (int c = 0; c < 3; ++c) cw[c] = lo[c] <= hi[c] ? 0.5 * (lo[c] + hi[c]) : qc[c];
            L.cen[wave] = make_double4(cw[0], cw[1], cw[2], 0.0);
        }
        if (hz == 0) L.qc[wave][run] = make_double4(qc[0], qc[1], qc[2], 0.0);
        __syncthreads();
        grad_lattice_item<NC>(L, item, sg, nk, active, p0, q, amp, w, t_hi, t_lo, origins, gpart);
        __syncthreads();
    }
}

// Sum pixel-chunk partials in chunk order, scale by f_j, scatter to the
// original atom index.
__global__ __launch_bounds__(kBlock) void k_grad_combine(const GradSeg *__restrict__ segs,
                                                         const double *__restrict__ gpart,
                                                         const int32_t *__restrict__ tile_atom,
                                                         const double *__restrict__ f,
                                                         float *__restrict__ g32,
                                                         double *__restrict__ g64) {
    const GradSeg sg = segs[blockIdx.y];
    const int64_t slot = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (slot >= static_cast<int64_t>(sg.n_tiles) * kTile) return;
    const int32_t j = tile_atom[sg.tile0 * kTile + slot];
    if (j < 0) return;
    // chunk partials summed in chunk order, kAhead chunks loaded before they are added
    // (one thread per atom: few threads, so each keeps several loads in flight)
    constexpr int kAhead = 8;
    const int64_t stride = static_cast<int64_t>(sg.n_tiles) * kTile;
    const double *src = gpart + 3 * (sg.part + slot);
    double gx = 0.0, gy = 0.0, gz = 0.0;
    for (int c0 = 0; c0 < sg.n_chunks; c0 += kAhead) {
        double v[kAhead][3];
#pragma unroll
        for (int u = 0; u < kAhead; ++u)
            if (c0 + u < sg.n_chunks) {
                const double *e = src + 3 * (c0 + u) * stride;
                v[u][0] = e[0];
                v[u][1] = e[1];
                v[u][2] = e[2];
            }
#pragma unroll
        for (int u = 0; u < kAhead; ++u)
            if (c0 + u < sg.n_chunks) {
                gx += v[u][0];
                gy += v[u][1];
                gz += v[u][2];
            }
    }
    const double fj = f[sg.f + j];
    const int64_t o = (sg.pos + j) * 3;
    const double r0 = fj * gx, r1 = fj * gy, r2 = fj * gz;
    if (g64) { g64[o] = r0; g64[o + 1] = r1; g64[o + 2] = r2; }
    if (g32) {
        g32[o] = static_cast<float>(r0);
        g32[o + 1] = static_cast<float>(r1);
        g32[o + 2] = static_cast<float>(r2);
    }
}

// ---------------------------------------------------------------- host side

int bits_for(int64_t n) {
    int b = 0;
    while ((int64_t(1) << b) < n) ++b;
    return b;
}

// Cells with more than kOrderSmall atoms, at most.
int64_t big_cells_bound(int64_t atoms) { return atoms / (kOrderSmall + 1) + 1; }

template <typename T>
std::vector<T> largest_first(const std::vector<T> &items, const std::vector<int64_t> &cost) {
    std::vector<int> order(items.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = static_cast<int>(i);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    std::vector<T> out(items.size());
    for (size_t i = 0; i < order.size(); ++i) out[i] = items[order[i]];
    return out;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

// Host tables of one batch layout: segments, pixel sets, work lists.
struct Plan::Tables {
    std::vector<BinSeg> bsegs;
    std::vector<PixSet> psets;
    std::vector<int> seg_set;
    std::vector<LatSet> lat;              // pixel sets found to be row lattices
    std::vector<RowSet> rows;             // pixel sets stored as rows sharing q_y
    std::vector<FwdSeg> fsegs;
    std::vector<FwdItem> fitems;          // general form
    std::vector<FwdItem> litems;          // lattice form
    std::vector<FwdItem> ritems;          // row form
    std::vector<GradSeg> gsegs;
    std::vector<GradItem> gitems;         // concatenated over sub-batches
    std::vector<int> gsub_seg0, gsub_seg1; // segment range of each sub-batch
    std::vector<int> gsub_item0, gsub_nitem;
    std::vector<double> gsub_work;
    std::vector<int> gsub_maxq;
    std::vector<int> gsub_lat;            // form of each sub-batch (1: lattice)
    std::vector<FwdItem> mitems;          // matrix-core gradient: (segment, rectangle, atom tiles),
    int mcount2 = 0;                      // two-component items first
    double mwork = 0.0;
    int64_t atoms = 0, cells = 0, tiles = 0, slots = 0, groups = 0, fpart = 0, gpart = 0;
    int max_atoms = 0, max_tiles = 0, max_q = 0, max_set_q = 0, max_slots_seg = 0;
    double fwork = 0.0, lwork = 0.0, rwork = 0.0;
    size_t sort_tmp = 0;
};

struct Plan::Buffers {
    BinSeg *bsegs = nullptr;
    PixSet *psets = nullptr;
    FwdSeg *fsegs = nullptr;
    FwdItem *fitems = nullptr;
    FwdItem *litems = nullptr;
    FwdItem *ritems = nullptr;
    GradSeg *gsegs = nullptr;
    GradItem *gitems = nullptr;
    FwdItem *mitems = nullptr;
    int32_t *counters = nullptr;
    int32_t *hist = nullptr, *start = nullptr, *cursor = nullptr, *scan_sums = nullptr;
    int32_t *big = nullptr;  // [0] large cells found, [1 ..] their indices (after hist)
    double *segbox = nullptr, *boxpart = nullptr;
    uint32_t *keys = nullptr;
    int32_t *sorted = nullptr;
    float4 *t_hi = nullptr, *t_lo = nullptr;
    int32_t *tile_atom = nullptr;
    double4 *origins = nullptr;
    uint64_t *pk = nullptr, *pk2 = nullptr;
    int32_t *pv = nullptr, *pix_order = nullptr;
    double *pbbox = nullptr;
    void *sort_tmp = nullptr;
    double2 *fpart = nullptr;
    double *gpart = nullptr;
    float4 *pdq = nullptr, *pw = nullptr;
    double4 *pq64 = nullptr, *centre = nullptr;
    size_t table_bytes = 0;
};

Plan::Plan() : T(new Tables()), B(new Buffers()) {}
Plan::~Plan() {
    if (owned_block) (void)hipFree(owned_block);
    delete T;
    delete B;
}

// Row-lattice test of each distinct pixel set: the step a and row length n2
// come from a prefix of the set read back to the host (n2: the first pixel
// off the progression q_0 + j (q_1 - q_0); a then refined from the row's
// ends), and a device pass bounds |q_p - (q_{row start} + j a)| over the set.
xs_status Plan::find_lattices(hipStream_t s, const Segment *segs, int n_segs, const double *q) {
    Tables &t = *T;
    t.lat.clear();
    t.rows.clear();
    std::vector<std::pair<int64_t, int32_t>> seen;
    double *dmax = nullptr;
    constexpr int kCheckBlocks = 512;
    std::vector<double> hmax(2 * kCheckBlocks);
    xs_status st = XS_OK;
    for (int i = 0; i < n_segs && st == XS_OK; ++i) {
        const int64_t qo = segs[i].q;
        const int32_t n_q = segs[i].n_q;
        if (n_q < 16) continue;
        bool done = false;
        for (auto &e : seen) done = done || (e.first == qo && e.second == n_q);
        if (done) continue;
        seen.emplace_back(qo, n_q);
        const int64_t m = std::min<int64_t>(n_q, 65536);
        std::vector<double> h(3 * m);
        if (hipMemcpyAsync(h.data(), q + 3 * qo, sizeof(double) * 3 * m, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            st = set_error(XS_EDEVICE, "lattice test: cannot read q");
            break;
        }
        if (!dmax) {
            if (hipMalloc(&dmax, sizeof(double) * 2 * kCheckBlocks) != hipSuccess) {
                (void)hipGetLastError();
                st = set_error(XS_ENOMEM, "structure test: cannot allocate");
                break;
            }
        }
        const int nb = static_cast<int>(std::min<int64_t>(kCheckBlocks, (n_q + kBlock - 1) / kBlock));
        // rows sharing q_y: row length from the prefix, then every pixel on the device
        {
            int64_t r2 = m;
            for (int64_t p = 1; p < m && r2 == m; ++p)
                if (!(h[3 * p + 1] == h[1])) r2 = p;
            if (!(r2 == m && m < n_q) && r2 >= 8 && n_q % r2 == 0) {
                hipLaunchKernelGGL(k_row_check, dim3(nb), dim3(kBlock), 0, s, q + 3 * qo, n_q,
                                   static_cast<int32_t>(r2), dmax);
                if (hipGetLastError() != hipSuccess ||
                    hipMemcpyAsync(hmax.data(), dmax, sizeof(double) * nb, hipMemcpyDeviceToHost, s) != hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess) {
                    st = set_error(XS_EDEVICE, "row test: device check failed");
                    break;
                }
                double bad = 0.0;
                for (int k = 0; k < nb; ++k) bad += hmax[k];
                if (bad == 0.0) {
                    RowSet rs;
                    rs.q = qo;
                    rs.n_q = n_q;
                    rs.n2 = static_cast<int32_t>(r2);
                    t.rows.push_back(rs);
                }
            }
        }
        double a[3];
        for (int c = 0; c < 3; ++c) a[c] = h[3 + c] - h[c];
        if (a[0] == 0.0 && a[1] == 0.0 && a[2] == 0.0) continue;
        int64_t n2 = m;
        for (int64_t p = 2; p < m && n2 == m; ++p)
            for (int c = 0; c < 3; ++c) {
                const double tol = 1e-6 * (std::fabs(a[c]) + 1e-300) * static_cast<double>(p) + kLatTol;
                if (!(std::fabs(h[3 * p + c] - std::fma(static_cast<double>(p), a[c], h[c])) <= tol)) {
                    n2 = p;
                    break;
                }
            }
        if (n2 == m && m < n_q) continue;  // row longer than the prefix read
        if (n2 < 8 || n_q % n2 != 0) continue;
        for (int c = 0; c < 3; ++c) a[c] = (h[3 * (n2 - 1) + c] - h[c]) / static_cast<double>(n2 - 1);
        hipLaunchKernelGGL(k_lattice_check, dim3(nb), dim3(kBlock), 0, s, q + 3 * qo, n_q, static_cast<int32_t>(n2),
                           a[0], a[1], a[2], dmax);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(hmax.data(), dmax, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            st = set_error(XS_EDEVICE, "lattice test: device check failed");
            break;
        }
        double worst = 0.0, zmax = 0.0;
        for (int k = 0; k < nb; ++k) worst = std::max(worst, hmax[k]);
        for (int k = 0; k < nb; ++k) zmax = hmax[nb + k] == hmax[nb + k] ? std::max(zmax, hmax[nb + k]) : INFINITY;
        if (!(worst <= kLatTol)) continue;
        LatSet ls;
        ls.flat = zmax == 0.0 ? 1 : 0;
        ls.pad = 0;
        ls.q = qo;
        ls.n_q = n_q;
        ls.n2 = static_cast<int32_t>(n2);
        for (int c = 0; c < 3; ++c) ls.a[c] = a[c];
        t.lat.push_back(ls);
    }
    if (dmax) (void)hipFree(dmax);
    return st;
}

// Build every host table of the batch (no device work).
xs_status Plan::build(const Segment *segs, int n_segs, const double *box, const xs_tile_shape &fsh,
                      const xs_tile_shape &gsh) {
    Tables &t = *T;
    fshape = fsh;
    gshape = gsh;
    n_seg = n_segs;
    auto find_lat = [&](int64_t q, int32_t n) -> const LatSet * {
        for (const LatSet &l : t.lat)
            if (l.q == q && l.n_q == n) return &l;
        return nullptr;
    };
    auto find_row = [&](int64_t q, int32_t n) -> const RowSet * {
        for (const RowSet &r : t.rows)
            if (r.q == q && r.n_q == n) return &r;
        return nullptr;
    };
    // forward form of a pixel set: 1 lattice (opt-in), 2 rows, 0 general (sorted pixels)
    auto fwd_form = [&](int64_t q, int32_t n) {
        if (fsh.lattice == 1 && find_lat(q, n)) return 1;
        if (fsh.lattice != 2 && find_row(q, n)) return 2;
        return 0;
    };
    // vector-unit gradient form: 1 lattice, 2 rows (both with the pixels in input order,
    // in groups of 64 along a row), 0 general (sorted pixels).  Input order only where the
    // forward does not read the sorted order.
    auto grad_form = [&](int64_t q, int32_t n) {
        if (fwd_form(q, n) == 0) return 0;
        const LatSet *l = find_lat(q, n);
        if (gsh.lattice == 1 && l && l->n2 % kPixStage == 0) return 1;
        const RowSet *r = find_row(q, n);
        if (gsh.lattice != 2 && r && r->n2 % kPixStage == 0) return 2;
        return 0;
    };
    t.bsegs.resize(n_segs);
    t.seg_set.resize(n_segs);
    for (int i = 0; i < n_segs; ++i) {
        const Segment &sg = segs[i];
        BinSeg &b = t.bsegs[i];
        b.pos = sg.pos;
        b.f = sg.f;
        b.n_atoms = sg.n_atoms;
        b.n_tiles = (sg.n_atoms + kTile - 1) / kTile;
        b.atom0 = t.atoms;
        b.tile0 = t.tiles;
        b.cell0 = t.cells;
        b.pad = 0;
        // cells: largest 2^bits per edge with about >= 2 atoms per cell (bits 1..10)
        int bits = 1;
        while (bits < 10 && (int64_t(1) << (3 * (bits + 1))) * 2 <= sg.n_atoms) ++bits;
        b.bits = bits;
        t.atoms += sg.n_atoms;
        t.tiles += b.n_tiles;
        t.cells += int64_t(1) << (3 * bits);
        t.max_atoms = std::max(t.max_atoms, sg.n_atoms);
        t.max_tiles = std::max(t.max_tiles, b.n_tiles);
        t.max_q = std::max(t.max_q, sg.n_q);
        t.max_slots_seg = std::max(t.max_slots_seg, b.n_tiles * kTile);
        int set = -1;
        for (size_t k = 0; k < t.psets.size(); ++k)
            if (t.psets[k].q == sg.q && t.psets[k].n_q == sg.n_q) { set = static_cast<int>(k); break; }
        if (set < 0) {
            PixSet ps;
            ps.q = sg.q;
            ps.n_q = sg.n_q;
            ps.slot0 = t.slots;
            ps.lattice = grad_form(sg.q, sg.n_q) != 0 ? 1 : 0;
            t.slots += sg.n_q;
            t.psets.push_back(ps);
            set = static_cast<int>(t.psets.size()) - 1;
            t.max_set_q = std::max(t.max_set_q, sg.n_q);
        }
        t.seg_set[i] = set;
    }
    if (t.cells >= (int64_t(1) << 31) || t.atoms >= (int64_t(1) << 31))
        return set_error(XS_ENOTSUP, "batch too large for one FP32C call (%lld atoms, %lld cells)",
                         (long long)t.atoms, (long long)t.cells);
    std::vector<int64_t> set_grp0(t.psets.size());
    for (size_t k = 0; k < t.psets.size(); ++k) {
        set_grp0[k] = t.groups;
        t.groups += (t.psets[k].n_q + kPixStage - 1) / kPixStage;
    }
    // forward work lists (general and lattice form)
    // q_per_lane 32 selects the matrix-core lattice form (64 x 64 pixel items); the
    // general form then runs 8 pixels per lane
    const bool mfma = fsh.q_per_lane == 32;
    const int QL = mfma ? 8 : fsh.q_per_lane, split = std::max(1, fsh.atom_split), ppi = kBlock * QL;
    const int LQ = std::max(2, QL), lcols = mfma ? kMfCols : kLatRuns * LQ, lrows = mfma ? kMfRows : kLatRows;
    t.fsegs.resize(n_segs);
    std::vector<FwdItem> items, litems, ritems;
    std::vector<int64_t> cost, lcost, rcost;
    for (int i = 0; i < n_segs; ++i) {
        FwdSeg &g = t.fsegs[i];
        std::memset(&g, 0, sizeof(g));
        g.q = segs[i].q;
        g.slot0 = t.psets[t.seg_set[i]].slot0;
        g.out = segs[i].out;
        g.tile0 = t.bsegs[i].tile0;
        g.n_q = segs[i].n_q;
        g.n_tiles = t.bsegs[i].n_tiles;
        g.n_chunks = g.n_tiles > 0 ? (g.n_tiles + split - 1) / split : 0;
        g.part = t.fpart;
        t.fpart += static_cast<int64_t>(g.n_chunks) * g.n_q;
        const int form = fwd_form(g.q, g.n_q);
        const LatSet *ls = form == 1 ? find_lat(g.q, g.n_q) : nullptr;
        const RowSet *rs = form == 2 ? find_row(g.q, g.n_q) : nullptr;
        g.form = form;
        if (rs) {
            const int rcols = kRowRuns * QL;
            g.n2 = rs->n2;
            g.n_jb = (g.n2 + rcols - 1) / rcols;
            const int n1 = g.n_q / g.n2;
            const int n_ib = (n1 + kRowRows - 1) / kRowRows;
            for (int r = 0; r < n_ib * g.n_jb; ++r)
                for (int c = 0; c < g.n_chunks; ++c) {
                    FwdItem it;
                    it.seg = i;
                    it.p0 = r;
                    it.t0 = c * split;
                    it.nt = std::min(split, g.n_tiles - c * split);
                    it.chunk = c;
                    it.pad = 0;
                    ritems.push_back(it);
                    const int64_t rows = std::min(kRowRows, n1 - (r / g.n_jb) * kRowRows);
                    const int64_t cols = std::min(rcols, g.n2 - (r % g.n_jb) * rcols);
                    rcost.push_back(rows * cols * it.nt);
                    t.rwork += static_cast<double>(rows * cols) * it.nt * kTile;
                }
            continue;
        }
        if (ls) {
            g.n2 = ls->n2;
            for (int c = 0; c < 3; ++c) g.a[c] = ls->a[c] * kInvTwoPi;
            g.n_jb = (g.n2 + lcols - 1) / lcols;
            const int n_ib = (g.n_q / g.n2 + lrows - 1) / lrows;
            for (int r = 0; r < n_ib * g.n_jb; ++r)
                for (int c = 0; c < g.n_chunks; ++c) {
                    FwdItem it;
                    it.seg = i;
                    it.p0 = r;
                    it.t0 = c * split;
                    it.nt = std::min(split, g.n_tiles - c * split);
                    it.chunk = c;
                    it.pad = 0;
                    litems.push_back(it);
                    const int64_t rows = std::min(lrows, g.n_q / g.n2 - (r / g.n_jb) * lrows);
                    const int64_t cols = std::min(lcols, g.n2 - (r % g.n_jb) * lcols);
                    lcost.push_back(rows * cols * it.nt);
                    t.lwork += static_cast<double>(rows * cols) * it.nt * kTile;
                }
            continue;
        }
        for (int p0 = 0; p0 < g.n_q; p0 += ppi)
            for (int c = 0; c < g.n_chunks; ++c) {
                FwdItem it;
                it.seg = i;
                it.p0 = p0;
                it.t0 = c * split;
                it.nt = std::min(split, g.n_tiles - c * split);
                it.chunk = c;
                it.pad = 0;
                items.push_back(it);
                const int64_t np = std::min(ppi, g.n_q - p0);
                cost.push_back(np * it.nt);
                t.fwork += static_cast<double>(np) * it.nt * kTile;
            }
    }
    t.fitems = largest_first(items, cost);
    t.litems = largest_first(litems, lcost);
    t.ritems = largest_first(ritems, rcost);
    // gradient work lists: segments sharing a pixel set go to different sub-batches;
    // q_per_lane 32 selects the matrix-core lattice form for lattice segments (their own
    // queue of 64 x 64 pixel rectangles x atom tiles), the others run 2 atoms per lane
    const bool gmfma = gsh.q_per_lane == 32;
    const int AL = gmfma ? 2 : gsh.q_per_lane, group = kWaves * AL;
    const int pchunk = std::max(kPixStage, (gsh.pixel_split / kPixStage) * kPixStage);
    t.gsegs.resize(n_segs);
    for (int i = 0; i < n_segs; ++i) {
        GradSeg &g = t.gsegs[i];
        g.q = segs[i].q;
        g.slot0 = t.psets[t.seg_set[i]].slot0;
        g.grp0 = set_grp0[t.seg_set[i]];
        g.out = segs[i].out;
        g.pos = segs[i].pos;
        g.f = segs[i].f;
        g.tile0 = t.bsegs[i].tile0;
        g.n_q = segs[i].n_q;
        g.n_tiles = t.bsegs[i].n_tiles;
        g.n_chunks = (g.n_q > 0 && g.n_tiles > 0) ? (g.n_q + pchunk - 1) / pchunk : 0;
        g.part = t.gpart;
        g.lat = grad_form(g.q, g.n_q) == 1 ? 1 : 0;
        for (int c = 0; c < 3; ++c) g.a[c] = 0.0;
        if (g.lat)
            for (const LatSet &l : t.lat)
                if (l.q == g.q && l.n_q == g.n_q)
                    for (int c = 0; c < 3; ++c) g.a[c] = l.a[c] * kInvTwoPi;
        g.mf = g.n2 = g.n_jb = g.pad = 0;
        if (gmfma && gsh.lattice == 1 && g.n_q > 0 && g.n_tiles > 0)
            for (const LatSet &l : t.lat)
                if (l.q == g.q && l.n_q == g.n_q) {
                    g.mf = l.flat ? 2 : 3;
                    g.n2 = l.n2;
                    g.n_jb = (l.n2 + kMfCols - 1) / kMfCols;
                    g.n_chunks = ((g.n_q / l.n2 + kMfRows - 1) / kMfRows) * g.n_jb;  // one partial per rectangle
                    for (int c = 0; c < 3; ++c) g.a[c] = l.a[c] * kInvTwoPi;
                }
        t.gpart += static_cast<int64_t>(g.n_chunks) * g.n_tiles * kTile;
    }
    int i0 = 0;
    while (i0 < n_segs) {
        int i1 = i0 + 1;
        for (; i1 < n_segs; ++i1) {
            bool clash = t.gsegs[i1].lat != t.gsegs[i0].lat;  // one form per sub-batch
            for (int k = i0; k < i1 && !clash; ++k) clash = t.seg_set[k] == t.seg_set[i1];
            if (clash) break;
        }
        std::vector<GradItem> sub;
        std::vector<int64_t> sc;
        double work = 0.0;
        int mq = 0;
        for (int i = i0; i < i1; ++i) {
            const GradSeg &g = t.gsegs[i];
            mq = std::max(mq, g.n_q);
            if (g.mf) continue;  // matrix-core queue below
            for (int t0 = 0; t0 < g.n_tiles; t0 += group)
                for (int c = 0; c < g.n_chunks; ++c) {
                    GradItem it;
                    it.seg = i;
                    it.t0 = t0;
                    it.nt = std::min(group, g.n_tiles - t0);
                    it.p0 = c * pchunk;
                    it.np = std::min(pchunk, g.n_q - c * pchunk);
                    it.chunk = c;
                    sub.push_back(it);
                    sc.push_back(static_cast<int64_t>(it.nt) * it.np);
                    work += static_cast<double>(it.np) * it.nt * kTile;
                }
        }
        sub = largest_first(sub, sc);
        t.gsub_seg0.push_back(i0);
        t.gsub_seg1.push_back(i1);
        t.gsub_item0.push_back(static_cast<int>(t.gitems.size()));
        t.gsub_nitem.push_back(static_cast<int>(sub.size()));
        t.gsub_work.push_back(work);
        t.gsub_maxq.push_back(mq);
        t.gsub_lat.push_back(t.gsegs[i0].lat);
        t.gitems.insert(t.gitems.end(), sub.begin(), sub.end());
        i0 = i1;
    }
    if (gmfma) {
        const int msplit = gsh.atom_split > 0 ? gsh.atom_split : 64;
        std::vector<FwdItem> mi[2];
        std::vector<int64_t> mc[2];
        for (int i = 0; i < n_segs; ++i) {
            const GradSeg &g = t.gsegs[i];
            if (!g.mf) continue;
            const int cls = g.mf == 2 ? 0 : 1;
            const int n1 = g.n_q / g.n2;
            for (int r = 0; r < g.n_chunks; ++r)
                for (int t0 = 0; t0 < g.n_tiles; t0 += msplit) {
                    FwdItem it;
                    it.seg = i;
                    it.p0 = r;
                    it.t0 = t0;
                    it.nt = std::min(msplit, g.n_tiles - t0);
                    it.chunk = r;
                    it.pad = 0;
                    mi[cls].push_back(it);
                    const int64_t rows = std::min(kMfRows, n1 - (r / g.n_jb) * kMfRows);
                    const int64_t cols = std::min(kMfCols, g.n2 - (r % g.n_jb) * kMfCols);
                    mc[cls].push_back(rows * cols * it.nt);
                    t.mwork += static_cast<double>(rows * cols) * it.nt * kTile;
                }
        }
        t.mitems = largest_first(mi[0], mc[0]);
        t.mcount2 = static_cast<int>(t.mitems.size());
        const std::vector<FwdItem> m3 = largest_first(mi[1], mc[1]);
        t.mitems.insert(t.mitems.end(), m3.begin(), m3.end());
    }
    if (!with_grad) {
        // forward-only plan: no adjoint work lists, partials or pixel prologue buffers
        t.gitems = {};
        t.mitems = {};
        t.gsub_seg0 = {};
        t.gsub_seg1 = {};
        t.gsub_item0 = {};
        t.gsub_nitem = {};
        t.gsub_work = {};
        t.gsub_maxq = {};
        t.gsub_lat = {};
        t.mcount2 = 0;
        t.mwork = 0.0;
        t.gpart = 0;
    }
    // radix-sort workspace for the pixel order
    if (t.slots > 0) {
        size_t bytes = 0;
        XS_HIP(rocprim::radix_sort_pairs(nullptr, bytes, static_cast<const uint64_t *>(nullptr),
                                         static_cast<uint64_t *>(nullptr), static_cast<const int32_t *>(nullptr),
                                         static_cast<int32_t *>(nullptr), static_cast<unsigned int>(t.slots), 0,
                                         3 * kHilbertBits + bits_for(static_cast<int64_t>(t.psets.size())), nullptr));
        t.sort_tmp = bytes;
    }
    return XS_OK;
}

// Carve every device buffer out of one block (plan-owned or stream scratch).
size_t Plan::layout(char *base) {
    Tables &t = *T;
    Buffers &b = *B;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += align256(std::max<size_t>(bytes, 1));
        return p;
    };
    const size_t tb0 = off;
    b.bsegs = reinterpret_cast<BinSeg *>(take(sizeof(BinSeg) * t.bsegs.size()));
    b.psets = reinterpret_cast<PixSet *>(take(sizeof(PixSet) * t.psets.size()));
    b.fsegs = reinterpret_cast<FwdSeg *>(take(sizeof(FwdSeg) * t.fsegs.size()));
    b.fitems = reinterpret_cast<FwdItem *>(take(sizeof(FwdItem) * t.fitems.size()));
    b.litems = reinterpret_cast<FwdItem *>(take(sizeof(FwdItem) * t.litems.size()));
    b.ritems = reinterpret_cast<FwdItem *>(take(sizeof(FwdItem) * t.ritems.size()));
    b.gsegs = reinterpret_cast<GradSeg *>(take(sizeof(GradSeg) * t.gsegs.size()));
    b.gitems = reinterpret_cast<GradItem *>(take(sizeof(GradItem) * t.gitems.size()));
    b.mitems = reinterpret_cast<FwdItem *>(take(sizeof(FwdItem) * t.mitems.size()));
    b.table_bytes = off - tb0;
    // counters: [0] general forward, [1] lattice forward, [2] row forward, [3 + k] gradient
    // sub-batch k, [3 + sub-batches] and [4 + sub-batches] matrix-core gradient (2 and 3 components)
    b.counters = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (t.gsub_seg0.size() + kFwdCounters + 2)));
    const int64_t nsb = (t.cells + kScanBlock - 1) / kScanBlock;
    // hist, then the large-cell count and list (cleared with hist: count only)
    b.hist = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * (t.cells + 1 + big_cells_bound(t.atoms))));
    b.big = b.hist + t.cells;
    b.segbox = reinterpret_cast<double *>(take(sizeof(double) * 6 * t.bsegs.size()));
    b.boxpart = reinterpret_cast<double *>(
        take(sizeof(double) * 6 * kBoxParts * std::max(t.bsegs.size(), t.psets.size())));
    b.start = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * t.cells));
    b.cursor = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * t.cells));
    b.scan_sums = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * nsb));
    b.keys = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * t.atoms));
    b.sorted = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * t.atoms));
    b.t_hi = reinterpret_cast<float4 *>(take(sizeof(float4) * kTile * t.tiles));
    b.t_lo = reinterpret_cast<float4 *>(take(sizeof(float4) * kTile * t.tiles));
    b.tile_atom = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * kTile * t.tiles));
    b.origins = reinterpret_cast<double4 *>(take(sizeof(double4) * t.tiles));
    b.pk = reinterpret_cast<uint64_t *>(take(sizeof(uint64_t) * t.slots));
    b.pk2 = reinterpret_cast<uint64_t *>(take(sizeof(uint64_t) * t.slots));
    b.pv = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * t.slots));
    b.pix_order = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * t.slots));
    b.pbbox = reinterpret_cast<double *>(take(sizeof(double) * 6 * t.psets.size()));
    b.sort_tmp = take(t.sort_tmp);
    b.fpart = reinterpret_cast<double2 *>(take(sizeof(double2) * t.fpart));
    b.gpart = reinterpret_cast<double *>(take(sizeof(double) * 3 * t.gpart));
    const int64_t gslots = with_grad ? t.slots : 0, ggroups = with_grad ? t.groups : 0;
    b.pdq = reinterpret_cast<float4 *>(take(sizeof(float4) * gslots));
    b.pw = reinterpret_cast<float4 *>(take(sizeof(float4) * gslots));
    b.pq64 = reinterpret_cast<double4 *>(take(sizeof(double4) * gslots));
    b.centre = reinterpret_cast<double4 *>(take(sizeof(double4) * ggroups));
    return off;
}

void Plan::describe(int *n_lattice_segs, int *n_row_segs, int *n_fwd_items, int *n_grad_items) const {
    const Tables &t = *T;
    int nl = 0, nr = 0;
    for (const FwdSeg &g : t.fsegs) {
        nl += g.form == 1;
        nr += g.form == 2;
    }
    *n_lattice_segs = nl;
    *n_row_segs = nr;
    *n_fwd_items = static_cast<int>(t.fitems.size() + t.litems.size() + t.ritems.size());
    *n_grad_items = static_cast<int>(t.gitems.size() + t.mitems.size());
}

// Host blob of all tables in the order and alignment of layout().
std::vector<char> Plan::table_blob() const {
    const Tables &t = *T;
    std::vector<char> blob(B->table_bytes, 0);
    size_t off = 0;
    auto put = [&](const void *src, size_t bytes) {
        if (bytes) std::memcpy(blob.data() + off, src, bytes);
        off += align256(std::max<size_t>(bytes, 1));
    };
    put(t.bsegs.data(), sizeof(BinSeg) * t.bsegs.size());
    put(t.psets.data(), sizeof(PixSet) * t.psets.size());
    put(t.fsegs.data(), sizeof(FwdSeg) * t.fsegs.size());
    put(t.fitems.data(), sizeof(FwdItem) * t.fitems.size());
    put(t.litems.data(), sizeof(FwdItem) * t.litems.size());
    put(t.ritems.data(), sizeof(FwdItem) * t.ritems.size());
    put(t.gsegs.data(), sizeof(GradSeg) * t.gsegs.size());
    put(t.gitems.data(), sizeof(GradItem) * t.gitems.size());
    put(t.mitems.data(), sizeof(FwdItem) * t.mitems.size());
    return blob;
}

// Device memory: owned (persistent plans) or the stream's scratch (one-shot).
xs_status Plan::allocate(hipStream_t s, bool owned) {
    const size_t bytes = layout(nullptr);
    char *base = nullptr;
    if (owned) {
        hipError_t e = hipMalloc(&owned_block, bytes);
        if (e != hipSuccess) {
            owned_block = nullptr;
            (void)hipGetLastError();
            return set_error(XS_ENOMEM, "plan: cannot allocate %zu bytes", bytes);
        }
        base = static_cast<char *>(owned_block);
    } else {
        void *p = nullptr;
        XS_TRY(scratch(s, SLOT_PLAN, bytes, &p));
        base = static_cast<char *>(p);
    }
    layout(base);
    device_bytes = bytes;
    const std::vector<char> blob = table_blob();
    if (owned) {
        XS_HIP(hipMemcpy(B->bsegs, blob.data(), blob.size(), hipMemcpyHostToDevice));
    } else {
        XS_TRY(stage_copy(s, SLOT_TABLES, blob.data(), blob.size(), B->bsegs));
    }
    return XS_OK;
}

// Pixel order of every pixel set along the Hilbert curve in q (radix sort).
xs_status Plan::sort_pixels(hipStream_t s, const double *q) {
    Tables &t = *T;
    Buffers &b = *B;
    if (t.slots == 0) return XS_OK;
    const int n_sets = static_cast<int>(t.psets.size());
    hipLaunchKernelGGL(k_bbox_part<PixSet>, dim3(kBoxParts, n_sets), dim3(kBlock), 0, s, b.psets, q, b.boxpart);
    hipLaunchKernelGGL(k_bbox_fold, dim3(n_sets), dim3(64), 0, s, b.boxpart, b.pbbox);
    hipLaunchKernelGGL(k_pix_keys, dim3((t.max_set_q + kBlock - 1) / kBlock, n_sets), dim3(kBlock), 0, s,
                       b.psets, q, b.pbbox, b.pk, b.pv);
    size_t bytes = t.sort_tmp;
    XS_HIP(rocprim::radix_sort_pairs(b.sort_tmp, bytes, b.pk, b.pk2, b.pv, b.pix_order,
                                     static_cast<unsigned int>(t.slots), 0, 3 * kHilbertBits + bits_for(n_sets), s));
    XS_HIP(hipGetLastError());
    return XS_OK;
}

// Atom tiles of every segment (kernels only: capturable in a graph).
xs_status Plan::tile_atoms(hipStream_t s, const double *pos, const double *f) {
    Tables &t = *T;
    Buffers &b = *B;
    if (t.max_atoms == 0) {
        tiled = true;
        return XS_OK;
    }
    TimerScope tm(s, TIMER_BIN);
    const int64_t nsb = (t.cells + kScanBlock - 1) / kScanBlock;
    const unsigned zb = static_cast<unsigned>(std::min<int64_t>((t.cells + kBlock - 1) / kBlock, 4096));
    hipLaunchKernelGGL(k_zero_i32, dim3(zb), dim3(kBlock), 0, s, b.hist, t.cells + 1);
    hipLaunchKernelGGL(k_bbox_part<BinSeg>, dim3(kBoxParts, n_seg), dim3(kBlock), 0, s, b.bsegs, pos, b.boxpart);
    hipLaunchKernelGGL(k_bbox_fold, dim3(n_seg), dim3(64), 0, s, b.boxpart, b.segbox);
    const dim3 ga((t.max_atoms + kBlock - 1) / kBlock, n_seg);
    hipLaunchKernelGGL(k_cell_keys, ga, dim3(kBlock), 0, s, b.bsegs, pos, b.segbox, b.keys, b.hist);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nsb), dim3(kBlock), 0, s, b.hist, t.cells, b.scan_sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, b.scan_sums, nsb);
    hipLaunchKernelGGL(k_scan_down, dim3(nsb), dim3(kBlock), 0, s, b.hist, t.cells, b.scan_sums, b.start,
                       b.cursor);
    hipLaunchKernelGGL(k_cell_scatter, ga, dim3(kBlock), 0, s, b.bsegs, b.keys, b.cursor, b.sorted);
    hipLaunchKernelGGL(k_cell_order, dim3((t.cells + kBlock - 1) / kBlock), dim3(kBlock), 0, s, b.start,
                       b.cursor, t.cells, b.sorted, b.big);
    // large cells, if any (the cell keys are no longer needed: their buffer holds the copies)
    hipLaunchKernelGGL(k_cell_order_big, dim3(static_cast<unsigned>(std::min<int64_t>(big_cells_bound(t.atoms), 256))),
                       dim3(kBlock), 0, s, b.bsegs, static_cast<int32_t>(n_seg), b.start, b.cursor, b.big,
                       reinterpret_cast<int32_t *>(b.keys), b.sorted);
    hipLaunchKernelGGL(k_make_tiles, dim3((t.max_tiles + kWaves - 1) / kWaves, n_seg), dim3(kBlock), 0, s,
                       b.bsegs, pos, f, b.sorted, b.t_hi, b.t_lo, b.origins, b.tile_atom);
    tm.end(static_cast<double>(t.atoms));
    XS_HIP(hipGetLastError());
    tiled = true;
    return XS_OK;
}

namespace {
template <int QL, int OCC>
void launch_forward(hipStream_t s, int n, int32_t *counter, const Plan::Buffers &b, const double *q) {
    const int slots = std::min(n, resident_blocks(reinterpret_cast<const void *>(k_forward_fp32c<QL, OCC>), kBlock));
    hipLaunchKernelGGL((k_forward_fp32c<QL, OCC>), dim3(slots), dim3(kBlock), 0, s, b.fitems, n, counter,
                       b.fsegs, q, b.pix_order, b.t_hi, b.t_lo, b.origins, b.fpart);
}

template <int AL, int OCC, bool LAT>
void launch_grad_form(hipStream_t s, const GradItem *items, int n, int32_t *counter, const Plan::Buffers &b) {
    const int slots =
        std::min(n, resident_blocks(reinterpret_cast<const void *>(k_grad_fp32c<AL, OCC, LAT>), kBlock));
    hipLaunchKernelGGL((k_grad_fp32c<AL, OCC, LAT>), dim3(slots), dim3(kBlock), 0, s, items, n, counter, b.gsegs,
                       b.t_hi, b.t_lo, b.origins, b.pdq, b.pw, b.pq64, b.centre, b.gpart);
}

// The items of one gradient sub-batch are all of one form (lattice or general).
template <int AL, int OCC>
void launch_grad(hipStream_t s, bool lat, const GradItem *items, int n, int32_t *counter,
                 const Plan::Buffers &b) {
    if (lat) launch_grad_form<AL, OCC, true>(s, items, n, counter, b);
    else launch_grad_form<AL, OCC, false>(s, items, n, counter, b);
}

template <int QL, int OCC>
void launch_lattice(hipStream_t s, int n, int32_t *counter, const Plan::Buffers &b, const double *q) {
    const int slots =
        std::min(n, resident_blocks(reinterpret_cast<const void *>(k_forward_lattice<QL, OCC>), kBlock));
    hipLaunchKernelGGL((k_forward_lattice<QL, OCC>), dim3(slots), dim3(kBlock), 0, s, b.litems, n, counter,
                       b.fsegs, q, b.t_hi, b.t_lo, b.origins, b.fpart);
}

template <int OCC>
void launch_lattice_mfma(hipStream_t s, int n, int32_t *counter, const Plan::Buffers &b, const double *q) {
    const int slots =
        std::min(n, resident_blocks(reinterpret_cast<const void *>(k_forward_lattice_mfma<OCC>), kBlock));
    hipLaunchKernelGGL((k_forward_lattice_mfma<OCC>), dim3(slots), dim3(kBlock), 0, s, b.litems, n, counter,
                       b.fsegs, q, b.t_hi, b.t_lo, b.origins, b.fpart);
}

template <int NC, int OCC>
void launch_grad_lattice_mfma(hipStream_t s, const FwdItem *items, int n, int32_t *counter, const Plan::Buffers &b,
                              const double *q, const double *amp, const double *w) {
    const int slots =
        std::min(n, resident_blocks(reinterpret_cast<const void *>(k_grad_lattice_mfma<NC, OCC>), kBlock));
    hipLaunchKernelGGL((k_grad_lattice_mfma<NC, OCC>), dim3(slots), dim3(kBlock), 0, s, items, n, counter,
                       b.gsegs, q, amp, w, b.t_hi, b.t_lo, b.origins, b.gpart);
}

bool launch_lattice_variant(hipStream_t s, int ql, int occ, int n, int32_t *cnt, const Plan::Buffers &b,
                            const double *q) {
    const bool o4 = occ == 4;
    switch (ql) {
    case 32: occ == 3 ? launch_lattice_mfma<3>(s, n, cnt, b, q) : launch_lattice_mfma<1>(s, n, cnt, b, q); return true;
    case 1:
    case 2: o4 ? launch_lattice<2, 4>(s, n, cnt, b, q) : launch_lattice<2, 1>(s, n, cnt, b, q); return true;
    case 4: o4 ? launch_lattice<4, 4>(s, n, cnt, b, q) : launch_lattice<4, 1>(s, n, cnt, b, q); return true;
    case 8: o4 ? launch_lattice<8, 4>(s, n, cnt, b, q) : launch_lattice<8, 1>(s, n, cnt, b, q); return true;
    default: return false;
    }
}

// Built variants: pixels (forward) or atoms (gradient) per lane, and an
// optional bound of 4 wavefronts per SIMD (at most 128 VGPRs).
bool launch_forward_variant(hipStream_t s, int ql, int occ, int n, int32_t *cnt, const Plan::Buffers &b,
                            const double *q) {
    const bool o4 = occ == 4;
    switch (ql) {
    case 1: launch_forward<1, 1>(s, n, cnt, b, q); return true;
    case 2: o4 ? launch_forward<2, 4>(s, n, cnt, b, q) : launch_forward<2, 1>(s, n, cnt, b, q); return true;
    case 4: o4 ? launch_forward<4, 4>(s, n, cnt, b, q) : launch_forward<4, 1>(s, n, cnt, b, q); return true;
    case 8: launch_forward<8, 1>(s, n, cnt, b, q); return true;
    default: return false;
    }
}

template <int QL, int OCC>
void launch_rows(hipStream_t s, int n, int32_t *counter, const Plan::Buffers &b, const double *q) {
    const int slots = std::min(n, resident_blocks(reinterpret_cast<const void *>(k_forward_rows<QL, OCC>), kBlock));
    hipLaunchKernelGGL((k_forward_rows<QL, OCC>), dim3(slots), dim3(kBlock), 0, s, b.ritems, n, counter, b.fsegs, q,
                       b.t_hi, b.t_lo, b.origins, b.fpart);
}

bool launch_rows_variant(hipStream_t s, int ql, int occ, int n, int32_t *cnt, const Plan::Buffers &b,
                         const double *q) {
    const bool o4 = occ == 4;
    switch (ql) {
    case 1: launch_rows<1, 1>(s, n, cnt, b, q); return true;
    case 2: o4 ? launch_rows<2, 4>(s, n, cnt, b, q) : launch_rows<2, 1>(s, n, cnt, b, q); return true;
    case 4: o4 ? launch_rows<4, 4>(s, n, cnt, b, q) : launch_rows<4, 1>(s, n, cnt, b, q); return true;
    case 8: occ == 3 ? launch_rows<8, 3>(s, n, cnt, b, q) : launch_rows<8, 1>(s, n, cnt, b, q); return true;
    default: return false;
    }
}

bool launch_grad_variant(hipStream_t s, int al, int occ, bool lat, const GradItem *items, int n, int32_t *cnt,
                         const Plan::Buffers &b) {
    const bool o4 = occ == 4;
    switch (al) {
    case 1: launch_grad<1, 1>(s, lat, items, n, cnt, b); return true;
    case 2:
        occ == 5 ? launch_grad<2, 5>(s, lat, items, n, cnt, b) : launch_grad<2, 1>(s, lat, items, n, cnt, b);
        return true;
    case 4:
        o4 ? launch_grad<4, 4>(s, lat, items, n, cnt, b) : launch_grad<4, 1>(s, lat, items, n, cnt, b);
        return true;
    case 8: launch_grad<8, 1>(s, lat, items, n, cnt, b); return true;
    default: return false;
    }
}
}  // namespace

xs_status Plan::forward(hipStream_t s, const double *q, double *I, double *amp) {
    Tables &t = *T;
    Buffers &b = *B;
    const int n = static_cast<int>(t.fitems.size()), nl = static_cast<int>(t.litems.size());
    const int nr = static_cast<int>(t.ritems.size());
    if (n + nl + nr > 0) {
        hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, s, b.counters, kFwdCounters);
        TimerScope tm(s, TIMER_FWD32);
        const int qlg = fshape.q_per_lane == 32 ? 8 : fshape.q_per_lane;  // general items of the matrix-core shape
        if (n > 0 && !launch_forward_variant(s, qlg, fshape.waves_per_simd, n, b.counters, b, q))
            return set_error(XS_EINVAL, "q_per_lane must be 1, 2, 4 or 8");
        if (nl > 0 &&
            !launch_lattice_variant(s, fshape.q_per_lane, fshape.waves_per_simd, nl, b.counters + 1, b, q))
            return set_error(XS_EINVAL, "q_per_lane must be 1, 2, 4 or 8");
        if (nr > 0 && !launch_rows_variant(s, qlg, fshape.waves_per_simd, nr, b.counters + 2, b, q))
            return set_error(XS_EINVAL, "q_per_lane must be 1, 2, 4 or 8");
        tm.end(t.fwork + t.lwork + t.rwork);
        XS_HIP(hipGetLastError());
    }
    if (t.max_q > 0) {
        hipLaunchKernelGGL(k_forward_combine, dim3((t.max_q + kBlock - 1) / kBlock, n_seg), dim3(kBlock), 0, s,
                           b.fsegs, b.fpart, I, amp);
        XS_HIP(hipGetLastError());
    }
    return XS_OK;
}

xs_status Plan::grad(hipStream_t s, const double *q, const double *f, const double *amp,
                     const double *dL_dI, float *g32, double *g64) {
    if (!with_grad) return set_error(XS_EINVAL, "the plan was created for the forward only");
    Tables &t = *T;
    Buffers &b = *B;
    for (size_t k = 0; k < t.gsub_seg0.size(); ++k) {
        const int i0 = t.gsub_seg0[k], i1 = t.gsub_seg1[k];
        // the prologue feeds the vector-unit queue only (matrix-core segments read amp and w)
        if (t.gsub_maxq[k] > 0 && t.gsub_nitem[k] > 0)
            hipLaunchKernelGGL(k_grad_prep, dim3((t.gsub_maxq[k] + kBlock - 1) / kBlock, i1 - i0), dim3(kBlock), 0,
                               s, b.gsegs + i0, q, b.pix_order, amp, dL_dI, b.pdq, b.pw, b.pq64, b.centre);
        const int n = t.gsub_nitem[k];
        if (n == 0) continue;
        int32_t *cnt = b.counters + kFwdCounters + k;
        hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, s, cnt, 1);
        const GradItem *items = b.gitems + t.gsub_item0[k];
        TimerScope tm(s, TIMER_GRAD32);
        const int al = gshape.q_per_lane == 32 ? 2 : gshape.q_per_lane;  // non-lattice systems of a ql-32 plan
        if (!launch_grad_variant(s, al, gshape.waves_per_simd, t.gsub_lat[k] != 0, items, n, cnt, b))
            return set_error(XS_EINVAL, "q_per_lane must be 1, 2, 4 or 8");
        tm.end(t.gsub_work[k]);
        XS_HIP(hipGetLastError());
    }
    if (!t.mitems.empty()) {
        const int n2 = t.mcount2, n3 = static_cast<int>(t.mitems.size()) - t.mcount2;
        int32_t *cnt = b.counters + kFwdCounters + t.gsub_seg0.size();
        hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, s, cnt, 2);
        TimerScope tm(s, TIMER_GRAD32);
        if (n2 > 0) launch_grad_lattice_mfma<2, 2>(s, b.mitems, n2, cnt, b, q, amp, dL_dI);
        if (n3 > 0) launch_grad_lattice_mfma<3, 1>(s, b.mitems + n2, n3, cnt + 1, b, q, amp, dL_dI);
        tm.end(t.mwork);
        XS_HIP(hipGetLastError());
    }
    if (t.max_slots_seg > 0) {
        hipLaunchKernelGGL(k_grad_combine, dim3((t.max_slots_seg + kBlock - 1) / kBlock, n_seg), dim3(kBlock), 0,
                           s, b.gsegs, b.gpart, b.tile_atom, f, g32, g64);
        XS_HIP(hipGetLastError());
    }
    return XS_OK;
}

// ---------------------------------------------------------------- one-shot calls

xs_status fp32c_forward(hipStream_t s, const Segment *segs, int n_segs, const double *box,
                        const double *pos, const double *f, const double *q, double *I,
                        double *amp, const xs_tile_shape &fsh, const xs_tile_shape &gsh) {
    if (n_segs <= 0) return XS_OK;
    Plan p;
    p.with_grad = false;
    XS_TRY(p.build(segs, n_segs, box, fsh, gsh));
    XS_TRY(p.allocate(s, false));
    XS_TRY(p.sort_pixels(s, q));
    XS_TRY(p.tile_atoms(s, pos, f));
    return p.forward(s, q, I, amp);
}

xs_status fp32c_grad(hipStream_t s, const Segment *segs, int n_segs, const double *box,
                     const double *pos, const double *f, const double *q, const double *amp,
                     const double *dL_dI, float *dL_dr, double *dL_dr64, const xs_tile_shape &fsh,
                     const xs_tile_shape &gsh) {
    if (n_segs <= 0) return XS_OK;
    Plan p;
    XS_TRY(p.build(segs, n_segs, box, fsh, gsh));
    XS_TRY(p.allocate(s, false));
    XS_TRY(p.sort_pixels(s, q));
    XS_TRY(p.tile_atoms(s, pos, f));
    return p.grad(s, q, f, amp, dL_dI, dL_dr, dL_dr64);
}

}  // namespace xs
