// FP32 compensated (FP32C) form of the direct method and of its position
// gradient, for batches of systems and frames in one persistent launch.
//
// Sec. 3.1 (Algorithm 1): every pixel's amplitude is an independent sum over
// atoms, p^e(q) = sum_j f_j exp(-i q.r_j) (Eq. (pe_ri)), I = |p^e|^2 (Eq. (Iq_pq)).
// The GPU form keeps the phase accurate in large boxes by splitting it:
//   q.r_j / (2 pi) = q_rev . o_k  +  q_rev . d_j,        d_j = r_j - o_k,
// where o_k is the centre of a compact spatial tile of atoms.  The first term
// is reduced modulo one revolution in FP64 once per (pixel, tile); the second
// is small (|d_j| <~ 10 Angstrom) and runs in FP32 together with the hardware
// sine and cosine (v_sin_f32 / v_cos_f32 take revolutions) and the tile
// partial sums, which are folded into FP64 after every tile.
//
// Pipeline per call:
//   binning   (per segment = system x frame)  Morton cell key -> counting sort
//             -> per-cell index sort (deterministic) -> tiles of 64 atoms with
//             FP64 origin and FP32 (d, f), zero-padded;
//   pair sum  persistent work queue over (segment, pixel tile, atom chunk),
//             largest items first; partial amplitudes in FP64 per chunk;
//   combine   chunks summed in fixed order -> amplitude and intensity.
// The gradient uses the same tiles; see k_grad_fp32c.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "xs_internal.h"

namespace xs {
namespace {

constexpr int kTile = 64;        // atoms per spatial tile (one wavefront)
constexpr int kBlock = 256;      // threads per workgroup (4 wavefronts)
constexpr int kWaves = kBlock / 64;
constexpr double kInvTwoPi = 0x1.45f306dc9c883p-3;  // RN(1/(2 pi))

// ---------------------------------------------------------------- tables

struct BinSeg {            // binning view of one segment
    int64_t pos;           // atom offset of the frame in pos
    int64_t f;             // offset into f
    int64_t atom0;         // offset of this segment's atoms in key / sorted arrays
    int64_t key0;          // offset of this segment's cells in the histogram
    int64_t tile0;         // first tile of this segment
    double lo[3];          // binning box origin (0)
    double inv_cell[3];    // cells per Angstrom
    int32_t ncell[3];      // cells per dimension (power of two)
    int32_t bits;          // Morton bits per dimension
    int32_t n_atoms;
    int32_t n_tiles;
};

struct FwdSeg {            // pair-sum view of one segment
    int64_t q;             // pixel offset into q
    int64_t out;           // pixel offset into outputs
    int64_t part;          // offset (pixels) of this segment's partials: chunk c at part + c*n_q
    int64_t tile0;
    int32_t n_q;
    int32_t n_tiles;
    int32_t n_chunks;
    int32_t pad;
};

struct FwdItem {
    int32_t seg;
    int32_t p0;            // first pixel
    int32_t t0;            // first tile
    int32_t nt;            // tiles in this chunk
    int32_t chunk;
    int32_t pad;
};

struct GradSeg {
    int64_t q;             // pixel offset into q / prepared pixel data
    int64_t out;           // pixel offset into amp / dL_dI
    int64_t pos;           // atom offset in pos (for outputs)
    int64_t f;             // offset into f
    int64_t tile0;
    int64_t part;          // offset (atom slots) of partials: chunk c at part + c*n_tiles*64
    int32_t n_q;
    int32_t n_tiles;
    int32_t n_chunks;
    int32_t pad;
};

struct GradItem {
    int32_t seg;
    int32_t t0;            // first tile of this group
    int32_t nt;            // tiles in the group (<= kWaves * AL)
    int32_t p0;            // first pixel of the chunk
    int32_t np;            // pixels in the chunk
    int32_t chunk;
};

// Morton interleave of three 10-bit coordinates.
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// ---------------------------------------------------------------- binning

__global__ __launch_bounds__(kBlock) void k_bin_key(const BinSeg *__restrict__ segs,
                                                    const double *__restrict__ pos,
                                                    uint32_t *__restrict__ keys,
                                                    int32_t *__restrict__ hist) {
    const BinSeg sg = segs[blockIdx.y];
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= sg.n_atoms) return;
    const double *r = pos + (sg.pos + j) * 3;
    uint32_t c[3];
    for (int d = 0; d < 3; ++d) {
        double x = (r[d] - sg.lo[d]) * sg.inv_cell[d];
        int ci = static_cast<int>(__builtin_floor(x));
        ci = ci < 0 ? 0 : (ci >= sg.ncell[d] ? sg.ncell[d] - 1 : ci);
        if (!(x == x)) ci = 0;  // NaN positions land in cell 0
        c[d] = static_cast<uint32_t>(ci);
    }
    const uint32_t key = spread3(c[0]) | (spread3(c[1]) << 1) | (spread3(c[2]) << 2);
    keys[sg.atom0 + j] = key;
    atomicAdd(&hist[sg.key0 + key], 1);
}

// Exclusive scan of each segment's cell histogram; start[] keeps the cell
// starts, hist[] becomes the scatter cursor.  One block per segment.
__global__ __launch_bounds__(1024) void k_bin_scan(const BinSeg *__restrict__ segs,
                                                   int32_t *__restrict__ hist,
                                                   int32_t *__restrict__ start) {
    const BinSeg sg = segs[blockIdx.x];
    const int64_t nk = int64_t(1) << (3 * sg.bits);
    __shared__ int32_t part[1024];
    const int64_t per = (nk + 1023) / 1024;
    const int64_t a = threadIdx.x * per, b = (a + per < nk) ? a + per : nk;
    int32_t s = 0;
    for (int64_t i = a; i < b; ++i) s += hist[sg.key0 + i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int i = 0; i < 1024; ++i) {
            const int32_t v = part[i];
            part[i] = run;
            run += v;
        }
    }
    __syncthreads();
    int32_t run = part[threadIdx.x];
    for (int64_t i = a; i < b; ++i) {
        const int32_t v = hist[sg.key0 + i];
        start[sg.key0 + i] = run;
        hist[sg.key0 + i] = run;
        run += v;
    }
}

__global__ __launch_bounds__(kBlock) void k_bin_scatter(const BinSeg *__restrict__ segs,
                                                        const uint32_t *__restrict__ keys,
                                                        int32_t *__restrict__ cursor,
                                                        int32_t *__restrict__ sorted) {
    const BinSeg sg = segs[blockIdx.y];
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= sg.n_atoms) return;
    const int32_t slot = atomicAdd(&cursor[sg.key0 + keys[sg.atom0 + j]], 1);
    sorted[sg.atom0 + slot] = j;
}

// Restore a deterministic order: each cell's atoms ascending by index.
// After the scatter, cursor[c] is the end of cell c and start[c] its start.
__global__ __launch_bounds__(kBlock) void k_bin_sort_cells(const BinSeg *__restrict__ segs,
                                                           const int32_t *__restrict__ start,
                                                           const int32_t *__restrict__ end,
                                                           int32_t *__restrict__ sorted) {
    const BinSeg sg = segs[blockIdx.y];
    const int64_t c = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (c >= (int64_t(1) << (3 * sg.bits))) return;
    int32_t *v = sorted + sg.atom0;
    const int32_t a = start[sg.key0 + c], b = end[sg.key0 + c];
    for (int32_t i = a + 1; i < b; ++i) {
        const int32_t x = v[i];
        int32_t k = i - 1;
        while (k >= a && v[k] > x) {
            v[k + 1] = v[k];
            --k;
        }
        v[k + 1] = x;
    }
}

// One wavefront per tile: bounding-box centre as origin (FP64), offsets and
// form factors in FP32, zero padding past the segment's last atom.
__global__ __launch_bounds__(kBlock) void k_bin_tiles(const BinSeg *__restrict__ segs,
                                                      const double *__restrict__ pos,
                                                      const double *__restrict__ f,
                                                      const int32_t *__restrict__ sorted,
                                                      float4 *__restrict__ tiles,
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
        r[0] = rp[0]; r[1] = rp[1]; r[2] = rp[2];
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
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (real)
        v = make_float4(static_cast<float>(r[0] - o[0]), static_cast<float>(r[1] - o[1]),
                        static_cast<float>(r[2] - o[2]), static_cast<float>(f[sg.f + j]));
    tiles[ti * kTile + lane] = v;
    tile_atom[ti * kTile + lane] = j;
    if (lane == 0) origins[ti] = make_double4(o[0], o[1], o[2], 0.0);
}

__global__ void k_reset_counter(int32_t *counter, int n) {
    if (threadIdx.x < n) counter[threadIdx.x] = 0;
}

// Zero fill (used instead of hipMemsetAsync so the sequence stays capturable).
__global__ __launch_bounds__(kBlock) void k_zero_i32(int32_t *__restrict__ p, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------- forward pair sum
//
// Workgroup = 4 wavefronts x 64 lanes; lane owns QL pixels (p0 + k*256 + tid).
// Atom tiles of the item's chunk are staged 4 at a time into LDS (double
// buffered) and read back as broadcasts.  Per (pixel, tile): FP64 base phase
// theta = frac(q_rev . o).  Per pair: phi = theta + q_rev . d (3 FMA, FP32),
// v_sin/v_cos, 2 FMA.  Tile partials fold into FP64.
template <int QL>
__global__ __launch_bounds__(kBlock) void k_forward_fp32c(
    const FwdItem *__restrict__ items, int32_t n_items, int32_t *__restrict__ counter,
    const FwdSeg *__restrict__ segs, const double *__restrict__ q,
    const float4 *__restrict__ tiles, const double4 *__restrict__ origins,
    double2 *__restrict__ partial) {
    __shared__ float4 s_atoms[2][kWaves * kTile];
    __shared__ double4 s_orig[2][kWaves];
    __shared__ int32_t s_item;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int32_t it = s_item;
        __syncthreads();  // everyone has read s_item before it is rewritten
        if (it >= n_items) break;
        const FwdItem item = items[it];
        const FwdSeg sg = segs[item.seg];
        // lane pixels
        float qx[QL], qy[QL], qz[QL];
        double dx[QL], dy[QL], dz[QL];
        double re64[QL], im64[QL];
#pragma unroll
        for (int k = 0; k < QL; ++k) {
            int p = item.p0 + k * kBlock + tid;
            p = p < sg.n_q ? p : sg.n_q - 1;
            const double *qp = q + (sg.q + p) * 3;
            dx[k] = qp[0] * kInvTwoPi;
            dy[k] = qp[1] * kInvTwoPi;
            dz[k] = qp[2] * kInvTwoPi;
            qx[k] = static_cast<float>(dx[k]);
            qy[k] = static_cast<float>(dy[k]);
            qz[k] = static_cast<float>(dz[k]);
            re64[k] = 0.0;
            im64[k] = 0.0;
        }
        const int64_t tbase = sg.tile0 + item.t0;
        // stage group 0
        const int n_groups = (item.nt + kWaves - 1) / kWaves;
        {
            const int tt = tid / kTile;
            if (tt < item.nt) s_atoms[0][tid] = tiles[(tbase + tt) * kTile + (tid & (kTile - 1))];
            if (tid < kWaves && tid < item.nt) s_orig[0][tid] = origins[tbase + tid];
        }
        __syncthreads();
        for (int g = 0; g < n_groups; ++g) {
            const int buf = g & 1;
            // prefetch the next group into registers, store after computing
            float4 nxt = make_float4(0.f, 0.f, 0.f, 0.f);
            double4 nxo = make_double4(0.0, 0.0, 0.0, 0.0);
            const int ng = g + 1;
            const bool have_next = ng < n_groups;
            if (have_next) {
                const int tt = ng * kWaves + tid / kTile;
                if (tt < item.nt) nxt = tiles[(tbase + tt) * kTile + (tid & (kTile - 1))];
                if (tid < kWaves && ng * kWaves + tid < item.nt) nxo = origins[tbase + ng * kWaves + tid];
            }
            const int tiles_here = min(kWaves, item.nt - g * kWaves);
            for (int w = 0; w < tiles_here; ++w) {
                const double4 o = s_orig[buf][w];
                float th[QL], re[QL], im[QL];
#pragma unroll
                for (int k = 0; k < QL; ++k) {
                    const double t = __builtin_fma(dz[k], o.z, __builtin_fma(dy[k], o.y, dx[k] * o.x));
                    th[k] = static_cast<float>(t - __builtin_rint(t));
                    re[k] = 0.f;
                    im[k] = 0.f;
                }
                const float4 *at = &s_atoms[buf][w * kTile];
#pragma unroll 4
                for (int j = 0; j < kTile; ++j) {
                    const float4 a = at[j];
#pragma unroll
                    for (int k = 0; k < QL; ++k) {
                        const float ph = __builtin_fmaf(qz[k], a.z, __builtin_fmaf(qy[k], a.y,
                                                        __builtin_fmaf(qx[k], a.x, th[k])));
                        const float sn = __builtin_amdgcn_sinf(ph);
                        const float cs = __builtin_amdgcn_cosf(ph);
                        re[k] = __builtin_fmaf(a.w, cs, re[k]);
                        im[k] = __builtin_fmaf(a.w, sn, im[k]);
                    }
                }
#pragma unroll
                for (int k = 0; k < QL; ++k) {
                    re64[k] += static_cast<double>(re[k]);
                    im64[k] += static_cast<double>(im[k]);
                }
            }
            if (have_next) {
                s_atoms[buf ^ 1][tid] = nxt;
                if (tid < kWaves) s_orig[buf ^ 1][tid] = nxo;
            }
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < QL; ++k) {
            const int p = item.p0 + k * kBlock + tid;
            if (p < sg.n_q)
                partial[sg.part + static_cast<int64_t>(item.chunk) * sg.n_q + p] =
                    make_double2(re64[k], im64[k]);
        }
    }
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
    double a = 0.0, sb = 0.0;
    for (int c = 0; c < sg.n_chunks; ++c) {
        const double2 v = partial[sg.part + static_cast<int64_t>(c) * sg.n_q + p];
        a += v.x;
        sb += v.y;
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
// Pixel prologue: FP32 (q_rev, W) and FP64 (q_rev, psi).
__global__ __launch_bounds__(kBlock) void k_grad_prep(const GradSeg *__restrict__ segs,
                                                      const double *__restrict__ q,
                                                      const double *__restrict__ amp,
                                                      const double *__restrict__ w,
                                                      float4 *__restrict__ pq32,
                                                      float4 *__restrict__ pw32,
                                                      double4 *__restrict__ pq64) {
    const GradSeg sg = segs[blockIdx.y];
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= sg.n_q) return;
    const double *qp = q + (sg.q + p) * 3;
    const double a = amp[2 * (sg.out + p)], b = amp[2 * (sg.out + p) + 1];
    const double mag = __builtin_sqrt(a * a + b * b);
    const double psi = atan2(b, a) * kInvTwoPi;
    const double c = -2.0 * w[sg.out + p] * mag;
    const double rx = qp[0] * kInvTwoPi, ry = qp[1] * kInvTwoPi, rz = qp[2] * kInvTwoPi;
    const int64_t i = sg.q + p;
    pq32[i] = make_float4(static_cast<float>(rx), static_cast<float>(ry), static_cast<float>(rz), 0.f);
    pw32[i] = make_float4(static_cast<float>(c * qp[0]), static_cast<float>(c * qp[1]),
                          static_cast<float>(c * qp[2]), 0.f);
    pq64[i] = make_double4(rx, ry, rz, psi);
}

// Workgroup = 4 wavefronts; wavefront w owns tiles t0 + w*AL + a (a < AL),
// lane l owns atom l of each.  Pixels of the item's chunk are staged 64 at a
// time into LDS; each wavefront also stages its base phases
// theta'(p, tile) = frac(q_rev.o + psi) (FP64 -> FP32).  Per pair: 3 FMA phase,
// one v_sin, 3 FMA accumulate.  Pixel sub-chunk partials fold into FP64.
constexpr int kPixStage = 64;
template <int AL>
__global__ __launch_bounds__(kBlock) void k_grad_fp32c(
    const GradItem *__restrict__ items, int32_t n_items, int32_t *__restrict__ counter,
    const GradSeg *__restrict__ segs, const float4 *__restrict__ tiles,
    const double4 *__restrict__ origins, const float4 *__restrict__ pq32,
    const float4 *__restrict__ pw32, const double4 *__restrict__ pq64,
    double *__restrict__ gpart) {
    __shared__ float4 s_q[kPixStage];
    __shared__ float4 s_w[kPixStage];
    __shared__ float s_th[kWaves][AL][kPixStage];
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
        double ox[AL], oy[AL], oz[AL];
        double gx64[AL], gy64[AL], gz64[AL];
#pragma unroll
        for (int a = 0; a < AL; ++a) {
            int t = wave * AL + a;
            const bool real = t < item.nt;
            t = real ? t : 0;
            const int64_t ti = sg.tile0 + item.t0 + t;
            const float4 v = tiles[ti * kTile + lane];
            const double4 o = origins[ti];
            dx[a] = v.x; dy[a] = v.y; dz[a] = v.z;
            ox[a] = o.x; oy[a] = o.y; oz[a] = o.z;
            gx64[a] = gy64[a] = gz64[a] = 0.0;
        }
        for (int s0 = 0; s0 < item.np; s0 += kPixStage) {
            const int n_here = min(kPixStage, item.np - s0);
            // stage pixel data (wave 0) and each wave's base phases
            {
                int p = item.p0 + s0 + lane;
                const bool real = lane < n_here;
                p = real ? p : item.p0;
                const int64_t i = sg.q + p;
                if (wave == 0) {
                    s_q[lane] = pq32[i];
                    s_w[lane] = real ? pw32[i] : make_float4(0.f, 0.f, 0.f, 0.f);
                }
                const double4 d = pq64[i];
#pragma unroll
                for (int a = 0; a < AL; ++a) {
                    const double t = __builtin_fma(d.z, oz[a], __builtin_fma(d.y, oy[a], d.x * ox[a])) + d.w;
                    s_th[wave][a][lane] = static_cast<float>(t - __builtin_rint(t));
                }
            }
            __syncthreads();
            float gx[AL], gy[AL], gz[AL];
#pragma unroll
            for (int a = 0; a < AL; ++a) gx[a] = gy[a] = gz[a] = 0.f;
#pragma unroll 2
            for (int m = 0; m < kPixStage; ++m) {
                const float4 qv = s_q[m];
                const float4 wv = s_w[m];
#pragma unroll
                for (int a = 0; a < AL; ++a) {
                    const float ph = __builtin_fmaf(qv.z, dz[a], __builtin_fmaf(qv.y, dy[a],
                                                    __builtin_fmaf(qv.x, dx[a], s_th[wave][a][m])));
                    const float sn = __builtin_amdgcn_sinf(ph);
                    gx[a] = __builtin_fmaf(wv.x, sn, gx[a]);
                    gy[a] = __builtin_fmaf(wv.y, sn, gy[a]);
                    gz[a] = __builtin_fmaf(wv.z, sn, gz[a]);
                }
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
    double gx = 0.0, gy = 0.0, gz = 0.0;
    for (int c = 0; c < sg.n_chunks; ++c) {
        const int64_t s = sg.part + static_cast<int64_t>(c) * sg.n_tiles * kTile + slot;
        gx += gpart[3 * s];
        gy += gpart[3 * s + 1];
        gz += gpart[3 * s + 2];
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

int device_slots(const void *kernel) {
    static std::mutex mu;
    static std::vector<std::pair<std::pair<const void *, int>, int>> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(mu);
    for (auto &e : cache)
        if (e.first.first == kernel && e.first.second == dev) return e.second;
    int cus = 0, per = 1;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kBlock, 0);
    const int n = std::max(1, cus) * std::max(1, per);
    cache.emplace_back(std::make_pair(kernel, dev), n);
    return n;
}

struct Binned {
    std::vector<BinSeg> bsegs;
    int64_t total_tiles = 0;
    float4 *tiles = nullptr;
    double4 *origins = nullptr;
    int32_t *tile_atom = nullptr;
};

// Bin every segment into tiles (see k_bin_*).  Cells target kTile/8 atoms so a
// tile of 64 Morton-consecutive atoms spans about 2x2x2 cells.
xs_status bin_segments(hipStream_t s, const Segment *segs, int n_segs, const double *box,
                       const double *pos, const double *f, Binned &out) {
    out.bsegs.resize(n_segs);
    int64_t atom0 = 0, key0 = 0, tile0 = 0;
    int max_atoms = 0, max_tiles = 0;
    int64_t max_keys = 0;
    for (int i = 0; i < n_segs; ++i) {
        const Segment &sg = segs[i];
        BinSeg &b = out.bsegs[i];
        b.pos = sg.pos;
        b.f = sg.f;
        b.n_atoms = sg.n_atoms;
        b.n_tiles = (sg.n_atoms + kTile - 1) / kTile;
        b.atom0 = atom0;
        b.key0 = key0;
        b.tile0 = tile0;
        const double *L = box + 3 * sg.sys;
        const double vol = std::max(L[0] * L[1] * L[2], 1e-300);
        const double rho = sg.n_atoms / vol;
        const double edge = std::cbrt((kTile / 8.0) / std::max(rho, 1e-300));
        int bits = 0;
        for (int d = 0; d < 3; ++d) {
            int nc = static_cast<int>(std::lround(L[d] / edge));
            nc = std::max(1, std::min(nc, 1024));
            int bb = 0;
            while ((1 << bb) < nc) ++bb;
            bits = std::max(bits, bb);
        }
        bits = std::min(bits, 7);  // at most 2^21 cells per segment
        for (int d = 0; d < 3; ++d) {
            b.lo[d] = 0.0;
            b.ncell[d] = 1 << bits;
            b.inv_cell[d] = L[d] > 0 ? (1 << bits) / L[d] : 0.0;
        }
        b.bits = bits;
        atom0 += sg.n_atoms;
        key0 += int64_t(1) << (3 * bits);
        tile0 += b.n_tiles;
        max_atoms = std::max(max_atoms, sg.n_atoms);
        max_tiles = std::max(max_tiles, b.n_tiles);
        max_keys = std::max<int64_t>(max_keys, int64_t(1) << (3 * bits));
    }
    out.total_tiles = tile0;
    void *d_b = nullptr, *keys = nullptr, *hist = nullptr, *sorted = nullptr, *tiles = nullptr,
         *orig = nullptr;
    XS_TRY(upload(s, SLOT_ITEMS, out.bsegs.data(), sizeof(BinSeg) * n_segs, &d_b));
    XS_TRY(scratch(s, SLOT_KEYS, sizeof(uint32_t) * std::max<int64_t>(atom0, 1), &keys));
    XS_TRY(scratch(s, SLOT_HIST, sizeof(int32_t) * 2 * std::max<int64_t>(key0, 1), &hist));
    XS_TRY(scratch(s, SLOT_SORTED, sizeof(int32_t) * std::max<int64_t>(atom0, 1), &sorted));
    XS_TRY(scratch(s, SLOT_TILES, (sizeof(float4) + sizeof(int32_t)) * kTile * std::max<int64_t>(tile0, 1), &tiles));
    XS_TRY(scratch(s, SLOT_ORIGINS, sizeof(double4) * std::max<int64_t>(tile0, 1), &orig));
    int32_t *h = static_cast<int32_t *>(hist);
    int32_t *start = h + key0;
    if (key0 > 0)
        hipLaunchKernelGGL(k_zero_i32, dim3(static_cast<unsigned>((key0 + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                           h, key0);
    const BinSeg *db = static_cast<const BinSeg *>(d_b);
    if (max_atoms > 0) {
        dim3 ga((max_atoms + kBlock - 1) / kBlock, n_segs);
        hipLaunchKernelGGL(k_bin_key, ga, dim3(kBlock), 0, s, db, pos, static_cast<uint32_t *>(keys), h);
        hipLaunchKernelGGL(k_bin_scan, dim3(n_segs), dim3(1024), 0, s, db, h, start);
        hipLaunchKernelGGL(k_bin_scatter, ga, dim3(kBlock), 0, s, db,
                           static_cast<const uint32_t *>(keys), h, static_cast<int32_t *>(sorted));
        dim3 gc(static_cast<unsigned>((max_keys + kBlock - 1) / kBlock), n_segs);
        hipLaunchKernelGGL(k_bin_sort_cells, gc, dim3(kBlock), 0, s, db, start, h,
                           static_cast<int32_t *>(sorted));
        dim3 gt((max_tiles + kWaves - 1) / kWaves, n_segs);
        out.tiles = static_cast<float4 *>(tiles);
        out.tile_atom = reinterpret_cast<int32_t *>(static_cast<float4 *>(tiles) + kTile * std::max<int64_t>(tile0, 1));
        out.origins = static_cast<double4 *>(orig);
        hipLaunchKernelGGL(k_bin_tiles, gt, dim3(kBlock), 0, s, db, pos, f,
                           static_cast<const int32_t *>(sorted), out.tiles, out.origins, out.tile_atom);
        XS_HIP(hipGetLastError());
    } else {
        out.tiles = static_cast<float4 *>(tiles);
        out.tile_atom = reinterpret_cast<int32_t *>(static_cast<float4 *>(tiles) + kTile);
        out.origins = static_cast<double4 *>(orig);
    }
    return XS_OK;
}

template <int QL>
void launch_forward(hipStream_t s, int slots, const FwdItem *items, int n_items, int32_t *counter,
                    const FwdSeg *segs, const double *q, const Binned &b, double2 *partial) {
    hipLaunchKernelGGL(k_forward_fp32c<QL>, dim3(slots), dim3(kBlock), 0, s, items, n_items, counter,
                       segs, q, b.tiles, b.origins, partial);
}

template <int AL>
void launch_grad(hipStream_t s, int slots, const GradItem *items, int n_items, int32_t *counter,
                 const GradSeg *segs, const Binned &b, const float4 *pq32, const float4 *pw32,
                 const double4 *pq64, double *gpart) {
    hipLaunchKernelGGL(k_grad_fp32c<AL>, dim3(slots), dim3(kBlock), 0, s, items, n_items, counter,
                       segs, b.tiles, b.origins, pq32, pw32, pq64, gpart);
}

}  // namespace

xs_status fp32c_forward(hipStream_t s, const Segment *segs, int n_segs, const double *box,
                        const double *pos, const double *f, const double *q, double *I,
                        double *amp, const xs_tile_shape &shape) {
    if (n_segs <= 0) return XS_OK;
    Binned b;
    XS_TRY(bin_segments(s, segs, n_segs, box, pos, f, b));
    const int QL = shape.q_per_lane;
    const int split = std::max(1, shape.atom_split);
    const int pix_per_item = kBlock * QL;
    std::vector<FwdSeg> fs(n_segs);
    std::vector<FwdItem> items;
    std::vector<int64_t> cost;
    int64_t part = 0;
    int max_q = 0;
    for (int i = 0; i < n_segs; ++i) {
        FwdSeg &g = fs[i];
        g.q = segs[i].q;
        g.out = segs[i].out;
        g.tile0 = b.bsegs[i].tile0;
        g.n_q = segs[i].n_q;
        g.n_tiles = b.bsegs[i].n_tiles;
        g.n_chunks = g.n_tiles > 0 ? (g.n_tiles + split - 1) / split : 0;
        g.part = part;
        g.pad = 0;
        part += static_cast<int64_t>(g.n_chunks) * g.n_q;
        max_q = std::max(max_q, g.n_q);
        for (int p0 = 0; p0 < g.n_q; p0 += pix_per_item)
            for (int c = 0; c < g.n_chunks; ++c) {
                FwdItem it;
                it.seg = i;
                it.p0 = p0;
                it.t0 = c * split;
                it.nt = std::min(split, g.n_tiles - c * split);
                it.chunk = c;
                it.pad = 0;
                items.push_back(it);
            }
    }
    // largest work first (pixels x tiles), stable for equal cost
    std::vector<int> order(items.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = static_cast<int>(i);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        const int64_t cx = static_cast<int64_t>(std::min(pix_per_item, fs[items[x].seg].n_q - items[x].p0)) * items[x].nt;
        const int64_t cy = static_cast<int64_t>(std::min(pix_per_item, fs[items[y].seg].n_q - items[y].p0)) * items[y].nt;
        return cx > cy;
    });
    std::vector<FwdItem> sorted_items(items.size());
    for (size_t i = 0; i < order.size(); ++i) sorted_items[i] = items[order[i]];
    void *d_fs = nullptr, *d_items = nullptr, *d_part = nullptr, *d_cnt = nullptr;
    XS_TRY(upload(s, SLOT_SEGS, fs.data(), sizeof(FwdSeg) * n_segs, &d_fs));
    XS_TRY(scratch(s, SLOT_PARTIAL, sizeof(double2) * std::max<int64_t>(part, 1), &d_part));
    XS_TRY(scratch(s, SLOT_COUNTER, 256, &d_cnt));
    if (!sorted_items.empty()) {
        XS_TRY(upload(s, SLOT_PIXEL, sorted_items.data(), sizeof(FwdItem) * sorted_items.size(), &d_items));
        hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, static_cast<int32_t *>(d_cnt), 1);
        const FwdItem *it = static_cast<const FwdItem *>(d_items);
        const FwdSeg *sg = static_cast<const FwdSeg *>(d_fs);
        int32_t *cnt = static_cast<int32_t *>(d_cnt);
        double2 *pp = static_cast<double2 *>(d_part);
        const int n = static_cast<int>(sorted_items.size());
        switch (QL) {
        case 1: launch_forward<1>(s, std::min(n, device_slots((const void *)k_forward_fp32c<1>)), it, n, cnt, sg, q, b, pp); break;
        case 2: launch_forward<2>(s, std::min(n, device_slots((const void *)k_forward_fp32c<2>)), it, n, cnt, sg, q, b, pp); break;
        case 4: launch_forward<4>(s, std::min(n, device_slots((const void *)k_forward_fp32c<4>)), it, n, cnt, sg, q, b, pp); break;
        case 8: launch_forward<8>(s, std::min(n, device_slots((const void *)k_forward_fp32c<8>)), it, n, cnt, sg, q, b, pp); break;
        default: return set_error(XS_EINVAL, "q_per_lane must be 1, 2, 4 or 8 (got %d)", QL);
        }
        XS_HIP(hipGetLastError());
    }
    if (max_q > 0) {
        hipLaunchKernelGGL(k_forward_combine, dim3((max_q + kBlock - 1) / kBlock, n_segs), dim3(kBlock), 0,
                           s, static_cast<const FwdSeg *>(d_fs), static_cast<const double2 *>(d_part), I,
                           amp);
        XS_HIP(hipGetLastError());
    }
    return XS_OK;
}

xs_status fp32c_grad(hipStream_t s, const Segment *segs, int n_segs, const double *box,
                     const double *pos, const double *f, const double *q, const double *amp,
                     const double *dL_dI, float *dL_dr, double *dL_dr64,
                     const xs_tile_shape &shape) {
    if (n_segs <= 0) return XS_OK;
    Binned b;
    XS_TRY(bin_segments(s, segs, n_segs, box, pos, f, b));
    const int AL = shape.q_per_lane;
    const int group = kWaves * AL;  // tiles per workgroup item
    int pchunk = std::max(kPixStage, (shape.pixel_split / kPixStage) * kPixStage);
    std::vector<GradSeg> gs(n_segs);
    std::vector<GradItem> items;
    int64_t part = 0, pix = 0;
    int max_q = 0, max_slots = 0;
    // the prepared pixel arrays are indexed by the segment's q offset; frames of
    // one system share q, so allocate over the largest q offset used
    for (int i = 0; i < n_segs; ++i) pix = std::max<int64_t>(pix, segs[i].q + segs[i].n_q);
    for (int i = 0; i < n_segs; ++i) {
        GradSeg &g = gs[i];
        g.q = segs[i].q;
        g.out = segs[i].out;
        g.pos = segs[i].pos;
        g.f = segs[i].f;
        g.tile0 = b.bsegs[i].tile0;
        g.n_q = segs[i].n_q;
        g.n_tiles = b.bsegs[i].n_tiles;
        g.n_chunks = g.n_q > 0 ? (g.n_q + pchunk - 1) / pchunk : 0;
        g.part = part;
        g.pad = 0;
        part += static_cast<int64_t>(g.n_chunks) * g.n_tiles * kTile;
        max_q = std::max(max_q, g.n_q);
        max_slots = std::max(max_slots, g.n_tiles * kTile);
        for (int t0 = 0; t0 < g.n_tiles; t0 += group)
            for (int c = 0; c < g.n_chunks; ++c) {
                GradItem it;
                it.seg = i;
                it.t0 = t0;
                it.nt = std::min(group, g.n_tiles - t0);
                it.p0 = c * pchunk;
                it.np = std::min(pchunk, g.n_q - c * pchunk);
                it.chunk = c;
                items.push_back(it);
            }
    }
    std::vector<int> order(items.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = static_cast<int>(i);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return static_cast<int64_t>(items[x].nt) * items[x].np > static_cast<int64_t>(items[y].nt) * items[y].np;
    });
    std::vector<GradItem> sorted_items(items.size());
    for (size_t i = 0; i < order.size(); ++i) sorted_items[i] = items[order[i]];
    void *d_gs = nullptr, *d_items = nullptr, *d_part = nullptr, *d_cnt = nullptr, *d_pix = nullptr;
    XS_TRY(upload(s, SLOT_SEGS, gs.data(), sizeof(GradSeg) * n_segs, &d_gs));
    XS_TRY(scratch(s, SLOT_PARTIAL, sizeof(double) * 3 * std::max<int64_t>(part, 1), &d_part));
    XS_TRY(scratch(s, SLOT_COUNTER, 256, &d_cnt));
    XS_TRY(scratch(s, SLOT_PIXEL2, (2 * sizeof(float4) + sizeof(double4)) * std::max<int64_t>(pix, 1), &d_pix));
    float4 *pq32 = static_cast<float4 *>(d_pix);
    float4 *pw32 = pq32 + std::max<int64_t>(pix, 1);
    double4 *pq64 = reinterpret_cast<double4 *>(pw32 + std::max<int64_t>(pix, 1));
    const GradSeg *dgs = static_cast<const GradSeg *>(d_gs);
    double *gp = static_cast<double *>(d_part);
    // The pixel prologue depends on the frame (amp, dL/dI), so segments run
    // one prologue + pair sum at a time when frames share pixel offsets.
    // Group segments whose q ranges do not overlap into one launch.
    int i0 = 0;
    while (i0 < n_segs) {
        int i1 = i0 + 1;
        // extend while the q range is new
        for (; i1 < n_segs; ++i1) {
            bool clash = false;
            for (int k = i0; k < i1 && !clash; ++k)
                clash = !(segs[i1].q + segs[i1].n_q <= segs[k].q || segs[k].q + segs[k].n_q <= segs[i1].q);
            if (clash) break;
        }
        int mq = 0;
        for (int k = i0; k < i1; ++k) mq = std::max(mq, segs[k].n_q);
        if (mq > 0) {
            hipLaunchKernelGGL(k_grad_prep, dim3((mq + kBlock - 1) / kBlock, i1 - i0), dim3(kBlock), 0, s,
                               dgs + i0, q, amp, dL_dI, pq32, pw32, pq64);
        }
        std::vector<GradItem> sub;
        for (auto &it : sorted_items)
            if (it.seg >= i0 && it.seg < i1) sub.push_back(it);
        if (!sub.empty()) {
            XS_TRY(upload(s, SLOT_ITEMS, sub.data(), sizeof(GradItem) * sub.size(), &d_items));
            hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, static_cast<int32_t *>(d_cnt), 1);
            const GradItem *it = static_cast<const GradItem *>(d_items);
            int32_t *cnt = static_cast<int32_t *>(d_cnt);
            const int n = static_cast<int>(sub.size());
            switch (AL) {
            case 1: launch_grad<1>(s, std::min(n, device_slots((const void *)k_grad_fp32c<1>)), it, n, cnt, dgs, b, pq32, pw32, pq64, gp); break;
            case 2: launch_grad<2>(s, std::min(n, device_slots((const void *)k_grad_fp32c<2>)), it, n, cnt, dgs, b, pq32, pw32, pq64, gp); break;
            case 4: launch_grad<4>(s, std::min(n, device_slots((const void *)k_grad_fp32c<4>)), it, n, cnt, dgs, b, pq32, pw32, pq64, gp); break;
            case 8: launch_grad<8>(s, std::min(n, device_slots((const void *)k_grad_fp32c<8>)), it, n, cnt, dgs, b, pq32, pw32, pq64, gp); break;
            default: return set_error(XS_EINVAL, "q_per_lane must be 1, 2, 4 or 8 (got %d)", AL);
            }
            XS_HIP(hipGetLastError());
        }
        i0 = i1;
    }
    if (max_slots > 0) {
        hipLaunchKernelGGL(k_grad_combine, dim3((max_slots + kBlock - 1) / kBlock, n_segs), dim3(kBlock), 0, s,
                           dgs, static_cast<const double *>(d_part), b.tile_atom, f, dL_dr, dL_dr64);
        XS_HIP(hipGetLastError());
    }
    return XS_OK;
}

}  // namespace xs
