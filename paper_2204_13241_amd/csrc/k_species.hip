// q-dependent atomic form factors, one table per species (Sec. 2.1: the form
// factor of an element is well parameterized by a sum of Gaussians):
//     f_s(q) = c + sum_{i=1..4} a_i exp(-b_i s^2),  s = |q| / (4 pi),
// and the intensity of Eqs. (Iq_rij), (pe_ri) with f_j(q) = f_{species(j)}(q).
//
// The pair sum is split by species: p^e(q) = sum_s f_s(|q|) P_s(q) with
// P_s(q) = sum_{j in s} e^{-i q.r_j}, so each species is one more segment of the
// ordinary batched pair kernels (unit weights, the same pixels), and a small
// kernel combines the per-species amplitudes.  The adjoint runs the same split
// with per-pixel weights w_p f_s(|q_p|) and the total amplitude, then scatters
// the gradients back to the caller's atom order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "xs_internal.h"

namespace xs {
namespace {

constexpr int kBlock = 256;
constexpr double kPi = 3.14159265358979323846;

unsigned blocks_for(int64_t n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }

__global__ __launch_bounds__(kBlock) void k_fill_f64(double *__restrict__ p, int64_t n, double v) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

// f_s(|q|) from coef[s] = {a_1..a_4, b_1..b_4, c}; the terms are added to c in
// order i = 1..4; s^2 = (q.q) / (16 pi^2).
__device__ __forceinline__ double form_factor(const double *__restrict__ coef, double qq) {
    const double s2 = qq / (16.0 * kPi * kPi);
    double f = coef[8];
#pragma unroll
    for (int i = 0; i < 4; ++i) f = f + coef[i] * exp(-coef[4 + i] * s2);
    return f;
}

__device__ __forceinline__ double qdotq(const double *__restrict__ q, int64_t p) {
    const double x = q[3 * p], y = q[3 * p + 1], z = q[3 * p + 2];
    return __builtin_fma(z, z, __builtin_fma(y, y, x * x));
}

struct SpSeg {            // one (system, frame) segment of the caller's batch
    int64_t pos;          // atom offset of the frame (positions and gradients)
    int64_t perm;         // offset of the system's species order in perm
    int64_t q;            // pixel offset into q
    int64_t out;          // pixel offset into the caller's outputs
    int32_t n_atoms;
    int32_t n_q;
};

// Positions in species order: pos_r[seg.pos + k] = pos[seg.pos + perm[seg.perm + k]].
__global__ __launch_bounds__(kBlock) void k_species_gather(const SpSeg *__restrict__ segs,
                                                           const int32_t *__restrict__ perm,
                                                           const double *__restrict__ pos,
                                                           double *__restrict__ pos_r) {
    const SpSeg sg = segs[blockIdx.y];
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= sg.n_atoms) return;
    const int64_t src = sg.pos + perm[sg.perm + k], dst = sg.pos + k;
    for (int c = 0; c < 3; ++c) pos_r[3 * dst + c] = pos[3 * src + c];
}

// Gradients back to the caller's order: g[seg.pos + perm[k]] = g_r[seg.pos + k].
template <typename T>
__global__ __launch_bounds__(kBlock) void k_species_scatter(const SpSeg *__restrict__ segs,
                                                            const int32_t *__restrict__ perm,
                                                            const T *__restrict__ g_r, T *__restrict__ g) {
    const SpSeg sg = segs[blockIdx.y];
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= sg.n_atoms) return;
    const int64_t dst = sg.pos + perm[sg.perm + k], src = sg.pos + k;
    for (int c = 0; c < 3; ++c) g[3 * dst + c] = g_r[3 * src + c];
}

// p^e = sum_s f_s(|q|) P_s for s ascending (species without atoms skipped):
// re = fma(f, P.re, re), im = fma(f, P.im, im) from +0.0; I = fma(re, re, im*im).
// sub[seg * n_species + s]: pixel offset of species s's amplitudes, or -1.
__global__ __launch_bounds__(kBlock) void k_species_combine(const SpSeg *__restrict__ segs,
                                                            const int64_t *__restrict__ sub, int32_t n_species,
                                                            const double *__restrict__ coef,
                                                            const double *__restrict__ q,
                                                            const double2 *__restrict__ amp_s,
                                                            double *__restrict__ I, double2 *__restrict__ amp) {
    const SpSeg sg = segs[blockIdx.y];
    const int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (p >= sg.n_q) return;
    const double qq = qdotq(q, sg.q + p);
    double re = 0.0, im = 0.0;
    for (int s = 0; s < n_species; ++s) {
        const int64_t o = sub[static_cast<int64_t>(blockIdx.y) * n_species + s];
        if (o < 0) continue;
        const double f = form_factor(coef + 9 * s, qq);
        const double2 P = amp_s[o + p];
        re = __builtin_fma(f, P.x, re);
        im = __builtin_fma(f, P.y, im);
    }
    I[sg.out + p] = __builtin_fma(re, re, im * im);
    if (amp) amp[sg.out + p] = make_double2(re, im);
}

// Adjoint inputs of species segment k (parent segment par[k], species sp[k]):
// w_k[p] = dL/dI[p] * f_s(|q_p|) and the parent's total amplitude.
__global__ __launch_bounds__(kBlock) void k_species_weights(const SpSeg *__restrict__ segs,
                                                            const int32_t *__restrict__ par,
                                                            const int32_t *__restrict__ sp,
                                                            const int64_t *__restrict__ sub_out,
                                                            const double *__restrict__ coef,
                                                            const double *__restrict__ q,
                                                            const double *__restrict__ dL_dI,
                                                            const double2 *__restrict__ amp,
                                                            double *__restrict__ w, double2 *__restrict__ amp_r) {
    const int k = blockIdx.y;
    const SpSeg sg = segs[par[k]];
    const int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (p >= sg.n_q) return;
    const double f = form_factor(coef + 9 * sp[k], qdotq(q, sg.q + p));
    const int64_t o = sub_out[k] + p;
    w[o] = dL_dI[sg.out + p] * f;
    amp_r[o] = amp[sg.out + p];
}

// Host side: the species order of every system, the species segments and the
// device tables, all carved from the stream's scratch.
struct SpeciesSplit {
    std::vector<SpSeg> segs;          // caller's segments
    std::vector<Segment> sub;         // one per (segment, species with atoms)
    std::vector<int32_t> sub_par, sub_sp;
    std::vector<int64_t> sub_off;     // [n_seg][n_species] pixel offsets or -1
    std::vector<int64_t> sub_out;     // per species segment
    std::vector<int32_t> perm;        // species order per system (concatenated)
    int64_t n_pos = 0;                // atoms spanned by the positions
    int64_t total_q = 0;              // pixels over all species segments
    int max_sub_atoms = 0, max_q = 0, max_atoms = 0;
};

xs_status split_species(hipStream_t s, const std::vector<Segment> &segs, const int32_t *species,
                        int32_t n_species, SpeciesSplit &sp) {
    // the caller's species array has the layout of f: read the span every system uses
    int64_t span = 0;
    for (const Segment &g : segs) span = std::max<int64_t>(span, g.f + g.n_atoms);
    std::vector<int32_t> h(static_cast<size_t>(std::max<int64_t>(span, 1)));
    if (span > 0) {
        XS_HIP(hipMemcpyAsync(h.data(), species, sizeof(int32_t) * span, hipMemcpyDeviceToHost, s));
        XS_HIP(hipStreamSynchronize(s));
    }
    // one species order per distinct (f offset, atom count): a stable counting sort
    std::vector<std::pair<int64_t, int32_t>> keys;
    std::vector<int64_t> key_perm;
    std::vector<std::vector<int32_t>> key_count;
    for (const Segment &g : segs) {
        const std::pair<int64_t, int32_t> key(g.f, g.n_atoms);
        if (std::find(keys.begin(), keys.end(), key) != keys.end()) continue;
        std::vector<int32_t> cnt(n_species + 1, 0);
        for (int32_t j = 0; j < g.n_atoms; ++j) {
            const int32_t v = h[g.f + j];
            if (v < 0 || v >= n_species)
                return set_error(XS_EINVAL, "species[%lld] = %d outside [0, %d)", (long long)(g.f + j), v,
                                 n_species);
            ++cnt[v + 1];
        }
        for (int32_t k = 0; k < n_species; ++k) cnt[k + 1] += cnt[k];
        std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
        const int64_t base = static_cast<int64_t>(sp.perm.size());
        sp.perm.resize(base + g.n_atoms);
        for (int32_t j = 0; j < g.n_atoms; ++j) sp.perm[base + fill[h[g.f + j]]++] = j;
        keys.push_back(key);
        key_perm.push_back(base);
        key_count.push_back(cnt);
    }
    sp.segs.clear();
    sp.sub.clear();
    sp.sub_off.assign(segs.size() * n_species, -1);
    for (size_t i = 0; i < segs.size(); ++i) {
        const Segment &g = segs[i];
        const size_t ki = std::find(keys.begin(), keys.end(), std::make_pair(g.f, g.n_atoms)) - keys.begin();
        SpSeg ss{g.pos, key_perm[ki], g.q, g.out, g.n_atoms, g.n_q};
        sp.segs.push_back(ss);
        sp.n_pos = std::max<int64_t>(sp.n_pos, g.pos + g.n_atoms);
        sp.max_q = std::max(sp.max_q, g.n_q);
        sp.max_atoms = std::max(sp.max_atoms, g.n_atoms);
        const std::vector<int32_t> &cnt = key_count[ki];
        for (int32_t k = 0; k < n_species; ++k) {
            const int32_t n = cnt[k + 1] - cnt[k];
            if (n == 0) continue;
            Segment u = g;
            u.pos = g.pos + cnt[k];
            u.f = 0;  // unit weights
            u.out = sp.total_q;
            u.n_atoms = n;
            sp.sub_off[i * n_species + k] = sp.total_q;
            sp.sub_out.push_back(sp.total_q);
            sp.sub_par.push_back(static_cast<int32_t>(i));
            sp.sub_sp.push_back(k);
            sp.sub.push_back(u);
            sp.total_q += g.n_q;
            sp.max_sub_atoms = std::max(sp.max_sub_atoms, n);
        }
    }
    if (sp.sub.size() > 65535)
        return set_error(XS_ENOTSUP, "at most 65535 (system, frame, species) segments per call (got %zu)",
                         sp.sub.size());
    return XS_OK;
}

// Device copies of the tables, positions in species order and unit weights.
struct SpeciesDev {
    SpSeg *segs = nullptr;
    int32_t *perm = nullptr;
    int64_t *sub_off = nullptr;
    int32_t *sub_par = nullptr, *sub_sp = nullptr;
    int64_t *sub_out = nullptr;
    double *coef = nullptr;
    double *ones = nullptr;
    double *pos_r = nullptr;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// The split's tables as one host blob of 256-byte-aligned sections: segments,
// species order, species offsets, parent / species / output of every species
// segment, form-factor coefficients.  off[i] = byte offset of section i.
constexpr int kTabSections = 7;
std::vector<char> species_tables(const SpeciesSplit &sp, int32_t n_species, const double *coef_host,
                                 size_t (&off)[kTabSections]) {
    const size_t n_seg = sp.segs.size(), n_sub = sp.sub.size();
    const size_t sz[kTabSections] = {sizeof(SpSeg) * n_seg,
                                     sizeof(int32_t) * std::max<size_t>(sp.perm.size(), 1),
                                     sizeof(int64_t) * std::max<size_t>(sp.sub_off.size(), 1),
                                     sizeof(int32_t) * std::max<size_t>(n_sub, 1),
                                     sizeof(int32_t) * std::max<size_t>(n_sub, 1),
                                     sizeof(int64_t) * std::max<size_t>(n_sub, 1),
                                     sizeof(double) * 9 * n_species};
    const void *src[kTabSections] = {sp.segs.data(), sp.perm.data(), sp.sub_off.data(), sp.sub_par.data(),
                                     sp.sub_sp.data(), sp.sub_out.data(), coef_host};
    const size_t used[kTabSections] = {sizeof(SpSeg) * n_seg, sizeof(int32_t) * sp.perm.size(),
                                       sizeof(int64_t) * sp.sub_off.size(), sizeof(int32_t) * n_sub,
                                       sizeof(int32_t) * n_sub, sizeof(int64_t) * n_sub,
                                       sizeof(double) * 9 * n_species};
    size_t o = 0;
    for (int i = 0; i < kTabSections; ++i) {
        off[i] = o;
        o += align256(sz[i]);
    }
    std::vector<char> blob(o, 0);
    for (int i = 0; i < kTabSections; ++i)
        if (used[i]) std::memcpy(blob.data() + off[i], src[i], used[i]);
    return blob;
}

void point_tables(char *t, const size_t (&off)[kTabSections], SpeciesDev &d) {
    d.segs = reinterpret_cast<SpSeg *>(t + off[0]);
    d.perm = reinterpret_cast<int32_t *>(t + off[1]);
    d.sub_off = reinterpret_cast<int64_t *>(t + off[2]);
    d.sub_par = reinterpret_cast<int32_t *>(t + off[3]);
    d.sub_sp = reinterpret_cast<int32_t *>(t + off[4]);
    d.sub_out = reinterpret_cast<int64_t *>(t + off[5]);
    d.coef = reinterpret_cast<double *>(t + off[6]);
}

xs_status gather_positions(hipStream_t s, const SpeciesSplit &sp, const SpeciesDev &d, const double *pos) {
    if (!sp.segs.empty() && sp.max_atoms > 0)
        hipLaunchKernelGGL(k_species_gather, dim3(blocks_for(sp.max_atoms), static_cast<unsigned>(sp.segs.size())),
                           dim3(kBlock), 0, s, d.segs, d.perm, pos, d.pos_r);
    XS_HIP(hipGetLastError());
    return XS_OK;
}

xs_status upload_species(hipStream_t s, const SpeciesSplit &sp, int32_t n_species, const double *coef_host,
                         const double *pos, SpeciesDev &d) {
    size_t off[kTabSections];
    const std::vector<char> blob = species_tables(sp, n_species, coef_host, off);
    const size_t ones_n = static_cast<size_t>(std::max(sp.max_sub_atoms, 1));
    const size_t pos_n = static_cast<size_t>(std::max<int64_t>(sp.n_pos, 1)) * 3;
    void *tab = nullptr, *big = nullptr;
    XS_TRY(upload(s, SLOT_SPECIES_TAB, blob.data(), blob.size(), &tab));
    XS_TRY(scratch(s, SLOT_SPECIES_POS, sizeof(double) * (ones_n + pos_n), &big));
    point_tables(static_cast<char *>(tab), off, d);
    d.ones = static_cast<double *>(big);
    d.pos_r = d.ones + ones_n;
    hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(static_cast<int64_t>(ones_n))), dim3(kBlock), 0, s, d.ones,
                       static_cast<int64_t>(ones_n), 1.0);
    XS_HIP(hipGetLastError());
    return gather_positions(s, sp, d, pos);
}

}  // namespace

xs_status species_forward(hipStream_t s, const std::vector<Segment> &segs, const double *box, const double *pos,
                          const int32_t *species, int32_t n_species, const double *coef_host, const double *q,
                          int32_t precision, double *I, double *amp, const xs_tile_shape &fsh,
                          const xs_tile_shape &gsh) {
    SpeciesSplit sp;
    XS_TRY(split_species(s, segs, species, n_species, sp));
    SpeciesDev d;
    XS_TRY(upload_species(s, sp, n_species, coef_host, pos, d));
    const int64_t tq = (std::max<int64_t>(sp.total_q, 1) + 1) & ~int64_t(1);  // keeps the double2 rows aligned
    void *outs = nullptr;
    XS_TRY(scratch(s, SLOT_SPECIES_OUT, sizeof(double) * 3 * tq, &outs));
    double *I_s = static_cast<double *>(outs);
    double *amp_s = I_s + tq;
    const int n_sub = static_cast<int>(sp.sub.size());
    if (n_sub > 0) {
        if (precision == XS_FP64)
            XS_TRY(fp64_forward(s, sp.sub.data(), n_sub, sp.max_q, d.pos_r, d.ones, q, I_s, amp_s));
        else
            XS_TRY(fp32c_forward(s, sp.sub.data(), n_sub, box, d.pos_r, d.ones, q, I_s, amp_s, fsh, gsh));
    }
    if (!sp.segs.empty() && sp.max_q > 0)
        hipLaunchKernelGGL(k_species_combine, dim3(blocks_for(sp.max_q), static_cast<unsigned>(sp.segs.size())),
                           dim3(kBlock), 0, s, d.segs, d.sub_off, n_species, d.coef, q,
                           reinterpret_cast<const double2 *>(amp_s), I, reinterpret_cast<double2 *>(amp));
    XS_HIP(hipGetLastError());
    return XS_OK;
}

xs_status species_grad(hipStream_t s, const std::vector<Segment> &segs, const double *box, const double *pos,
                       const int32_t *species, int32_t n_species, const double *coef_host, const double *q,
                       const double *amp, const double *dL_dI, int32_t precision, float *dL_dr, double *dL_dr64,
                       const xs_tile_shape &fsh, const xs_tile_shape &gsh) {
    SpeciesSplit sp;
    XS_TRY(split_species(s, segs, species, n_species, sp));
    SpeciesDev d;
    XS_TRY(upload_species(s, sp, n_species, coef_host, pos, d));
    const int64_t tq = (std::max<int64_t>(sp.total_q, 1) + 1) & ~int64_t(1), np = std::max<int64_t>(sp.n_pos, 1);
    void *outs = nullptr;
    XS_TRY(scratch(s, SLOT_SPECIES_OUT, sizeof(double) * 3 * tq, &outs));
    double *w = static_cast<double *>(outs);
    double2 *amp_r = reinterpret_cast<double2 *>(w + tq);
    void *gbuf = nullptr;
    XS_TRY(scratch(s, SLOT_SPECIES_GRAD, (sizeof(float) + sizeof(double)) * 3 * np, &gbuf));
    double *g64_r = static_cast<double *>(gbuf);
    float *g32_r = reinterpret_cast<float *>(g64_r + 3 * np);
    const int n_sub = static_cast<int>(sp.sub.size());
    if (n_sub > 0 && sp.max_q > 0)
        hipLaunchKernelGGL(k_species_weights, dim3(blocks_for(sp.max_q), static_cast<unsigned>(n_sub)),
                           dim3(kBlock), 0, s, d.segs, d.sub_par, d.sub_sp, d.sub_out, d.coef, q, dL_dI,
                           reinterpret_cast<const double2 *>(amp), w, amp_r);
    XS_HIP(hipGetLastError());
    if (n_sub > 0) {
        float *o32 = dL_dr ? g32_r : nullptr;
        double *o64 = dL_dr64 ? g64_r : nullptr;
        if (precision == XS_FP64)
            XS_TRY(fp64_grad(s, sp.sub.data(), n_sub, sp.max_sub_atoms, d.pos_r, d.ones, q,
                             reinterpret_cast<const double *>(amp_r), w, o32, o64));
        else
            XS_TRY(fp32c_grad(s, sp.sub.data(), n_sub, box, d.pos_r, d.ones, q,
                              reinterpret_cast<const double *>(amp_r), w, o32, o64, fsh, gsh));
    }
    if (!sp.segs.empty() && sp.max_atoms > 0) {
        const dim3 grid(blocks_for(sp.max_atoms), static_cast<unsigned>(sp.segs.size()));
        if (dL_dr) hipLaunchKernelGGL(k_species_scatter<float>, grid, dim3(kBlock), 0, s, d.segs, d.perm, g32_r, dL_dr);
        if (dL_dr64)
            hipLaunchKernelGGL(k_species_scatter<double>, grid, dim3(kBlock), 0, s, d.segs, d.perm, g64_r, dL_dr64);
    }
    XS_HIP(hipGetLastError());
    return XS_OK;
}

// ---------------------------------------------------------------- species plans
//
// The species split of a batch (read once, when the plan is made), its device
// tables, the unit weights, the species-ordered positions and the per-species
// work buffers, in one allocation owned by the plan.  The pair sums of the
// species segments run through the caller's inner FP32C plan.  After creation
// every call only launches kernels.
struct SpeciesPlan {
    SpeciesSplit sp;
    int32_t n_species = 0;
    void *block = nullptr;
    SpeciesDev d;
    double *buf = nullptr;   // forward: I_s [tq], amp_s [tq][2]; adjoint: w [tq], amp_r [tq][2]
    int64_t tq = 0;
    double *g64_r = nullptr;
    float *g32_r = nullptr;
    size_t bytes = 0;
    ~SpeciesPlan() {
        if (block) (void)hipFree(block);
    }
};

xs_status species_plan_create(hipStream_t s, const std::vector<Segment> &segs, const int32_t *species,
                              int32_t n_species, const double *coef_host, SpeciesPlan **out,
                              std::vector<Segment> *sub) {
    *out = nullptr;
    auto *p = new (std::nothrow) SpeciesPlan();
    if (!p) return set_error(XS_ENOMEM, "species plan: host allocation failed");
    xs_status st = split_species(s, segs, species, n_species, p->sp);
    if (st != XS_OK) {
        delete p;
        return st;
    }
    const SpeciesSplit &sp = p->sp;
    p->n_species = n_species;
    size_t off[kTabSections];
    const std::vector<char> blob = species_tables(sp, n_species, coef_host, off);
    const size_t ones_n = static_cast<size_t>(std::max(sp.max_sub_atoms, 1));
    const size_t np = static_cast<size_t>(std::max<int64_t>(sp.n_pos, 1));
    p->tq = (std::max<int64_t>(sp.total_q, 1) + 1) & ~int64_t(1);  // keeps the double2 rows aligned
    // layout: tables | ones | pos_r [np][3] | buf [3 tq] | g64_r [np][3] | g32_r [np][3]
    const size_t o_ones = blob.size();
    const size_t o_pos = o_ones + align256(sizeof(double) * ones_n);
    const size_t o_buf = o_pos + align256(sizeof(double) * 3 * np);
    const size_t o_g64 = o_buf + align256(sizeof(double) * 3 * static_cast<size_t>(p->tq));
    const size_t o_g32 = o_g64 + align256(sizeof(double) * 3 * np);
    const size_t total = o_g32 + align256(sizeof(float) * 3 * np);
    hipError_t e = hipMalloc(&p->block, total);
    if (e != hipSuccess) {
        p->block = nullptr;
        (void)hipGetLastError();
        delete p;
        return set_error(XS_ENOMEM, "species plan: cannot allocate %zu bytes (%s)", total, hipGetErrorString(e));
    }
    p->bytes = total;
    char *b = static_cast<char *>(p->block);
    e = hipMemcpy(b, blob.data(), blob.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        delete p;
        return hip_error(e, "species plan: table upload");
    }
    point_tables(b, off, p->d);
    p->d.ones = reinterpret_cast<double *>(b + o_ones);
    p->d.pos_r = reinterpret_cast<double *>(b + o_pos);
    p->buf = reinterpret_cast<double *>(b + o_buf);
    p->g64_r = reinterpret_cast<double *>(b + o_g64);
    p->g32_r = reinterpret_cast<float *>(b + o_g32);
    hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(static_cast<int64_t>(ones_n))), dim3(kBlock), 0, s, p->d.ones,
                       static_cast<int64_t>(ones_n), 1.0);
    e = hipGetLastError();
    if (e != hipSuccess) {
        delete p;
        return hip_error(e, "species plan: unit weights");
    }
    *sub = sp.sub;
    *out = p;
    return XS_OK;
}

void species_plan_destroy(SpeciesPlan *p) { delete p; }

size_t species_plan_bytes(const SpeciesPlan *p) { return p->bytes; }

xs_status species_plan_forward(hipStream_t s, SpeciesPlan *p, Plan &inner, const double *q, const double *pos,
                               double *I, double *amp) {
    const SpeciesSplit &sp = p->sp;
    double *I_s = p->buf, *amp_s = p->buf + p->tq;
    XS_TRY(gather_positions(s, sp, p->d, pos));
    if (!sp.sub.empty()) {
        XS_TRY(inner.tile_atoms(s, p->d.pos_r, p->d.ones));
        XS_TRY(inner.forward(s, q, I_s, amp_s));
    }
    if (!sp.segs.empty() && sp.max_q > 0)
        hipLaunchKernelGGL(k_species_combine, dim3(blocks_for(sp.max_q), static_cast<unsigned>(sp.segs.size())),
                           dim3(kBlock), 0, s, p->d.segs, p->d.sub_off, p->n_species, p->d.coef, q,
                           reinterpret_cast<const double2 *>(amp_s), I, reinterpret_cast<double2 *>(amp));
    XS_HIP(hipGetLastError());
    return XS_OK;
}

xs_status species_plan_grad(hipStream_t s, SpeciesPlan *p, Plan &inner, const double *q, const double *pos,
                            const double *amp, const double *dL_dI, int32_t retile, float *dL_dr,
                            double *dL_dr64) {
    const SpeciesSplit &sp = p->sp;
    double *w = p->buf;
    double2 *amp_r = reinterpret_cast<double2 *>(p->buf + p->tq);
    const int n_sub = static_cast<int>(sp.sub.size());
    if (n_sub > 0 && !retile && !inner.tiled)
        return set_error(XS_EINVAL,
                         "retile = 0 needs the atom tiles of an earlier xs_plan_intensity_species on this plan");
    if (n_sub > 0 && sp.max_q > 0)
        hipLaunchKernelGGL(k_species_weights, dim3(blocks_for(sp.max_q), static_cast<unsigned>(n_sub)),
                           dim3(kBlock), 0, s, p->d.segs, p->d.sub_par, p->d.sub_sp, p->d.sub_out, p->d.coef, q,
                           dL_dI, reinterpret_cast<const double2 *>(amp), w, amp_r);
    XS_HIP(hipGetLastError());
    if (n_sub > 0) {
        if (retile) {
            XS_TRY(gather_positions(s, sp, p->d, pos));
            XS_TRY(inner.tile_atoms(s, p->d.pos_r, p->d.ones));
        }
        XS_TRY(inner.grad(s, q, p->d.ones, reinterpret_cast<const double *>(amp_r), w, dL_dr ? p->g32_r : nullptr,
                          dL_dr64 ? p->g64_r : nullptr));
    }
    if (!sp.segs.empty() && sp.max_atoms > 0) {
        const dim3 grid(blocks_for(sp.max_atoms), static_cast<unsigned>(sp.segs.size()));
        if (dL_dr)
            hipLaunchKernelGGL(k_species_scatter<float>, grid, dim3(kBlock), 0, s, p->d.segs, p->d.perm, p->g32_r,
                               dL_dr);
        if (dL_dr64)
            hipLaunchKernelGGL(k_species_scatter<double>, grid, dim3(kBlock), 0, s, p->d.segs, p->d.perm, p->g64_r,
                               dL_dr64);
    }
    XS_HIP(hipGetLastError());
    return XS_OK;
}

}  // namespace xs
