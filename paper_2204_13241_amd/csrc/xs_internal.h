// Internal declarations of the xs library (host side and kernel launchers).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "xs.h"

namespace xs {

// ---------------------------------------------------------------- errors
xs_status set_error(xs_status st, const char *fmt, ...);
xs_status hip_error(hipError_t e, const char *what);
#define XS_HIP(call)                                           \
    do {                                                       \
        hipError_t xs_e_ = (call);                             \
        if (xs_e_ != hipSuccess) return ::xs::hip_error(xs_e_, #call); \
    } while (0)
#define XS_TRY(expr)                                           \
    do {                                                       \
        xs_status xs_s_ = (expr);                              \
        if (xs_s_ != XS_OK) return xs_s_;                      \
    } while (0)

// ---------------------------------------------------------------- scratch
// Grow-only device buffers cached per (device, stream).  A slot is reused by
// every call on the same stream; calls on one stream are ordered, so reuse is
// safe.  Growth synchronises the stream first (refused during graph capture).
enum Slot {
    SLOT_SEGS = 0,      // segment / item tables
    SLOT_ITEMS,
    SLOT_COUNTER,       // work-queue counters
    SLOT_KEYS,          // binning: cell key per atom
    SLOT_HIST,          // binning: per-cell counts / cursors
    SLOT_SORTED,        // binning: sorted atom index
    SLOT_TILES,         // FP32C tile atoms (float4)
    SLOT_ORIGINS,       // FP32C tile origins (double4)
    SLOT_PARTIAL,       // partial sums
    SLOT_PIXEL,         // per-pixel prologue data
    SLOT_PIXEL2,
    SLOT_RING_KEY,      // reductions: per-pixel ring key
    SLOT_RING_CNT,      // reductions: per-block ring counts / offsets
    SLOT_RING_LIST,     // reductions: ring-order rank of each pixel, ring-ordered pixel list
    SLOT_G,             // g2 / F(q, tau) per-pixel values (rows in ring order)
    SLOT_LEVEL_A,       // XSVS coarser-level window sums (ping)
    SLOT_LEVEL_B,       // XSVS window sums (pong)
    SLOT_BWIN,          // XSVS per-window contrast
    SLOT_PSETS,         // FP32C pixel-set table
    SLOT_PIXKEYS,       // FP32C pixel sort keys / order
    SLOT_SORT_TMP,      // radix-sort temporary storage
    SLOT_GITEMS,        // FP32C gradient work items
    SLOT_PLAN,          // one-shot FP32C plan buffers
    SLOT_TABLES,        // one-shot FP32C plan tables (staging)
    SLOT_SPECIES_TAB,   // species split: segment tables, species order, form-factor coefficients
    SLOT_SPECIES_POS,   // species split: unit weights and positions in species order
    SLOT_SPECIES_OUT,   // species split: per-species amplitudes / adjoint weights
    SLOT_SPECIES_GRAD,  // species split: gradients in species order
    SLOT_FFT_RHO,       // FFT method: smeared density on the grid
    SLOT_FFT_SPEC,      // FFT method: its half spectrum
    SLOT_FFT_GAUSS,     // FFT method: half spectrum of the centred Gaussian
    SLOT_FFT_GAUSS2,    // FFT method: its squared modulus
    SLOT_XSVS_ORDER,    // XSVS: launch order of the gathering blocks
    SLOT_COUNT
};
xs_status scratch(hipStream_t stream, Slot slot, size_t bytes, void **ptr);
// Copy a host table to a device address through the slot's pinned staging buffer.
xs_status stage_copy(hipStream_t stream, Slot slot, const void *host, size_t bytes, void *dst);
// Stage a host table into the stream's scratch slot (async copy from a
// library-owned pinned staging buffer).
xs_status upload(hipStream_t stream, Slot slot, const void *host, size_t bytes, void **dev);
void release_all_scratch();

// ---------------------------------------------------------------- segments
// One (system, frame) pair of a batch.
struct Segment {
    int64_t pos;       // atom offset of the frame in pos (units of atoms)
    int64_t f;         // offset into f
    int64_t q;         // pixel offset into q
    int64_t out;       // pixel offset into outputs
    int32_t n_atoms;
    int32_t n_q;
    int32_t sys;
    int32_t frame;
};

// ---------------------------------------------------------------- launchers
xs_status fp64_forward(hipStream_t s, const Segment *segs_host, int n_segs, int max_q,
                       const double *pos, const double *f, const double *q, double *I,
                       double *amp);
xs_status fp64_grad(hipStream_t s, const Segment *segs_host, int n_segs, int max_atoms,
                    const double *pos, const double *f, const double *q, const double *amp,
                    const double *dL_dI, float *dL_dr, double *dL_dr64);

// FP32C batch plan: host tables and work lists of one batch layout, device
// buffers carved from one block, and the steps of a call.  The pixel order
// depends on q only; atom tiles depend on the positions.  Every step after
// allocate() is kernel launches only (capturable in a HIP graph), except
// sort_pixels, which uses a library radix sort.
class Plan {
public:
    struct Tables;
    struct Buffers;
    Plan();
    ~Plan();
    Plan(const Plan &) = delete;
    Plan &operator=(const Plan &) = delete;
    // Structure tests of every distinct pixel set (device checks, synchronizes s): rows of
    // n2 pixels sharing q_y (row form of the per-pair sums) and row lattices (lattice forms);
    // build() then picks each set's form from the tile shapes.
    xs_status find_lattices(hipStream_t s, const Segment *segs, int n_segs, const double *q);
    xs_status build(const Segment *segs, int n_segs, const double *box, const xs_tile_shape &fsh,
                    const xs_tile_shape &gsh);
    xs_status allocate(hipStream_t s, bool owned);
    xs_status sort_pixels(hipStream_t s, const double *q);
    xs_status tile_atoms(hipStream_t s, const double *pos, const double *f);
    xs_status forward(hipStream_t s, const double *q, double *I, double *amp);
    xs_status grad(hipStream_t s, const double *q, const double *f, const double *amp,
                   const double *dL_dI, float *g32, double *g64);
    size_t layout(char *base);
    std::vector<char> table_blob() const;
    void describe(int *n_lattice_segs, int *n_row_segs, int *n_fwd_items, int *n_grad_items) const;

    Tables *T;
    Buffers *B;
    void *owned_block = nullptr;
    size_t device_bytes = 0;
    bool tiled = false;        // tile_atoms has been enqueued at least once
    bool with_grad = true;     // set before build(): false leaves out the adjoint's lists and buffers
    int n_seg = 0;
    xs_tile_shape fshape{}, gshape{};
};

xs_status fp32c_forward(hipStream_t s, const Segment *segs_host, int n_segs, const double *box,
                        const double *pos, const double *f, const double *q, double *I,
                        double *amp, const xs_tile_shape &fsh, const xs_tile_shape &gsh);
xs_status fp32c_grad(hipStream_t s, const Segment *segs_host, int n_segs, const double *box,
                     const double *pos, const double *f, const double *q, const double *amp,
                     const double *dL_dI, float *dL_dr, double *dL_dr64,
                     const xs_tile_shape &fsh, const xs_tile_shape &gsh);

constexpr int kMaxRings = 256;
struct RingEdges {
    double e[kMaxRings + 1];
    int32_t n_rings;
};
xs_status g2_rings(hipStream_t s, const double *I, int64_t n_frames, int64_t n_q,
                   const double *q, const RingEdges &edges, int32_t n_tau, double *g2_out,
                   int32_t *ring_count);
// g2_rings with every working buffer carved from the library's fixed per-device
// array (g2_fixed_scratch_bytes() bytes): no allocation; XS_EINVAL if it does not fit.
xs_status g2_rings_fixed(hipStream_t s, const double *I, int64_t n_frames, int64_t n_q,
                         const double *q, const RingEdges &edges, int32_t n_tau, double *g2_out,
                         int32_t *ring_count);
size_t g2_fixed_scratch_bytes();
xs_status xsvs_contrast(hipStream_t s, const double *I, int64_t n_frames, int64_t n_q,
                        const double *q, const RingEdges &edges, int32_t n_levels,
                        double *beta_out, double *beta_win);
xs_status species_forward(hipStream_t s, const std::vector<Segment> &segs, const double *box, const double *pos,
                          const int32_t *species, int32_t n_species, const double *coef_host, const double *q,
                          int32_t precision, double *I, double *amp, const xs_tile_shape &fsh,
                          const xs_tile_shape &gsh);
xs_status species_grad(hipStream_t s, const std::vector<Segment> &segs, const double *box, const double *pos,
                       const int32_t *species, int32_t n_species, const double *coef_host, const double *q,
                       const double *amp, const double *dL_dI, int32_t precision, float *dL_dr, double *dL_dr64,
                       const xs_tile_shape &fsh, const xs_tile_shape &gsh);
// Plans for q-dependent form factors: the species split and its buffers; the pair
// sums of the species segments (*sub) run through an inner FP32C plan built by the caller.
struct SpeciesPlan;
xs_status species_plan_create(hipStream_t s, const std::vector<Segment> &segs, const int32_t *species,
                              int32_t n_species, const double *coef_host, SpeciesPlan **out,
                              std::vector<Segment> *sub);
void species_plan_destroy(SpeciesPlan *p);
size_t species_plan_bytes(const SpeciesPlan *p);
xs_status species_plan_forward(hipStream_t s, SpeciesPlan *p, Plan &inner, const double *q, const double *pos,
                               double *I, double *amp);
xs_status species_plan_grad(hipStream_t s, SpeciesPlan *p, Plan &inner, const double *q, const double *pos,
                            const double *amp, const double *dL_dI, int32_t retile, float *dL_dr,
                            double *dL_dr64);
xs_status frame_sums(hipStream_t s, const double *I, int64_t n_q, int64_t n_out, int64_t s_out, int64_t n_sum,
                     int64_t s_sum, double scale, double *J);
xs_status ring_histogram(hipStream_t s, const double *I, int64_t F, int64_t n_q, const double *q,
                         const RingEdges &edges, int32_t n_bins, double kappa_max, int64_t *counts, double *mean);
xs_status isf_rings(hipStream_t s, const double *amp, int64_t n_frames, int64_t n_q, const double *q,
                    const RingEdges &edges, int32_t n_tau, double f2, double *F_out, int32_t *ring_count);
xs_status siegert(hipStream_t s, const double *g2, const double *F, int32_t n_rings, int32_t n_tau,
                  int32_t n_levels, double *lhs, double *fhat2, double *beta);
// FFT-based method (Algorithm 2), one frame on an n^3 grid; I [n^3], amp [n^3][2] or NULL.
xs_status fft_intensity(hipStream_t s, const double *pos, const double *f, int64_t n_atoms, double box,
                        int32_t n, double eta, int32_t k, double *I, double *amp);
void release_fft_plans();

// ---------------------------------------------------------------- timing
// Optional HIP-event timing of kernel launches on the stream they run on.
enum TimerKind {
    TIMER_FWD32 = 0,   // FP32C forward pair kernel
    TIMER_GRAD32 = 1,  // FP32C gradient pair kernel
    TIMER_FWD64 = 2,   // FP64 forward kernel
    TIMER_GRAD64 = 3,  // FP64 gradient kernel
    TIMER_BIN = 4,     // FP32C binning (all binning kernels of a call)
    TIMER_G2 = 5,      // g2 reduction (whole call)
    TIMER_XSVS = 6,    // XSVS reduction (whole call)
    TIMER_ISF = 7,     // intermediate scattering function on rings (whole call)
};
#define XS_TIMER_KINDS 8
bool timing_on();
void timer_begin(hipStream_t s, int kind, void **token);
void timer_end(hipStream_t s, int kind, void *token, double work);
void timer_discard(void *token);

// Event timer of one library call (when timing is on): begun at construction, end()
// records it with its work; a scope left early (an error return) discards its events.
class TimerScope {
public:
    TimerScope(hipStream_t s, int kind, bool on = true) : s_(s), kind_(kind) {
        if (on) timer_begin(s, kind, &tok_);
    }
    ~TimerScope() { timer_discard(tok_); }
    TimerScope(const TimerScope &) = delete;
    TimerScope &operator=(const TimerScope &) = delete;
    void end(double work) {
        timer_end(s_, kind_, tok_, work);
        tok_ = nullptr;
    }

private:
    hipStream_t s_;
    int kind_;
    void *tok_ = nullptr;
};
xs_status timing_enable(int on);
xs_status timing_read(int kind, double *ms, int64_t *launches, double *work);

xs_status speckle_loss(hipStream_t s, const double *I, const double *It, int64_t n, double *out,
                       double *dL_dI);
xs_status position_step(hipStream_t s, double *pos, const float *g32, const double *g64, int64_t n,
                        double step);
xs_status roofline_probe(hipStream_t s, int kind, int64_t bytes, double *rate);

// Blocks of `block` threads of `kernel` that the current device holds at once
// (occupancy x compute units), cached per kernel and device.
int resident_blocks(const void *kernel, int block);

}  // namespace xs
