/*
 * xs.h -- C ABI of the MI355X (gfx950) library for the direct X-ray speckle
 * method of Mohanty, Cooper, Wang, Liang, Cai, "Computational approaches to
 * model X-ray photon correlation spectroscopy from molecular dynamics"
 * (arXiv:2204.13241).
 *
 * The library computes, for every detector pixel q and every frame t of an
 * atomic trajectory, the scattering amplitude and intensity of the direct
 * method (Sec. 3.1, Algorithm 1):
 *     p^e(q,t) = sum_j f_j exp(-i q . r_j(t))          Sec. 2.2, Eq. (pe_ri)
 *     I(q,t)   = |p^e(q,t)|^2                          Sec. 2.2, Eq. (Iq_pq)
 * its gradient with respect to the positions, and the reductions of I to the
 * intensity autocorrelation g2(|q|, tau) (Sec. 2.3, Eq. (g2_def)) and to the
 * exposure-time speckle contrast beta (Sec. 2.3, Eqs. (inte_Iq), (bq_Iq)).
 *
 * General conventions
 *   - Every array argument documented "device" is a pointer to GPU memory on
 *     the current HIP device, owned by the caller; the library reads or writes
 *     it only during the enqueued work and never frees or retains it.
 *     "host" arguments are read before the call returns.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = legacy default
 *     stream).  Calls return once the work is enqueued; results are valid
 *     after the stream is synchronised.
 *   - Argument validation is synchronous: XS_EINVAL / XS_ENOTSUP return before
 *     anything is enqueued.  HIP failures return XS_EDEVICE.  Scratch memory
 *     the library cannot obtain returns XS_ENOMEM.  xs_last_error() gives a
 *     thread-local message for the last non-OK status of the calling thread.
 *   - Scratch memory (binning tiles, partial sums, ring lists) is owned by the
 *     library, cached per (device, stream) and released by xs_shutdown().
 *     Concurrent calls on the same stream from different host threads are not
 *     supported.
 *   - Lengths are in Angstrom, wavevectors in 1/Angstrom.  Positions are used
 *     verbatim: the library never wraps or images them.
 *   - Nothing is printed; no C++ exception crosses the ABI.
 */
#ifndef XS_H
#define XS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t xs_status;
enum {
    XS_OK = 0,       /* success                                                   */
    XS_EINVAL = 1,   /* bad argument (size, pointer, layout, non-finite scalar)   */
    XS_ENOMEM = 2,   /* scratch allocation failed                                  */
    XS_EDEVICE = 3,  /* HIP runtime / kernel launch failure                        */
    XS_ENOTSUP = 4   /* valid request this build does not support                  */
};

/* Arithmetic of the pair sums. */
enum {
    /* Exact FP64 form: phase q.r/(2 pi) in FP64, sine and cosine from the
     * Taylor series after exact reduction to |angle| <= pi/4, atoms (forward)
     * or pixels (gradient) summed sequentially in input order.  Bit-for-bit
     * reproducible and equal to the CPU FP64 oracle's result.               */
    XS_FP64 = 0,
    /* FP32 compensated form: atoms are binned into compact spatial tiles;
     * the phase of each tile origin is reduced in FP64 per (pixel, tile),
     * the in-tile phase, sine/cosine (hardware, revolutions) and the tile
     * partial sums run in FP32, and tile partials are folded into FP64.     */
    XS_FP32C = 1
};

/*
 * Layout of a batch of independent systems (one system = one sample with its
 * own atoms, pixels and frames).  All members are host arrays of n_sys
 * entries; `box` has 3 entries per system.
 *
 *   system s, frame t, atom j  -> pos[(pos_off[s] + t * n_atoms[s] + j) * 3 + {0,1,2}]
 *   system s, atom j           -> f[f_off[s] + j]            (same for every frame)
 *   system s, pixel p          -> q[(q_off[s] + p) * 3 + {0,1,2}]
 *   system s, frame t, pixel p -> out[out_off[s] + t * n_q[s] + p]   (I, dL/dI)
 *                                 amp[(out_off[s] + t * n_q[s] + p) * 2 + {re, im}]
 *
 * box[s*3 + c] is the orthorhombic box edge of system s (Sec. 3.1: the
 * simulation cell; Algorithm 1 takes q on its reciprocal lattice, but any q
 * is accepted).  It must be positive and finite for the FP32C form, which
 * bins each frame's atoms on a grid over the bounding box of that frame's
 * positions (so atoms outside [0, box), as in unwrapped trajectories, still form
 * compact tiles).  The FP64 form ignores it.
 *
 * Limits: 1 <= n_sys; 0 <= n_atoms[s] < 2^31; 0 <= n_q[s] < 2^31;
 * 1 <= n_frames[s]; offsets >= 0.
 */
typedef struct xs_batch {
    int32_t n_sys;
    const int64_t *n_atoms;
    const int64_t *n_q;
    const int32_t *n_frames;
    const int64_t *pos_off;
    const int64_t *f_off;
    const int64_t *q_off;
    const int64_t *out_off;
    const double *box;
} xs_batch;

/*
 * Direct method, Sec. 3.1 Algorithm 1 with Eqs. (pe_ri) and (Iq_pq): for every
 * system, frame and pixel,
 *     amp = a + i b = sum_j f_j exp(-i q.r_j),   I = a^2 + b^2.
 *   b         host   batch layout (see xs_batch)
 *   pos       device double, positions (Angstrom)
 *   f         device double, per-atom form factors (q-independent)
 *   q         device double, wavevectors (1/Angstrom)
 *   precision XS_FP64 or XS_FP32C
 *   I_out     device double, intensities
 *   amp_out   device double [..][2] amplitudes (a, b), or NULL
 * A system with n_atoms = 0 gives I = 0 and amp = 0.  All systems and frames
 * of the batch run in one persistent launch per phase (binning, pair sum,
 * combine).
 */
xs_status xs_intensity_direct(const xs_batch *b, const double *pos, const double *f,
                              const double *q, int32_t precision, double *I_out,
                              double *amp_out, void *stream);

/*
 * Gradient of a scalar L(I) with respect to the positions, through
 * Eqs. (pe_ri) and (Iq_pq):
 *     dI/dr_j = -2 f_j q (a sin(q.r_j) + b cos(q.r_j)),
 *     dL/dr_j = sum_{t-independent pixels p} (dL/dI_p) dI_p/dr_j   (per frame).
 *   amp       device double [..][2], the amplitude of the same positions
 *             (from xs_intensity_direct), batch output layout
 *   dL_dI     device double, upstream gradient, batch output layout
 *   precision XS_FP32C: the sum over pixels runs as
 *             sum_p W_p sin(q_p.r_j + arg amp_p), W_p = -2 f_j w_p |amp_p| q_p,
 *             in FP32 with FP64 folding of pixel-chunk partials;
 *             XS_FP64: the exact FP64 form, pixels in input order.
 *   dL_dr     device float [..][3] (positions layout), or NULL
 *   dL_dr64   device double [..][3] (positions layout), or NULL
 * At least one of dL_dr / dL_dr64 must be non-NULL.
 */
xs_status xs_intensity_grad(const xs_batch *b, const double *pos, const double *f,
                            const double *q, const double *amp, const double *dL_dI,
                            int32_t precision, float *dL_dr, double *dL_dr64, void *stream);

/*
 * Intensity with q-dependent atomic form factors, Eqs. (Iq_rij), (pe_ri) with
 * f_j(q) = f_{species[j]}(|q|), each species' form factor a sum of Gaussians
 * (Sec. 2.1):
 *     f_s(q) = c + sum_{i=1..4} a_i exp(-b_i s^2),   s = |q| / (4 pi)  (1/A),
 * computed on the device per pixel and species.
 *   b          batch descriptor as for xs_intensity_direct; species[] has the
 *              layout of f (offset f_off[s] per system, shared by its frames)
 *   pos, q     as for xs_intensity_direct
 *   species    device int32 [..] species index of every atom, 0 <= v < n_species
 *   n_species  1 .. 4096
 *   ff_coef    host double [n_species][9]: a_1..a_4, b_1..b_4 (A^2), c
 *   precision  XS_FP64 or XS_FP32C (as for xs_intensity_direct)
 *   I_out      device double, same layout as for xs_intensity_direct
 *   amp_out    device double [..][2] (a, b) of p^e = a + i b, or NULL
 * The atoms of each species form their own pair sum P_s(q) = sum_{j in s}
 * e^{-i q.r_j} (unit weights, the ordinary batched pair kernels), and
 * p^e = sum_s f_s(|q|) P_s.  The species array is read back to the host to
 * build that split: the call waits for the stream's earlier work.  Errors:
 * XS_EINVAL for a species index out of range, non-finite coefficients, or the
 * conditions of xs_intensity_direct.
 */
xs_status xs_intensity_species(const xs_batch *b, const double *pos, const int32_t *species,
                               int32_t n_species, const double *ff_coef, const double *q,
                               int32_t precision, double *I_out, double *amp_out, void *stream);

/*
 * Gradient of L = sum_p w_p I_p with q-dependent form factors (the chain rule
 * through Eqs. (pe_ri), (Iq_pq) with f_j(q)):
 *     dL/dr_j = -2 sum_p w_p f_j(q_p) q_p (a_p sin(q_p.r_j) + b_p cos(q_p.r_j)),
 * amp the amplitude from xs_intensity_species of the same positions, dL_dI =
 * w.  Arguments and outputs as for xs_intensity_grad plus species, n_species
 * and ff_coef as for xs_intensity_species; gradients in the caller's atom order.
 */
xs_status xs_intensity_species_grad(const xs_batch *b, const double *pos, const int32_t *species,
                                    int32_t n_species, const double *ff_coef, const double *q,
                                    const double *amp, const double *dL_dI, int32_t precision,
                                    float *dL_dr, double *dL_dr64, void *stream);

/*
 * Intensity autocorrelation on |q| rings, Sec. 2.3 Eq. (g2_def), ring mean of
 * Sec. 4.2:
 *     G_p(tau) = [sum_{t < F - tau} I_t,p I_t+tau,p / (F - tau)] / <I_p>_t^2,
 *     <I_p>_t  = sum_t I_t,p / F,
 *     g2(r, tau) = mean over pixels p of ring r of G_p(tau).
 *   I          device double [n_frames][n_q] (pixel fastest)
 *   q          device double [n_q][3]; ring r holds e_r <= |q| < e_{r+1}
 *   ring_edges host double [n_rings + 1], strictly increasing
 *   n_tau      lags 0 .. n_tau - 1, 1 <= n_tau <= n_frames
 *   g2_out     device double [n_rings][n_tau]; NaN for rings with no pixel
 *   ring_count device int32 [n_rings] pixels used per ring, or NULL
 * Pixels whose <I>_t^2 is zero are left out.  Every sum has a fixed order
 * (time sums sequential in t; ring sums pairwise over the ring's pixels in
 * ascending index: adjacent pairs added level by level, an odd last element
 * carried up), so the result is bit-for-bit reproducible and equal to the
 * oracle's.
 */
xs_status xs_g2_rings(const double *I, int64_t n_frames, int64_t n_q, const double *q,
                      const double *ring_edges, int32_t n_rings, int32_t n_tau,
                      double *g2_out, int32_t *ring_count, void *stream);

/*
 * xs_g2_rings without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Arguments, results and summation order are those of
 * xs_g2_rings (bit-for-bit equal).  The working buffers (ring keys, ring-order
 * lists, per-pixel lag rows, tree levels) are carved from one fixed array of
 * 64 MiB per device that the library holds until the process ends; no
 * hipMalloc, hipFree or allocating library routine is called, and no timing
 * event is recorded.  Requires n_q * n_tau * 8 bytes (the lag rows) plus the
 * smaller buffers to fit in 64 MiB (e.g. 65,536 pixels x 100 lags); larger
 * requests return XS_EINVAL before anything is enqueued.  Every call on one
 * device shares that array: calls that overlap on one device (different
 * streams or host threads without ordering) race and give wrong results; the
 * array keeps the last call's contents, and each call rewrites every value it
 * reads.
 */
xs_status xs_g2_rings_noalloc(const double *I, int64_t n_frames, int64_t n_q, const double *q,
                              const double *ring_edges, int32_t n_rings, int32_t n_tau,
                              double *g2_out, int32_t *ring_count, void *stream);

/*
 * XSVS contrast versus exposure time, Sec. 2.3 Eqs. (inte_Iq) and (bq_Iq):
 * exposure windows of W = 2^l frames (l = 0 .. n_levels-1), non-overlapping
 * from frame 0, trailing partial window dropped, window sums built pairwise
 * (J_{l+1}[k] = J_l[2k] + J_l[2k+1]);
 *     beta(l, k, r) = (m2 - m1^2) / m1^2,  m1 = mean_r(J_l[k]),
 *                     m2 = mean_r(J_l[k]^2)   (the moments of Eq. (bq_Iq), read once),
 *     beta_out[l][r] = mean over the K_l = floor(F / 2^l) windows.
 *   I          device double [n_frames][n_q]
 *   q, ring_edges, n_rings as for xs_g2_rings
 *   n_levels   1 <= n_levels, 2^(n_levels-1) <= n_frames
 *   beta_out   device double [n_levels][n_rings]; NaN for empty rings
 *   beta_win   device double [n_levels][n_frames][n_rings] per-window values
 *              (entries k >= K_l are NaN), or NULL
 * Fixed summation order as for xs_g2_rings: bit-for-bit equal to the oracle.
 */
xs_status xs_xsvs_contrast(const double *I, int64_t n_frames, int64_t n_q, const double *q,
                           const double *ring_edges, int32_t n_rings, int32_t n_levels,
                           double *beta_out, double *beta_win, void *stream);

/*
 * Intermediate scattering function on |q| rings, Sec. 2.3 Eq. (Fq_pq), with
 * the per-pixel-then-ring-mean average used for g2 (Sec. 4.2):
 *     F_p(tau) = [sum_{t < F - tau} p_t,p conj(p_t+tau,p) / (F - tau)] / f2_sum,
 *     F(r, tau) = mean over every pixel p of ring r of F_p(tau),
 * with p = a + i b the amplitude of Eq. (pe_ri) as xs_intensity_direct writes
 * it.  F-hat of Eq. (norm_Fq) is F(r, tau) / F(r, 0).
 *   amp        device double [n_frames][n_q][2] (a, b), 16-byte aligned
 *   q, ring_edges, n_rings, n_tau as for xs_g2_rings
 *   f2_sum     sum_j f_j^2 of the sample (> 0, finite)
 *   F_out      device double [n_rings][n_tau][2] (re, im); NaN for empty rings
 *   ring_count device int32 [n_rings] pixels per ring, or NULL
 * Fixed order: for t ascending, re = fma(a_t, a_t+tau, re), fma(b_t, b_t+tau, re);
 * im = fma(b_t, a_t+tau, im), fma(-a_t, b_t+tau, im); ring sums pairwise as
 * for xs_g2_rings.  Bit-for-bit equal to the oracle.
 */
xs_status xs_isf_rings(const double *amp, int64_t n_frames, int64_t n_q, const double *q,
                       const double *ring_edges, int32_t n_rings, int32_t n_tau, double f2_sum,
                       double *F_out, int32_t *ring_count, void *stream);

/*
 * Siegert relation and the exposure contrast it predicts, Sec. 2.3
 * Eqs. (bq_g2), (norm_Fq), (g2_from_fq), (beta_alt_int), per ring r:
 *     beta0(r)       = g2(r, 0) - 1
 *     lhs(r, tau)    = (g2(r, tau) - 1) / beta0(r)     (equals |F-hat|^2 when
 *                                                       the relation holds)
 *     fhat2(r, tau)  = |F(r, tau)|^2 / |F(r, 0)|^2
 *     beta(l, r)     = beta0(r) (1 + 2 sum_{k=1}^{W-1} (1 - k/W) fhat2(r, k)) / W,
 *                      W = 2^l: Eq. (beta_alt_int) for exposures that are sums
 *                      of W consecutive frames, comparable with
 *                      xs_xsvs_contrast's beta_out[l].
 *   g2         device double [n_rings][n_tau] (xs_g2_rings)
 *   F          device double [n_rings][n_tau][2] (xs_isf_rings)
 *   n_levels   0 <= n_levels, 2^(n_levels-1) <= n_tau
 *   lhs_out, fhat2_out  device double [n_rings][n_tau], or NULL
 *   beta_out   device double [n_levels][n_rings] (may be NULL if n_levels = 0)
 * |z|^2 = fma(re, re, im * im); the sum over k runs k = 1, 2, ... by fma.
 * Bit-for-bit equal to the oracle.
 */
xs_status xs_siegert(const double *g2, const double *F, int32_t n_rings, int32_t n_tau, int32_t n_levels,
                     double *lhs_out, double *fhat2_out, double *beta_out, void *stream);

/*
 * Sums of frames, one definition for the uses of Sec. 4.5, Eq. (inte_Iq) and
 * the pixel integral of Sec. 3.1:
 *     J[k][p] = scale * sum_{i < n_sum} I[k * s_out + i * s_sum][p],   k < n_out,
 * - incoherent superposition of M independent configurations stored as blocks
 *   of F frames: n_out = F, s_out = 1, n_sum = M, s_sum = F;
 * - exposure integrals over W frames (rectangle rule): n_sum = W, s_sum = 1,
 *   s_out = W (non-overlapping) or 1 (sliding); xs_g2_rings of J is then the
 *   g2 of the exposure-integrated intensity, Eq. (g2_def_pulse);
 * - a detector pixel's mean over S sub-pixel wavevectors (Sec. 3.1: a pixel
 *   covers a small range of q), the intensity computed on q stored as S blocks
 *   of the Q pixels, so that a frame's row reads as S rows of Q: n_frames =
 *   F S, n_out = F, s_out = S, n_sum = S, s_sum = 1, scale = 1/S.
 *   I      device double [n_frames][n_q];  J_out device double [n_out][n_q]
 *   scale  finite; the sum is multiplied by it once (1: the plain sum)
 * Each sum is the pairwise tree over i in ascending order (adjacent pairs added
 * level by level, an odd last element carried up; for n_sum = 2^l, s_sum = 1 it
 * is the dyadic window sum of xs_xsvs_contrast), bit-for-bit equal to the
 * oracle.  Needs (n_out-1) s_out + (n_sum-1) s_sum < n_frames, n_sum <= 2^24.
 */
xs_status xs_frame_sums(const double *I, int64_t n_frames, int64_t n_q, int64_t n_out, int64_t s_out,
                        int64_t n_sum, int64_t s_sum, double scale, double *J_out, void *stream);

/*
 * Distribution of the normalized intensity kappa = I / <I>_ring per frame and
 * ring (Sec. 4.5, Eq. (Erlang): kappa of M superposed speckle patterns follows
 * the Erlang law of order M):
 *     <I>_ring = (pairwise sum over the ring's pixels, ascending index) / n,
 *     u = (I / <I>_ring) * (n_bins / kappa_max),
 *     bin = floor(u) for 0 <= u < n_bins (u <= 0: bin 0), else bin n_bins
 *           (overflow; NaN too).
 *   I, q, ring_edges, n_rings as for xs_g2_rings; n_frames <= 65535
 *   counts_out device int64 [n_frames][n_rings][n_bins + 1]
 *   mean_out   device double [n_frames][n_rings] (NaN for empty rings), or NULL
 * n_rings * (n_bins + 1) <= 16384.  Counts are exact; bins are decided in FP64
 * exactly as the oracle decides them.
 */
xs_status xs_ring_histogram(const double *I, int64_t n_frames, int64_t n_q, const double *q,
                            const double *ring_edges, int32_t n_rings, int32_t n_bins, double kappa_max,
                            int64_t *counts_out, double *mean_out, void *stream);

/*
 * FFT-based method of Sec. 3.2 (Algorithm 2, Eqs. (modified_r), (pq_rq_app_alt),
 * (Iq_pq_new)): the comparison baseline of the direct method, one frame, FP64.
 * Every atom's Gaussian of width eta (weight f_j) is added to the k grid points
 * nearest to it along each axis of an n_grid^3 grid over the periodic box
 * [0, box)^3 (indices modulo n_grid); the grid is Fourier transformed (hipFFT);
 * f^eta is the same transform of one Gaussian centred at the origin, and
 *     I(q_h) = |p^eta(q_h)|^2 / f^eta(q_h)^2,   q_h = 2 pi h / box,
 * amp = p^eta / f^eta (the amplitude of Eq. (pe_ri), exp(-i q.r) convention).
 *   pos, f     device double [n_atoms][3] (inside [0, box)) and [n_atoms]
 *   box        cube edge, Angstrom;  n_grid in [2, 1024];  eta > 0 (Angstrom);
 *              k in [1, n_grid] (the paper takes the nearest integer above
 *              10 eta n_grid / box)
 *   I_out      device double [n_grid][n_grid][n_grid], index h per axis in FFT
 *              order (h for h < n_grid / 2, h - n_grid above)
 *   amp_out    device double [n_grid^3][2], or NULL
 * The density is accumulated with FP64 atomics (last bits vary from run to run).
 * Working memory (about 40 n_grid^3 bytes) comes from the stream's scratch; the
 * FFT plan and the Gaussian's transform are cached per (device, stream).
 */
xs_status xs_fft_intensity(const double *pos, const double *f, int64_t n_atoms, double box, int32_t n_grid,
                           double eta, int32_t k, double *I_out, double *amp_out, void *stream);

/* Thread-local message for the last non-OK status returned to this thread. */
const char *xs_last_error(void);

/* Library version as an integer (major * 10000 + minor * 100 + patch). */
int32_t xs_version(void);

/* Release every cached scratch buffer on every device.  Call with no work of
 * this library in flight.  Safe to call more than once. */
xs_status xs_shutdown(void);

/*
 * Tile shape of the FP32C pair kernels (the autotuner's search space):
 *   atoms_per_tile  atoms in one spatial tile (64: one wavefront)
 *   q_per_lane      pixels (forward) or atoms (gradient) per lane (1, 2, 4, 8);
 *                   32 selects the matrix-core lattice form for the lattice
 *                   systems of a plan (FP16 split factors, 64 x 64 pixel
 *                   rectangles; other systems run at 8 pixels or 2 atoms per
 *                   lane)
 *   atom_split      atom tiles per forward work item (>= 1); with q_per_lane
 *                   32 also per gradient work item
 *   pixel_split     pixels per gradient work item (multiple of 64)
 *   waves_per_simd  0: compiler's register allocation; 4: variant bounded to
 *                   128 VGPRs (4 wavefronts per SIMD), built for forward
 *                   q_per_lane 2, 4 and (lattice form only; the general form
 *                   keeps its own allocation) 8, and gradient q_per_lane 4;
 *                   5: bounded to 96 VGPRs, built for gradient q_per_lane 2;
 *                   3: bounded to 168 registers, built for forward q_per_lane 32
 *                   and for the row form at q_per_lane 8 (the general form at 8
 *                   keeps its own allocation)
 *   lattice         plans only.  0 (default): the per-pair forms, in which every
 *                   atom-pixel pair takes the sine and cosine of its own phase
 *                   (forward) or the sine (adjoint); on pixel sets stored as rows
 *                   (every run of n2 >= 8 consecutive pixels shares q_y exactly, as
 *                   planar and Ewald-sphere detectors stored row by row do; see
 *                   xs_plan_create) the row form: a lane's q_per_lane pixels lie in
 *                   one row, the q_y part of the phase is formed once per (lane,
 *                   atom), and the adjoint's 64-pixel groups run along rows (rows
 *                   of a multiple of 64 pixels).  2: the general per-pair form
 *                   only (rows ignored).  1: the lattice factorizations where a
 *                   system's pixels come in rows of n2 consecutive q-vectors that
 *                   each step by one common vector a (a planar grid stored row by
 *                   row), the row form elsewhere.  Forward: a lane owns a run of
 *                   q_per_lane (2, 4 or 8; 1 acts as 2) pixels along a row and
 *                   forms the in-tile phase factors of the run from one
 *                   v_sin/v_cos and per-atom factors f_j exp(2 pi i k a.d_j).
 *                   Gradient (rows of a multiple of 64 pixels): the in-group
 *                   phase offset of pixel m is (m - 31.5) a.d_j.  With q_per_lane
 *                   32 both directions run as complex matrix products per atom
 *                   tile on 64 x 64 pixel rectangles (any row length), the
 *                   adjoint with two components when every q_z of the set is 0,
 *                   else three.  The factorized forms evaluate no sine per pair.
 * Shapes apply to calls and plans created after they are set.
 * Defaults: forward {64, 4, 64, 0, 0, 0}, gradient {64, 2, 128, 2048, 0, 0}.
 */
typedef struct xs_tile_shape {
    int32_t atoms_per_tile;
    int32_t q_per_lane;
    int32_t atom_split;
    int32_t pixel_split;
    int32_t waves_per_simd;
    int32_t lattice;
} xs_tile_shape;

/* kind: 0 = forward pair kernel, 1 = gradient pair kernel. */
xs_status xs_get_tile_shape(int32_t kind, xs_tile_shape *out);
xs_status xs_set_tile_shape(int32_t kind, const xs_tile_shape *shape);

/*
 * Batch plans (FP32C only): the one persistent, graph-capturable form of the
 * pair sums for a fixed batch layout and fixed pixels.
 *
 * xs_plan_create builds the work lists of the batch (every system and frame
 * of uneven atom count in one work queue, largest items first), allocates all
 * device memory the calls need, and orders the pixels along a Hilbert curve in
 * q (enqueued on `stream`).  The q array must stay at the same address and
 * unchanged for the life of the plan.  Tile shapes are those set by
 * xs_set_tile_shape when the plan is created.  It also tests every distinct
 * pixel set for rows (runs of n2 >= 8 consecutive pixels, n2 dividing n_q, whose
 * q_y are bitwise equal within each run) and for the row lattice (each q_p
 * within 1e-11 per Angstrom of q_row_start + j a), synchronizing `stream` to
 * read the results; the tile shapes' `lattice` then picks each set's form.
 *
 * xs_plan_intensity and xs_plan_grad then only launch kernels on `stream`
 * (no allocation, copy or memset), so a caller may capture them in a HIP
 * graph and replay it; positions, form factors and outputs may change between
 * replays in place.  Arguments as for xs_intensity_direct / xs_intensity_grad
 * with the plan's batch layout.  xs_plan_grad re-tiles the atoms when
 * `retile` is non-zero; with retile = 0 it reuses the tiles of the last
 * xs_plan_intensity (the positions must not have changed since; XS_EINVAL if
 * the plan has no tiles yet).  Calls on one plan must be ordered (one
 * stream); plans are not thread-safe.
 */
typedef struct xs_plan xs_plan;
xs_status xs_plan_create(const xs_batch *b, const double *q, xs_plan **plan, void *stream);
/*
 * xs_plan_create_forward: the same plan for the forward direct sum only (the
 * intensities of many frames, as the g2 and XSVS reductions of Secs. 4.4-4.5
 * consume them).  It leaves out the adjoint's work lists, its per-chunk partial
 * sums (3 doubles per atom and pixel chunk, the largest buffer of a full plan)
 * and its pixel prologue buffers; xs_plan_grad on it fails with XS_EINVAL and
 * launches nothing.  xs_plan_intensity is unchanged, bit for bit.
 */
xs_status xs_plan_create_forward(const xs_batch *b, const double *q, xs_plan **plan, void *stream);
xs_status xs_plan_intensity(xs_plan *plan, const double *pos, const double *f, double *I_out,
                            double *amp_out, void *stream);
xs_status xs_plan_grad(xs_plan *plan, const double *pos, const double *f, const double *amp,
                       const double *dL_dI, int32_t retile, float *dL_dr, double *dL_dr64,
                       void *stream);
/*
 * Species plans: the plan form of xs_intensity_species / xs_intensity_species_grad
 * (q-dependent form factors f_s(|q|) per species, Sec. 2.1, Eq. (pe_ri) with f_j(q)).
 * xs_plan_create_species reads `species` (device int32, the layout of f in the
 * batch, values in [0, n_species)) once and synchronizes `stream`; the species
 * assignment and `ff_coef` (host, [n_species][9] as for xs_intensity_species) are
 * fixed for the life of the plan.  The calls then only launch kernels (capturable
 * like xs_plan_intensity / xs_plan_grad): positions are gathered into species
 * order, the species segments run through the plan's pair sums with unit weights,
 * and the per-species amplitudes are combined with f_s(|q|) (adjoint: weighted by
 * f_s(|q|), gradients scattered back to the caller's atom order).  FP32C only.
 * pos, I_out, amp_out, amp, dL_dI, dL_dr, dL_dr64 as for the one-shot calls;
 * retile as for xs_plan_grad.  A species plan refuses xs_plan_intensity /
 * xs_plan_grad and the reverse (XS_EINVAL).  xs_plan_describe counts its species
 * segments.
 */
xs_status xs_plan_create_species(const xs_batch *b, const double *q, const int32_t *species,
                                 int32_t n_species, const double *ff_coef, xs_plan **plan,
                                 void *stream);
xs_status xs_plan_intensity_species(xs_plan *plan, const double *pos, double *I_out,
                                    double *amp_out, void *stream);
xs_status xs_plan_grad_species(xs_plan *plan, const double *pos, const double *amp,
                               const double *dL_dI, int32_t retile, float *dL_dr,
                               double *dL_dr64, void *stream);

/* Waits for the device, then frees the plan's memory.  NULL is accepted. */
xs_status xs_plan_destroy(xs_plan *plan);

/* What a plan holds: segments (systems x frames), the segments whose forward
 * pair sum uses the lattice form, the work items of the forward (all forms)
 * and gradient queues, the device memory owned by the plan, and the segments
 * whose forward pair sum uses the row form. */
typedef struct xs_plan_info {
    int32_t n_segments;
    int32_t n_lattice_segments;
    int32_t n_forward_items;
    int32_t n_gradient_items;
    int64_t device_bytes;
    int32_t n_row_segments;
    int32_t pad;             /* 0 */
} xs_plan_info;
xs_status xs_plan_describe(const xs_plan *plan, xs_plan_info *info);

/*
 * Speckle-matching loss of the differentiation workload and its gradient with
 * respect to the intensities (deterministic two-pass reduction, FP64):
 *     L = sum_p (I_p - It_p)^2 / sum_p It_p^2,   dL/dI_p = 2 (I_p - It_p) / sum_p It_p^2.
 *   I, I_target  device double [n]
 *   loss_out     device double [2]: (L, sum It^2)
 *   dL_dI        device double [n], or NULL
 */
xs_status xs_speckle_loss(const double *I, const double *I_target, int64_t n, double *loss_out,
                          double *dL_dI, void *stream);

/*
 * Gradient-descent update of positions, pos -= step * dL/dr (FP64 fused
 * multiply-add), from either gradient buffer (dL_dr64 preferred when both are
 * given).  pos, dL_dr, dL_dr64: device arrays of n values.
 */
xs_status xs_position_step(double *pos, const float *dL_dr, const double *dL_dr64, int64_t n,
                           double step, void *stream);

/*
 * Kernel timing with HIP events recorded on the stream each kernel runs on.
 * xs_timing_enable(1) clears the counters and starts recording; (0) stops.
 * xs_timing_read(kind) waits for the recorded events and returns the summed
 * duration (ms), number of launches and work (atom-pixel pairs for kinds 0-3,
 * atoms for 4, input bytes read once for 5-7) since enabling.
 *   kind 0: FP32C forward pair kernel   1: FP32C gradient pair kernel
 *        2: FP64 forward kernel         3: FP64 gradient kernel
 *        4: FP32C binning               5: g2 call     6: XSVS call
 *        7: xs_isf_rings call
 */
xs_status xs_timing_enable(int32_t on);
xs_status xs_timing_read(int32_t kind, double *total_ms, int64_t *launches, double *work);

/*
 * Roofline microbenchmarks (throughput of the units the kernels are bound by):
 *   kind 0: v_sin_f32 + v_cos_f32 lane operations per second
 *   kind 1: FP32 fused multiply-add lane operations per second (not packed)
 *   kind 2: FP64 fused multiply-add lane operations per second
 *   kind 3: HBM bytes per second (read + write) of a plain copy of `bytes`
 *   kind 4: FP16 matrix flops per second (v_mfma_f32_32x32x16_f16)
 *   kind 5: the same, each matrix instruction followed by 8 independent FP32
 *           FMAs of the same wavefront (equal to kind 4 if the two overlap)
 *   kind 6: HBM bytes per second of a plain read of `bytes`
 * Kinds 3 and 6 keep four 16-byte loads per thread in flight.
 * `rate` is a host double.  Uses the library's scratch memory.
 */
xs_status xs_roofline_probe(int32_t kind, int64_t bytes, double *rate, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* XS_H */
