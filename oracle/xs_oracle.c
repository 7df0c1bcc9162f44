/*
 * xs_oracle.c -- CPU FP64 oracle for the direct speckle-intensity method.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
 * its Python binding) may include, link, load or call this file; only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark do.  It
 * shares no code, header or constant with the GPU library: every formula here
 * is written out again from the paper (Mohanty, Cooper, Wang, Liang, Cai,
 * "Computational approaches to model X-ray photon correlation spectroscopy
 * from molecular dynamics", arXiv:2204.13241).
 *
 * Conventions (paper notation):
 *   - positions r_j: double [N][3] (Angstrom), used verbatim (no wrapping).
 *   - form factors f_j: double [N], q-independent per atom.
 *   - wavevectors q: double [Q][3] (1/Angstrom).
 *   - scattering amplitude, Sec. 2.2 Eq. (pe_ri):
 *         p^e(q) = sum_j f_j exp(-i q.r_j) = a + i b,
 *     stored as amp[p][0] = a, amp[p][1] = b.
 *   - intensity, Sec. 2.2 Eq. (Iq_pq): I(q) = |p^e(q)|^2.
 *
 * The "FP64 form" below fixes one exact operation sequence for the direct
 * method of Sec. 3.1 (Algorithm 1): it is the definition of Eq. (pe_ri) and
 * Eq. (Iq_pq) with the phase kept in revolutions and a sine/cosine built from
 * the Taylor series of sin and cos (coefficients (-1)^k/(2k+1)! and
 * (-1)^k/(2k)!) after an exact reduction to |angle| <= pi/4.  The GPU FP64
 * path implements the same sequence independently, so the two agree bit for
 * bit.  The libm and pair-sum variants are independent accuracy references.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math -shared -fPIC
 * (contraction off so that every fused multiply-add is an explicit fma()).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL 1
#define OR_ENOMEM 2

/* RN(1/(2 pi)), RN(2 pi), RN(2 pi - RN(2 pi)). */
static const double OR_INV2PI = 0x1.45f306dc9c883p-3;
static const double OR_TWOPI_HI = 0x1.921fb54442d18p+2;
static const double OR_TWOPI_LO = 0x1.1a62633145c07p-52;

/* Taylor coefficients RN((-1)^k/(2k+1)!) for sin (k = 1..7) and
 * RN((-1)^k/(2k)!) for cos (k = 1..8): each is one correctly rounded
 * division of exactly representable integers. */
static const double OR_S1 = -1.0 / 6.0;
static const double OR_S2 = 1.0 / 120.0;
static const double OR_S3 = -1.0 / 5040.0;
static const double OR_S4 = 1.0 / 362880.0;
static const double OR_S5 = -1.0 / 39916800.0;
static const double OR_S6 = 1.0 / 6227020800.0;
static const double OR_S7 = -1.0 / 1307674368000.0;
static const double OR_C1 = -1.0 / 2.0;
static const double OR_C2 = 1.0 / 24.0;
static const double OR_C3 = -1.0 / 720.0;
static const double OR_C4 = 1.0 / 40320.0;
static const double OR_C5 = -1.0 / 3628800.0;
static const double OR_C6 = 1.0 / 479001600.0;
static const double OR_C7 = -1.0 / 87178291200.0;
static const double OR_C8 = 1.0 / 20922789888000.0;

static int or_threads(int n_threads)
{
#ifdef _OPENMP
    return n_threads > 0 ? n_threads : omp_get_max_threads();
#else
    (void)n_threads;
    return 1;
#endif
}

static int omp_thread_index(void)
{
#ifdef _OPENMP
    return omp_get_thread_num();
#else
    return 0;
#endif
}

int32_t or_max_threads(void) { return or_threads(0); }

void or_constants(double *out)
{
    out[0] = OR_INV2PI;
    out[1] = OR_TWOPI_HI;
    out[2] = OR_TWOPI_LO;
}

/*
 * sin(2 pi t) and cos(2 pi t) for t in revolutions (the FP64 form).
 *   n = rint(t), u = t - n            exact, |u| <= 1/2
 *   m = rint(4u), v = u - m/4          exact (Sterbenz), |v| <= 1/8
 *   x = 2 pi v (two-term constant), z = x^2
 *   s = x + x z P_s(z), c = 1 + z P_c(z)   Taylor series, Horner with fma
 *   quadrant m mod 4 rotates (s, c) by m quarter turns.
 */
void or_sincos_rev(double t, double *sin_out, double *cos_out)
{
    double n = rint(t);
    double u = t - n;
    double mq = rint(4.0 * u);
    double v = u - mq * 0.25;
    double x = fma(OR_TWOPI_HI, v, OR_TWOPI_LO * v);
    double z = x * x;
    double ps = fma(z, OR_S7, OR_S6);
    ps = fma(z, ps, OR_S5);
    ps = fma(z, ps, OR_S4);
    ps = fma(z, ps, OR_S3);
    ps = fma(z, ps, OR_S2);
    ps = fma(z, ps, OR_S1);
    double s = fma(x * z, ps, x);
    double pc = fma(z, OR_C8, OR_C7);
    pc = fma(z, pc, OR_C6);
    pc = fma(z, pc, OR_C5);
    pc = fma(z, pc, OR_C4);
    pc = fma(z, pc, OR_C3);
    pc = fma(z, pc, OR_C2);
    pc = fma(z, pc, OR_C1);
    double c = fma(z, pc, 1.0);
    int quadrant = ((int)mq) & 3;
    switch (quadrant) {
    case 0: *sin_out = s;  *cos_out = c;  break;
    case 1: *sin_out = c;  *cos_out = -s; break;
    case 2: *sin_out = -s; *cos_out = -c; break;
    default: *sin_out = -c; *cos_out = s; break;
    }
}

void or_sincos_rev_n(int64_t n, const double *t, double *s, double *c)
{
    for (int64_t i = 0; i < n; ++i) or_sincos_rev(t[i], &s[i], &c[i]);
}

/* Phase of atom r under wavevector q, in revolutions: q.r / (2 pi). */
static inline double or_phase_rev(const double *qrev, const double *r)
{
    return fma(qrev[2], r[2], fma(qrev[1], r[1], qrev[0] * r[0]));
}

/*
 * Direct method (Sec. 3.1, Algorithm 1; Eqs. (pe_ri), (Iq_pq)), FP64 form.
 * For every pixel p, atoms are summed in input order starting from +0.0:
 *   ac += f_j cos(q.r_j), as += f_j sin(q.r_j)   (fma)
 *   a = ac, b = -as  (the amplitude carries exp(-i q.r)),  I = a*a + b*b.
 * amp may be NULL.
 */
int or_intensity(int64_t n_atoms, const double *pos, const double *f,
                 int64_t n_q, const double *q, double *I, double *amp,
                 int n_threads)
{
    if (n_atoms < 0 || n_q < 0 || (n_q > 0 && (!q || !I)) ||
        (n_atoms > 0 && (!pos || !f)))
        return OR_EINVAL;
#pragma omp parallel for schedule(static) num_threads(or_threads(n_threads))
    for (int64_t p = 0; p < n_q; ++p) {
        double qrev[3];
        for (int k = 0; k < 3; ++k) qrev[k] = q[3 * p + k] * OR_INV2PI;
        double ac = 0.0, as = 0.0;
        for (int64_t j = 0; j < n_atoms; ++j) {
            double s, c;
            or_sincos_rev(or_phase_rev(qrev, pos + 3 * j), &s, &c);
            ac = fma(f[j], c, ac);
            as = fma(f[j], s, as);
        }
        double a = ac, b = -as;
        I[p] = fma(a, a, b * b);
        if (amp) { amp[2 * p] = a; amp[2 * p + 1] = b; }
    }
    return OR_OK;
}

/*
 * Same sum with the C library's long-double sine and cosine of the phase in
 * radians: an independent accuracy reference for the FP64 form.
 */
int or_intensity_libm(int64_t n_atoms, const double *pos, const double *f,
                      int64_t n_q, const double *q, double *I, double *amp,
                      int n_threads)
{
    if (n_atoms < 0 || n_q < 0) return OR_EINVAL;
#pragma omp parallel for schedule(static) num_threads(or_threads(n_threads))
    for (int64_t p = 0; p < n_q; ++p) {
        long double ac = 0.0L, as = 0.0L;
        for (int64_t j = 0; j < n_atoms; ++j) {
            long double ph = (long double)q[3 * p] * pos[3 * j] +
                             (long double)q[3 * p + 1] * pos[3 * j + 1] +
                             (long double)q[3 * p + 2] * pos[3 * j + 2];
            ac += f[j] * cosl(ph);
            as += f[j] * sinl(ph);
        }
        double a = (double)ac, b = (double)(-as);
        I[p] = (double)(ac * ac + as * as);
        if (amp) { amp[2 * p] = a; amp[2 * p + 1] = b; }
    }
    return OR_OK;
}

/*
 * Pair double sum, Sec. 2.1 Eq. (Iq_rij):
 *   I(q) = sum_i sum_j f_i f_j exp(-i q.(r_i - r_j)) = sum_i sum_j f_i f_j cos(q.(r_i - r_j)),
 * the sine terms cancelling pairwise.  O(N^2) per pixel: brute force for small N.
 */
int or_intensity_pairsum(int64_t n_atoms, const double *pos, const double *f,
                         int64_t n_q, const double *q, double *I)
{
    if (n_atoms < 0 || n_q < 0) return OR_EINVAL;
    for (int64_t p = 0; p < n_q; ++p) {
        long double acc = 0.0L;
        for (int64_t i = 0; i < n_atoms; ++i)
            for (int64_t j = 0; j < n_atoms; ++j) {
                long double ph = 0.0L;
                for (int k = 0; k < 3; ++k)
                    ph += (long double)q[3 * p + k] *
                          ((long double)pos[3 * i + k] - (long double)pos[3 * j + k]);
                acc += (long double)f[i] * f[j] * cosl(ph);
            }
        I[p] = (double)acc;
    }
    return OR_OK;
}

/*
 * Gradient of a functional of the intensities with respect to the positions
 * (the chain rule through Eqs. (pe_ri) and (Iq_pq)).  Given w_p = dL/dI_p and
 * the amplitude a_p + i b_p of the same positions:
 *   dI_p/dr_j = -2 f_j q_p (a_p sin(q_p.r_j) + b_p cos(q_p.r_j)),
 *   dL/dr_j   = sum_p w_p dI_p/dr_j.
 * FP64 form: per atom, pixels in input order from +0.0;
 *   h = fma(a, s, b*c); k = w*h; g += k*q (fma per component);
 *   dL/dr_j = (-2 f_j) * g.
 */
int or_intensity_grad(int64_t n_atoms, const double *pos, const double *f,
                      int64_t n_q, const double *q, const double *amp,
                      const double *dL_dI, double *dL_dr, int n_threads)
{
    if (n_atoms < 0 || n_q < 0 || (n_atoms > 0 && (!pos || !f || !dL_dr)) ||
        (n_q > 0 && (!q || !amp || !dL_dI)))
        return OR_EINVAL;
#pragma omp parallel for schedule(static) num_threads(or_threads(n_threads))
    for (int64_t j = 0; j < n_atoms; ++j) {
        double gx = 0.0, gy = 0.0, gz = 0.0;
        for (int64_t p = 0; p < n_q; ++p) {
            double qrev[3];
            for (int k = 0; k < 3; ++k) qrev[k] = q[3 * p + k] * OR_INV2PI;
            double s, c;
            or_sincos_rev(or_phase_rev(qrev, pos + 3 * j), &s, &c);
            double h = fma(amp[2 * p], s, amp[2 * p + 1] * c);
            double k = dL_dI[p] * h;
            gx = fma(k, q[3 * p], gx);
            gy = fma(k, q[3 * p + 1], gy);
            gz = fma(k, q[3 * p + 2], gz);
        }
        double m = -2.0 * f[j];
        dL_dr[3 * j] = m * gx;
        dL_dr[3 * j + 1] = m * gy;
        dL_dr[3 * j + 2] = m * gz;
    }
    return OR_OK;
}

/* Kahan-Babuska (Neumaier) compensated sum step in long double. */
static inline void or_nsum(long double *sum, long double *comp, long double x)
{
    long double t = *sum + x;
    if (fabsl(*sum) >= fabsl(x)) *comp += (*sum - t) + x;
    else *comp += (x - t) + *sum;
    *sum = t;
}

/*
 * Central finite differences of L(r) = sum_p w_p I_p(r) for selected atoms:
 *   dL/dr_{j,c} ~ (L(r + h e_{jc}) - L(r - h e_{jc})) / (2h).
 * Displacing one atom changes the amplitude by a rank-one term,
 *   p'(q) = p(q) + f_j (exp(-i q.r_j') - exp(-i q.r_j)),
 * so each evaluation costs O(Q); the difference of the two sums is formed
 * term by term, sum_p w_p (I+ - I-), with a compensated long-double sum.
 * Sines and cosines come from the C library (independent of the FP64 form).
 * out: [n_sel][3].
 */
int or_fd_grad(int64_t n_atoms, const double *pos, const double *f,
               int64_t n_q, const double *q, const double *dL_dI,
               int64_t n_sel, const int64_t *atoms, double h, double *out,
               int n_threads)
{
    if (n_atoms <= 0 || n_q < 0 || n_sel < 0 || !(h > 0.0)) return OR_EINVAL;
    for (int64_t s = 0; s < n_sel; ++s)
        if (atoms[s] < 0 || atoms[s] >= n_atoms) return OR_EINVAL;
    long double *ar = malloc(sizeof(long double) * (size_t)(n_q > 0 ? n_q : 1));
    long double *ai = malloc(sizeof(long double) * (size_t)(n_q > 0 ? n_q : 1));
    if (!ar || !ai) { free(ar); free(ai); return OR_ENOMEM; }
    /* Amplitude of the unperturbed positions, long double. */
#pragma omp parallel for schedule(static) num_threads(or_threads(n_threads))
    for (int64_t p = 0; p < n_q; ++p) {
        long double sr = 0.0L, si = 0.0L;
        for (int64_t j = 0; j < n_atoms; ++j) {
            long double ph = (long double)q[3 * p] * pos[3 * j] +
                             (long double)q[3 * p + 1] * pos[3 * j + 1] +
                             (long double)q[3 * p + 2] * pos[3 * j + 2];
            sr += f[j] * cosl(ph);
            si -= f[j] * sinl(ph);
        }
        ar[p] = sr; ai[p] = si;
    }
    for (int64_t s = 0; s < n_sel; ++s) {
        int64_t j = atoms[s];
        for (int c = 0; c < 3; ++c) {
            long double sum = 0.0L, comp = 0.0L;
#pragma omp parallel num_threads(or_threads(n_threads))
            {
                long double lsum = 0.0L, lcomp = 0.0L;
#pragma omp for schedule(static)
                for (int64_t p = 0; p < n_q; ++p) {
                    long double r0[3] = {pos[3 * j], pos[3 * j + 1], pos[3 * j + 2]};
                    long double ph0 = q[3 * p] * r0[0] + q[3 * p + 1] * r0[1] + q[3 * p + 2] * r0[2];
                    long double dph = (long double)q[3 * p + c] * h;
                    long double php = ph0 + dph, phm = ph0 - dph;
                    /* p(r +/- h e) = p(r) + f_j (exp(-i ph+-) - exp(-i ph0)) */
                    long double br = ar[p] - f[j] * cosl(ph0);
                    long double bi = ai[p] + f[j] * sinl(ph0);
                    long double pr = br + f[j] * cosl(php), pi = bi - f[j] * sinl(php);
                    long double mr = br + f[j] * cosl(phm), mi = bi - f[j] * sinl(phm);
                    long double Ip = pr * pr + pi * pi, Im = mr * mr + mi * mi;
                    or_nsum(&lsum, &lcomp, (long double)dL_dI[p] * (Ip - Im));
                }
#pragma omp critical
                {
                    or_nsum(&sum, &comp, lsum);
                    or_nsum(&sum, &comp, lcomp);
                }
            }
            out[3 * s + c] = (double)((sum + comp) / (2.0L * h));
        }
    }
    free(ar); free(ai);
    return OR_OK;
}

/*
 * |q| ring of every pixel: ring r holds e_r <= |q| < e_{r+1} (the half-open
 * shell q - dq/2 <= |q| < q + dq/2 of Sec. 2.3, Eq. (bq_Iq)); pixels outside
 * [e_0, e_R) get -1.  |q| = sqrt(fma(qz, qz, fma(qy, qy, qx*qx))).
 */
int or_ring_index(int64_t n_q, const double *q, int32_t n_rings,
                  const double *edges, int32_t *ring)
{
    if (n_q < 0 || n_rings <= 0 || !edges || (n_q > 0 && (!q || !ring))) return OR_EINVAL;
    for (int32_t r = 0; r < n_rings; ++r)
        if (!(edges[r] < edges[r + 1])) return OR_EINVAL;
    for (int64_t p = 0; p < n_q; ++p) {
        double qx = q[3 * p], qy = q[3 * p + 1], qz = q[3 * p + 2];
        double qn = sqrt(fma(qz, qz, fma(qy, qy, qx * qx)));
        int32_t idx = -1;
        for (int32_t r = 0; r < n_rings; ++r)
            if (edges[r] <= qn && qn < edges[r + 1]) { idx = r; break; }
        ring[p] = idx;
    }
    return OR_OK;
}

/*
 * Pairwise sum of x[0..n), n >= 1, in the given order: adjacent pairs are
 * added level by level, x'[i] = x[2i] + x[2i+1], an odd last element moving up
 * unchanged, until one value is left.  This is the tree that splits [0, n) at
 * the largest power of two below n and sums both parts the same way.
 * Overwrites x.
 */
static double or_pairwise(double *x, int64_t n)
{
    while (n > 1) {
        int64_t h = n / 2;
        for (int64_t i = 0; i < h; ++i) x[i] = x[2 * i] + x[2 * i + 1];
        if (n & 1) x[h] = x[n - 1];
        n = h + (n & 1);
    }
    return x[0];
}

/* Members of each ring in ascending pixel index: start[r] .. start[r+1] of
 * list (start has n_rings + 1 entries).  Pixels with ring < 0 or keep[p] == 0
 * (keep may be NULL) are left out. */
static int or_ring_lists(int64_t n_q, const int32_t *ring, const unsigned char *keep,
                         int32_t n_rings, int64_t **start_out, int64_t **list_out)
{
    int64_t *start = calloc((size_t)n_rings + 1, sizeof(int64_t));
    int64_t *list = malloc(sizeof(int64_t) * (size_t)(n_q > 0 ? n_q : 1));
    if (!start || !list) { free(start); free(list); return OR_ENOMEM; }
    for (int64_t p = 0; p < n_q; ++p)
        if (ring[p] >= 0 && (!keep || keep[p])) start[ring[p] + 1]++;
    for (int32_t r = 0; r < n_rings; ++r) start[r + 1] += start[r];
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)n_rings);
    if (!fill) { free(start); free(list); return OR_ENOMEM; }
    for (int32_t r = 0; r < n_rings; ++r) fill[r] = start[r];
    for (int64_t p = 0; p < n_q; ++p)
        if (ring[p] >= 0 && (!keep || keep[p])) list[fill[ring[p]]++] = p;
    free(fill);
    *start_out = start;
    *list_out = list;
    return OR_OK;
}

/*
 * Intensity autocorrelation on |q| rings, Sec. 2.3 Eq. (g2_def) with the
 * ring average of Sec. 4.2:
 *   per pixel  G_p(tau) = [ sum_{t < F-tau} I_t I_{t+tau} / (F - tau) ] / <I>_t^2,
 *              <I>_t = sum_t I_t / F   (all F frames),
 *   per ring   g2(r, tau) = mean of G_p(tau) over the ring's pixels.
 * I: [F][Q] (pixel fastest).  Pixels whose <I>_t^2 is zero are left out and
 * not counted.  Fixed order: time sums sequential in t (products by fma),
 * ring sums pairwise over the ring's pixels in ascending index (or_pairwise).
 * Empty rings give NaN.  g2: [n_rings][n_tau]; count (may be NULL): [n_rings].
 */
int or_g2_rings(const double *I, int64_t n_frames, int64_t n_q, const double *q,
                const double *edges, int32_t n_rings, int32_t n_tau,
                double *g2, int32_t *count, int n_threads)
{
    if (n_frames <= 0 || n_q < 0 || n_rings <= 0 || n_tau <= 0 || n_tau > n_frames ||
        !g2)
        return OR_EINVAL;
    int32_t *ring = malloc(sizeof(int32_t) * (size_t)(n_q > 0 ? n_q : 1));
    double *G = malloc(sizeof(double) * (size_t)(n_q > 0 ? n_q : 1) * (size_t)n_tau);
    unsigned char *used = malloc((size_t)(n_q > 0 ? n_q : 1));
    if (!ring || !G || !used) { free(ring); free(G); free(used); return OR_ENOMEM; }
    int rc = or_ring_index(n_q, q, n_rings, edges, ring);
    if (rc != OR_OK) { free(ring); free(G); free(used); return rc; }
#pragma omp parallel for schedule(static) num_threads(or_threads(n_threads))
    for (int64_t p = 0; p < n_q; ++p) {
        double S = 0.0;
        for (int64_t t = 0; t < n_frames; ++t) S = S + I[t * n_q + p];
        double mean = S / (double)n_frames;
        double den = mean * mean;
        used[p] = (den != 0.0);
        for (int32_t tau = 0; tau < n_tau; ++tau) {
            double acc = 0.0;
            for (int64_t t = 0; t + tau < n_frames; ++t)
                acc = fma(I[t * n_q + p], I[(t + tau) * n_q + p], acc);
            G[p * n_tau + tau] = (acc / (double)(n_frames - tau)) / den;
        }
    }
    int64_t *start = NULL, *list = NULL;
    rc = or_ring_lists(n_q, ring, used, n_rings, &start, &list);
    if (rc != OR_OK) { free(ring); free(G); free(used); return rc; }
    double *buf = malloc(sizeof(double) * (size_t)(n_q > 0 ? n_q : 1));
    if (!buf) { free(ring); free(G); free(used); free(start); free(list); return OR_ENOMEM; }
    for (int32_t r = 0; r < n_rings; ++r) {
        const int64_t cnt = start[r + 1] - start[r];
        if (count) count[r] = (int32_t)cnt;
        for (int32_t tau = 0; tau < n_tau; ++tau) {
            double mean = NAN;
            if (cnt > 0) {
                for (int64_t m = 0; m < cnt; ++m) buf[m] = G[list[start[r] + m] * n_tau + tau];
                mean = or_pairwise(buf, cnt) / (double)cnt;
            }
            g2[(int64_t)r * n_tau + tau] = mean;
        }
    }
    free(ring); free(G); free(used); free(start); free(list); free(buf);
    return OR_OK;
}

/*
 * XSVS contrast versus exposure, Sec. 2.3 Eqs. (inte_Iq), (bq_Iq):
 *   exposure integral over W = 2^l frames as non-overlapping windows from
 *   frame 0 (trailing partial window dropped), built pairwise:
 *       J_0[k] = I_k,   J_{l+1}[k] = J_l[2k] + J_l[2k+1],  K_l = floor(F / 2^l);
 *   per (level l, window k, ring r) over the ring's pixels in ascending order,
 *   the moments of Eq. (bq_Iq) as written there:
 *       m1 = sum J / n,  m2 = sum J^2 / n  (both sums pairwise, or_pairwise,
 *       over the rounded values J and J*J),
 *       beta = (m2 - m1^2) / m1^2,  m1^2 rounded once;
 *   beta_out[l][r] = sum_k beta / K_l  (sequential in k).
 * I: [F][Q].  beta_out: [n_levels][n_rings].  beta_win (may be NULL):
 * [n_levels][F][n_rings], entries k >= K_l set to NaN.  Empty rings: NaN.
 */
int or_xsvs_contrast(const double *I, int64_t n_frames, int64_t n_q, const double *q,
                     const double *edges, int32_t n_rings, int32_t n_levels,
                     double *beta_out, double *beta_win, int n_threads)
{
    if (n_frames <= 0 || n_q < 0 || n_rings <= 0 || n_levels <= 0 || n_levels > 62 ||
        ((int64_t)1 << (n_levels - 1)) > n_frames || !beta_out)
        return OR_EINVAL;
    int32_t *ring = malloc(sizeof(int32_t) * (size_t)(n_q > 0 ? n_q : 1));
    double *J = malloc(sizeof(double) * (size_t)n_frames * (size_t)(n_q > 0 ? n_q : 1));
    if (!ring || !J) { free(ring); free(J); return OR_ENOMEM; }
    int rc = or_ring_index(n_q, q, n_rings, edges, ring);
    if (rc != OR_OK) { free(ring); free(J); return rc; }
    memcpy(J, I, sizeof(double) * (size_t)n_frames * (size_t)n_q);
    int64_t *start = NULL, *list = NULL;
    rc = or_ring_lists(n_q, ring, NULL, n_rings, &start, &list);
    if (rc != OR_OK) { free(ring); free(J); return rc; }
    int32_t *cnt = calloc((size_t)n_rings, sizeof(int32_t));
    if (!cnt) { free(ring); free(J); free(start); free(list); return OR_ENOMEM; }
    for (int32_t r = 0; r < n_rings; ++r) cnt[r] = (int32_t)(start[r + 1] - start[r]);
    const int nth = or_threads(n_threads);
    double *bufs = malloc(sizeof(double) * (size_t)(n_q > 0 ? n_q : 1) * (size_t)nth);
    if (!bufs) { free(ring); free(J); free(start); free(list); free(cnt); return OR_ENOMEM; }
    if (beta_win)
        for (int64_t i = 0; i < (int64_t)n_levels * n_frames * n_rings; ++i) beta_win[i] = NAN;
    int64_t K = n_frames;
    for (int32_t l = 0; l < n_levels; ++l) {
        if (l > 0) {
            int64_t Kn = K / 2;
            for (int64_t k = 0; k < Kn; ++k)
                for (int64_t p = 0; p < n_q; ++p)
                    J[k * n_q + p] = J[(2 * k) * n_q + p] + J[(2 * k + 1) * n_q + p];
            K = Kn;
        }
        double *bw = malloc(sizeof(double) * (size_t)K * (size_t)n_rings);
        if (!bw) { free(ring); free(J); free(cnt); free(start); free(list); free(bufs); return OR_ENOMEM; }
#pragma omp parallel for schedule(static) num_threads(nth)
        for (int64_t k = 0; k < K; ++k) {
            double *buf = bufs + (size_t)omp_thread_index() * (size_t)(n_q > 0 ? n_q : 1);
            for (int32_t r = 0; r < n_rings; ++r) {
                double b = NAN;
                const int64_t n = cnt[r];
                if (n > 0) {
                    const int64_t *mem = list + start[r];
                    for (int64_t m = 0; m < n; ++m) buf[m] = J[k * n_q + mem[m]];
                    const double m1 = or_pairwise(buf, n) / (double)n;
                    for (int64_t m = 0; m < n; ++m) {
                        const double x = J[k * n_q + mem[m]];
                        buf[m] = x * x;
                    }
                    const double m2 = or_pairwise(buf, n) / (double)n;
                    const double sq = m1 * m1;
                    b = (m2 - sq) / sq;
                }
                bw[k * n_rings + r] = b;
            }
        }
        for (int32_t r = 0; r < n_rings; ++r) {
            double acc = 0.0;
            for (int64_t k = 0; k < K; ++k) acc = acc + bw[k * n_rings + r];
            beta_out[(int64_t)l * n_rings + r] = cnt[r] > 0 ? acc / (double)K : NAN;
            if (beta_win)
                for (int64_t k = 0; k < K; ++k)
                    beta_win[((int64_t)l * n_frames + k) * n_rings + r] = bw[k * n_rings + r];
        }
        free(bw);
    }
    free(ring); free(J); free(cnt); free(start); free(list); free(bufs);
    return OR_OK;
}

/*
 * Intermediate scattering function on |q| rings, Sec. 2.3 Eq. (Fq_pq) with the
 * ring average of Sec. 4.2:
 *   per pixel  F_p(tau) = [ sum_{t < F-tau} p_t conj(p_{t+tau}) / (F - tau) ] / sum_j f_j^2,
 *              p_t = a_t + i b_t, the amplitude of Eq. (pe_ri) in frame t, so
 *              p_t conj(p_{t+tau}) = (a_t a_{t+tau} + b_t b_{t+tau})
 *                                  + i (b_t a_{t+tau} - a_t b_{t+tau});
 *   per ring   F(r, tau) = mean of F_p(tau) over every pixel of the ring (real
 *              and imaginary parts separately).
 * amp: [F][Q][2] (a, b).  f2_sum = sum_j f_j^2 > 0.  Fixed order: for each t
 * ascending, re = fma(a_t, a_{t+tau}, re), re = fma(b_t, b_{t+tau}, re),
 * im = fma(b_t, a_{t+tau}, im), im = fma(-a_t, b_{t+tau}, im), from +0.0;
 * F_p = (sum / (F - tau)) / f2_sum; ring sums pairwise (or_pairwise) in
 * ascending pixel index, then / n.  Empty rings give NaN.
 * F_out: [n_rings][n_tau][2]; count (may be NULL): [n_rings].
 */
int or_isf_rings(const double *amp, int64_t n_frames, int64_t n_q, const double *q,
                 const double *edges, int32_t n_rings, int32_t n_tau, double f2_sum,
                 double *F_out, int32_t *count, int n_threads)
{
    if (n_frames <= 0 || n_q < 0 || n_rings <= 0 || n_tau <= 0 || n_tau > n_frames ||
        !(f2_sum > 0.0) || !isfinite(f2_sum) || !F_out)
        return OR_EINVAL;
    int32_t *ring = malloc(sizeof(int32_t) * (size_t)(n_q > 0 ? n_q : 1));
    double *Fp = malloc(sizeof(double) * (size_t)(n_q > 0 ? n_q : 1) * (size_t)n_tau * 2);
    if (!ring || !Fp) { free(ring); free(Fp); return OR_ENOMEM; }
    int rc = or_ring_index(n_q, q, n_rings, edges, ring);
    if (rc != OR_OK) { free(ring); free(Fp); return rc; }
#pragma omp parallel for schedule(static) num_threads(or_threads(n_threads))
    for (int64_t p = 0; p < n_q; ++p) {
        for (int32_t tau = 0; tau < n_tau; ++tau) {
            double re = 0.0, im = 0.0;
            for (int64_t t = 0; t + tau < n_frames; ++t) {
                const double a0 = amp[2 * (t * n_q + p)], b0 = amp[2 * (t * n_q + p) + 1];
                const double a1 = amp[2 * ((t + tau) * n_q + p)], b1 = amp[2 * ((t + tau) * n_q + p) + 1];
                re = fma(a0, a1, re);
                re = fma(b0, b1, re);
                im = fma(b0, a1, im);
                im = fma(-a0, b1, im);
            }
            const double nt = (double)(n_frames - tau);
            Fp[(p * n_tau + tau) * 2] = (re / nt) / f2_sum;
            Fp[(p * n_tau + tau) * 2 + 1] = (im / nt) / f2_sum;
        }
    }
    int64_t *start = NULL, *list = NULL;
    rc = or_ring_lists(n_q, ring, NULL, n_rings, &start, &list);
    if (rc != OR_OK) { free(ring); free(Fp); return rc; }
    double *buf = malloc(sizeof(double) * (size_t)(n_q > 0 ? n_q : 1));
    if (!buf) { free(ring); free(Fp); free(start); free(list); return OR_ENOMEM; }
    for (int32_t r = 0; r < n_rings; ++r) {
        const int64_t cnt = start[r + 1] - start[r];
        if (count) count[r] = (int32_t)cnt;
        for (int32_t tau = 0; tau < n_tau; ++tau)
            for (int c = 0; c < 2; ++c) {
                double mean = NAN;
                if (cnt > 0) {
                    for (int64_t m = 0; m < cnt; ++m) buf[m] = Fp[(list[start[r] + m] * n_tau + tau) * 2 + c];
                    mean = or_pairwise(buf, cnt) / (double)cnt;
                }
                F_out[((int64_t)r * n_tau + tau) * 2 + c] = mean;
            }
    }
    free(ring); free(Fp); free(start); free(list); free(buf);
    return OR_OK;
}

/*
 * Siegert relation and the exposure contrast it predicts, Sec. 2.3
 * Eqs. (bq_g2), (norm_Fq), (g2_from_fq), (beta_alt_int), per ring r:
 *   beta0(r)      = g2(r, 0) - 1                          Eq. (bq_g2)
 *   lhs(r, tau)   = (g2(r, tau) - 1) / beta0(r)           measured side of Eq. (g2_from_fq)
 *   fhat2(r, tau) = |F(r, tau)|^2 / |F(r, 0)|^2           |F-hat|^2, Eq. (norm_Fq)
 *   beta(l, r)    = beta0(r) * (1 + 2 s) / W,  W = 2^l,
 *                   s = sum_{k=1}^{W-1} (1 - k/W) fhat2(r, k)
 * The last line is Eq. (beta_alt_int) for an exposure that is the sum of W
 * consecutive frames (the rectangle rule of Eq. (inte_Iq)): the variance of
 * the window sum is the double sum of the frame covariances, and the Siegert
 * relation gives each as <I>^2 beta0 |F-hat(k)|^2 at lag k.
 * |z|^2 = fma(re, re, im*im); s by fma over k = 1, 2, ..., from +0.0, with
 * the exact weight 1 - k/W; 1 + 2 s as fma(2, s, 1).
 * g2: [R][n_tau]; F: [R][n_tau][2]; lhs, fhat2: [R][n_tau]; beta_pred:
 * [n_levels][R]; needs 2^(n_levels-1) <= n_tau.
 */
int or_siegert(const double *g2, const double *F, int32_t n_rings, int32_t n_tau,
               int32_t n_levels, double *lhs, double *fhat2, double *beta_pred)
{
    if (n_rings <= 0 || n_tau <= 0 || n_levels < 0 || n_levels > 30 ||
        (n_levels > 0 && ((int64_t)1 << (n_levels - 1)) > n_tau) || !g2 || !F)
        return OR_EINVAL;
    for (int32_t r = 0; r < n_rings; ++r) {
        const double beta0 = g2[(int64_t)r * n_tau] - 1.0;
        const double *Fr = F + (int64_t)r * n_tau * 2;
        const double f0 = fma(Fr[0], Fr[0], Fr[1] * Fr[1]);
        for (int32_t tau = 0; tau < n_tau; ++tau) {
            if (lhs) lhs[(int64_t)r * n_tau + tau] = (g2[(int64_t)r * n_tau + tau] - 1.0) / beta0;
            if (fhat2)
                fhat2[(int64_t)r * n_tau + tau] =
                    fma(Fr[2 * tau], Fr[2 * tau], Fr[2 * tau + 1] * Fr[2 * tau + 1]) / f0;
        }
        for (int32_t l = 0; l < n_levels && beta_pred; ++l) {
            const int64_t W = (int64_t)1 << l;
            double s = 0.0;
            for (int64_t k = 1; k < W; ++k) {
                const double fh = fma(Fr[2 * k], Fr[2 * k], Fr[2 * k + 1] * Fr[2 * k + 1]) / f0;
                s = fma(1.0 - (double)k / (double)W, fh, s);
            }
            beta_pred[(int64_t)l * n_rings + r] = beta0 * fma(2.0, s, 1.0) / (double)W;
        }
    }
    return OR_OK;
}

/*
 * X-ray atomic form factor of a species at wavevector magnitude |q|, as a sum
 * of Gaussians (Sec. 2.1: the form factor is well parameterized by a sum of
 * Gaussians, the International Tables form):
 *     f_s(q) = c + sum_{i=1..4} a_i exp(-b_i s^2),   s = |q| / (4 pi),
 * coef[s] = {a_1, a_2, a_3, a_4, b_1, b_2, b_3, b_4, c} (b in Angstrom^2).
 * s^2 = (q.q) / (16 pi^2); the four terms are added to c in order i = 1..4.
 */
static double or_form_factor(const double *coef, const double *qv)
{
    const double qq = fma(qv[2], qv[2], fma(qv[1], qv[1], qv[0] * qv[0]));
    const double s2 = qq / (16.0 * M_PI * M_PI);
    double f = coef[8];
    for (int i = 0; i < 4; ++i) f = f + coef[i] * exp(-coef[4 + i] * s2);
    return f;
}

/* f_s(|q|) for every pixel and species: out[p][s]. */
int or_form_factors(int64_t n_q, const double *q, int32_t n_species, const double *coef, double *out)
{
    if (n_q < 0 || n_species <= 0 || !coef || (n_q > 0 && (!q || !out))) return OR_EINVAL;
    for (int64_t p = 0; p < n_q; ++p)
        for (int32_t s = 0; s < n_species; ++s) out[p * n_species + s] = or_form_factor(coef + 9 * s, q + 3 * p);
    return OR_OK;
}

/*
 * Direct method with q-dependent form factors, Eqs. (Iq_rij), (pe_ri) with
 * f_j(q) = f_{species[j]}(|q|): for every pixel, atoms summed in input order
 * from +0.0 with the FP64-form sine and cosine,
 *   ac += f_j(q) cos(q.r_j), as += f_j(q) sin(q.r_j)   (fma),
 *   a = ac, b = -as, I = a*a + b*b.
 * species: [N] in 0 .. n_species-1; coef: [n_species][9] as above.
 */
int or_intensity_species(int64_t n_atoms, const double *pos, const int32_t *species, int32_t n_species,
                         const double *coef, int64_t n_q, const double *q, double *I, double *amp,
                         int n_threads)
{
    if (n_atoms < 0 || n_q < 0 || n_species <= 0 || !coef || (n_q > 0 && (!q || !I)) ||
        (n_atoms > 0 && (!pos || !species)))
        return OR_EINVAL;
    for (int64_t j = 0; j < n_atoms; ++j)
        if (species[j] < 0 || species[j] >= n_species) return OR_EINVAL;
    int rc = OR_OK;
#pragma omp parallel num_threads(or_threads(n_threads))
    {
        double *fs = malloc(sizeof(double) * (size_t)n_species);
        if (!fs) {
#pragma omp atomic write
            rc = OR_ENOMEM;
        }
#pragma omp for schedule(static)
        for (int64_t p = 0; p < n_q; ++p) {
            if (!fs) continue;
            double qrev[3];
            for (int k = 0; k < 3; ++k) qrev[k] = q[3 * p + k] * OR_INV2PI;
            for (int32_t s = 0; s < n_species; ++s) fs[s] = or_form_factor(coef + 9 * s, q + 3 * p);
            double ac = 0.0, as = 0.0;
            for (int64_t j = 0; j < n_atoms; ++j) {
                double sn, cs;
                or_sincos_rev(or_phase_rev(qrev, pos + 3 * j), &sn, &cs);
                const double fj = fs[species[j]];
                ac = fma(fj, cs, ac);
                as = fma(fj, sn, as);
            }
            double a = ac, b = -as;
            I[p] = fma(a, a, b * b);
            if (amp) { amp[2 * p] = a; amp[2 * p + 1] = b; }
        }
        free(fs);
    }
    return rc;
}

/*
 * Gradient of L = sum_p w_p I_p with q-dependent form factors (chain rule
 * through Eqs. (pe_ri), (Iq_pq) with f_j(q)): with the amplitude a_p + i b_p of
 * the same positions,
 *   dI_p/dr_j = -2 f_j(q_p) q_p (a_p sin(q_p.r_j) + b_p cos(q_p.r_j)),
 *   dL/dr_j   = sum_p w_p dI_p/dr_j.
 * FP64 form: per atom, pixels in input order from +0.0;
 *   h = fma(a, s, b*c); k = (w * f_j(q)) * h; g += k*q (fma per component);
 *   dL/dr_j = -2 g.
 */
int or_intensity_species_grad(int64_t n_atoms, const double *pos, const int32_t *species, int32_t n_species,
                              const double *coef, int64_t n_q, const double *q, const double *amp,
                              const double *dL_dI, double *grad, int n_threads)
{
    if (n_atoms < 0 || n_q < 0 || n_species <= 0 || !coef || (n_atoms > 0 && (!pos || !species || !grad)) ||
        (n_q > 0 && (!q || !amp || !dL_dI)))
        return OR_EINVAL;
    for (int64_t j = 0; j < n_atoms; ++j)
        if (species[j] < 0 || species[j] >= n_species) return OR_EINVAL;
    double *fq = malloc(sizeof(double) * (size_t)(n_q > 0 ? n_q : 1) * (size_t)n_species);
    if (!fq) return OR_ENOMEM;
    or_form_factors(n_q, q, n_species, coef, fq);
#pragma omp parallel for schedule(static) num_threads(or_threads(n_threads))
    for (int64_t j = 0; j < n_atoms; ++j) {
        double g[3] = {0.0, 0.0, 0.0};
        for (int64_t p = 0; p < n_q; ++p) {
            double qrev[3];
            for (int k = 0; k < 3; ++k) qrev[k] = q[3 * p + k] * OR_INV2PI;
            double sn, cs;
            or_sincos_rev(or_phase_rev(qrev, pos + 3 * j), &sn, &cs);
            const double a = amp[2 * p], b = amp[2 * p + 1];
            const double h = fma(a, sn, b * cs);
            const double k = (dL_dI[p] * fq[p * n_species + species[j]]) * h;
            for (int c = 0; c < 3; ++c) g[c] = fma(k, q[3 * p + c], g[c]);
        }
        for (int c = 0; c < 3; ++c) grad[3 * j + c] = -2.0 * g[c];
    }
    free(fq);
    return OR_OK;
}

/*
 * Sums of frames: incoherent superposition of independent configurations
 * (Sec. 4.5: the speckle of several scattering volumes is the sum of their
 * intensities) and exposure integrals over consecutive frames (Eq. (inte_Iq),
 * rectangle rule), one definition for both:
 *     J[k][p] = sum_{i < n_sum} I[k * s_out + i * s_sum][p],   k < n_out,
 * each sum the pairwise tree over i in ascending order (adjacent pairs added
 * level by level, an odd last element carried up: for n_sum = 2^l and
 * s_sum = 1 this is the dyadic window sum of or_xsvs_contrast), then
 * multiplied by `scale` (one rounding; 1 leaves the sum as it is).  With
 * scale = 1/S over S sub-pixel wavevectors stored as S blocks of a frame's
 * pixels, J is the pixel's mean intensity: the integral over the pixel's
 * small range of q that Sec. 3.1 notes a detector pixel needs.
 * I: [n_frames][n_q]; J: [n_out][n_q].
 */
int or_frame_sums(const double *I, int64_t n_frames, int64_t n_q, int64_t n_out, int64_t s_out,
                  int64_t n_sum, int64_t s_sum, double scale, double *J, int n_threads)
{
    if (n_frames <= 0 || n_q < 0 || n_out <= 0 || n_sum <= 0 || s_out < 0 || s_sum < 0 || !J ||
        (n_out - 1) * s_out + (n_sum - 1) * s_sum >= n_frames || (n_q > 0 && !I))
        return OR_EINVAL;
    const int nth = or_threads(n_threads);
    double *bufs = malloc(sizeof(double) * (size_t)n_sum * (size_t)nth);
    if (!bufs) return OR_ENOMEM;
#pragma omp parallel for schedule(static) num_threads(nth)
    for (int64_t p = 0; p < n_q; ++p) {
        double *buf = bufs + (size_t)omp_thread_index() * (size_t)n_sum;
        for (int64_t k = 0; k < n_out; ++k) {
            for (int64_t i = 0; i < n_sum; ++i) buf[i] = I[(k * s_out + i * s_sum) * n_q + p];
            J[k * n_q + p] = or_pairwise(buf, n_sum) * scale;
        }
    }
    free(bufs);
    return OR_OK;
}

/*
 * Distribution of the normalized intensity kappa = I / <I>_ring per frame and
 * ring (Sec. 4.5, Eq. (Erlang): for M superposed configurations kappa follows
 * the Erlang distribution of order M):
 *   <I>_ring = (pairwise sum over the ring's pixels, ascending index) / n,
 *   u = (I / <I>_ring) * (n_bins / kappa_max)   (the factor rounded once),
 *   bin = u < n_bins ? max(0, floor(u)) : n_bins   (n_bins: the overflow bin,
 *         also taken by NaN).
 * counts: [n_frames][n_rings][n_bins + 1]; mean (may be NULL):
 * [n_frames][n_rings], NaN for an empty ring.
 */
int or_ring_histogram(const double *I, int64_t n_frames, int64_t n_q, const double *q, const double *edges,
                      int32_t n_rings, int32_t n_bins, double kappa_max, int64_t *counts, double *mean)
{
    if (n_frames <= 0 || n_q < 0 || n_rings <= 0 || n_bins <= 0 || !(kappa_max > 0.0) || !counts)
        return OR_EINVAL;
    int32_t *ring = malloc(sizeof(int32_t) * (size_t)(n_q > 0 ? n_q : 1));
    double *buf = malloc(sizeof(double) * (size_t)(n_q > 0 ? n_q : 1));
    if (!ring || !buf) { free(ring); free(buf); return OR_ENOMEM; }
    int rc = or_ring_index(n_q, q, n_rings, edges, ring);
    if (rc != OR_OK) { free(ring); free(buf); return rc; }
    int64_t *start = NULL, *list = NULL;
    rc = or_ring_lists(n_q, ring, NULL, n_rings, &start, &list);
    if (rc != OR_OK) { free(ring); free(buf); return rc; }
    const double scale = (double)n_bins / kappa_max;
    memset(counts, 0, sizeof(int64_t) * (size_t)n_frames * (size_t)n_rings * (size_t)(n_bins + 1));
    for (int64_t t = 0; t < n_frames; ++t)
        for (int32_t r = 0; r < n_rings; ++r) {
            const int64_t n = start[r + 1] - start[r];
            double m = NAN;
            if (n > 0) {
                for (int64_t i = 0; i < n; ++i) buf[i] = I[t * n_q + list[start[r] + i]];
                m = or_pairwise(buf, n) / (double)n;
            }
            if (mean) mean[t * n_rings + r] = m;
            int64_t *c = counts + (t * n_rings + r) * (int64_t)(n_bins + 1);
            for (int64_t i = 0; i < n; ++i) {
                const double u = (I[t * n_q + list[start[r] + i]] / m) * scale;
                int64_t b = n_bins;
                if (u < (double)n_bins) b = u > 0.0 ? (int64_t)floor(u) : 0;
                c[b]++;
            }
        }
    free(ring); free(buf); free(start); free(list);
    return OR_OK;
}

/*
 * Speckle-matching loss of the differentiation workload (fitting positions to a
 * target speckle pattern I_t through Eqs. (pe_ri), (Iq_pq)):
 *     L       = sum_p (I_p - It_p)^2 / S,   S = sum_p It_p^2,
 *     dL/dI_p = 2 (I_p - It_p) / S.
 * Both sums are long-double compensated sums over p in order (accurate to
 * about one double rounding), so this is the definition evaluated as exactly
 * as a double result allows, not a particular summation order.  d = I - It is
 * one double subtraction, as the definition reads; dL/dI_p is (2 d) / S with
 * S rounded once to double.  out: (L, S).  dL_dI may be NULL.  S = 0 gives
 * L = NaN (0/0) or Inf, as the formula does.
 */
int or_speckle_loss(int64_t n, const double *I, const double *It, double *out, double *dL_dI)
{
    if (n < 0 || !out || (n > 0 && (!I || !It))) return OR_EINVAL;
    long double a = 0.0L, ac = 0.0L, b = 0.0L, bc = 0.0L;
    for (int64_t p = 0; p < n; ++p) {
        long double d = (long double)(I[p] - It[p]);
        or_nsum(&a, &ac, d * d);
        or_nsum(&b, &bc, (long double)It[p] * (long double)It[p]);
    }
    double S = (double)(b + bc);
    out[0] = (double)((a + ac) / (b + bc));
    out[1] = S;
    if (dL_dI)
        for (int64_t p = 0; p < n; ++p) dL_dI[p] = (2.0 * (I[p] - It[p])) / S;
    return OR_OK;
}

/*
 * Gradient-descent update of the positions, r <- r - alpha g, each component
 * rounded once: r = fma(-alpha, g, r).  n values, in place.
 */
int or_position_step(int64_t n, double *pos, const double *g, double alpha)
{
    if (n < 0 || (n > 0 && (!pos || !g))) return OR_EINVAL;
    for (int64_t i = 0; i < n; ++i) pos[i] = fma(-alpha, g[i], pos[i]);
    return OR_OK;
}

/*
 * Central finite differences of the speckle-matching loss itself (not of a
 * linearisation), for selected atoms:
 *     dL/dr_{j,c} ~ (L(r + h e_{jc}) - L(r - h e_{jc})) / (2h),
 * L as in or_speckle_loss with the target fixed.  One displaced atom changes
 * the amplitude by a rank-one term (as in or_fd_grad), and
 *     L+ - L- = sum_p (I+_p - I-_p)(I+_p + I-_p - 2 It_p) / S,
 * so the difference is formed term by term in long double (compensated), with
 * no cancellation of two O(1) losses.  Sines and cosines from the C library.
 * out: [n_sel][3].
 */
int or_fd_loss_grad(int64_t n_atoms, const double *pos, const double *f,
                    int64_t n_q, const double *q, const double *It,
                    int64_t n_sel, const int64_t *atoms, double h, double *out,
                    int n_threads)
{
    if (n_atoms <= 0 || n_q < 0 || n_sel < 0 || !(h > 0.0)) return OR_EINVAL;
    for (int64_t s = 0; s < n_sel; ++s)
        if (atoms[s] < 0 || atoms[s] >= n_atoms) return OR_EINVAL;
    long double *ar = malloc(sizeof(long double) * (size_t)(n_q > 0 ? n_q : 1));
    long double *ai = malloc(sizeof(long double) * (size_t)(n_q > 0 ? n_q : 1));
    if (!ar || !ai) { free(ar); free(ai); return OR_ENOMEM; }
    long double S = 0.0L, Sc = 0.0L;
    for (int64_t p = 0; p < n_q; ++p) or_nsum(&S, &Sc, (long double)It[p] * (long double)It[p]);
    S += Sc;
#pragma omp parallel for schedule(static) num_threads(or_threads(n_threads))
    for (int64_t p = 0; p < n_q; ++p) {
        long double sr = 0.0L, si = 0.0L;
        for (int64_t j = 0; j < n_atoms; ++j) {
            long double ph = (long double)q[3 * p] * pos[3 * j] +
                             (long double)q[3 * p + 1] * pos[3 * j + 1] +
                             (long double)q[3 * p + 2] * pos[3 * j + 2];
            sr += f[j] * cosl(ph);
            si -= f[j] * sinl(ph);
        }
        ar[p] = sr; ai[p] = si;
    }
    for (int64_t s = 0; s < n_sel; ++s) {
        int64_t j = atoms[s];
        for (int c = 0; c < 3; ++c) {
            long double sum = 0.0L, comp = 0.0L;
#pragma omp parallel num_threads(or_threads(n_threads))
            {
                long double lsum = 0.0L, lcomp = 0.0L;
#pragma omp for schedule(static)
                for (int64_t p = 0; p < n_q; ++p) {
                    long double ph0 = (long double)q[3 * p] * pos[3 * j] +
                                      (long double)q[3 * p + 1] * pos[3 * j + 1] +
                                      (long double)q[3 * p + 2] * pos[3 * j + 2];
                    long double dph = (long double)q[3 * p + c] * h;
                    long double br = ar[p] - f[j] * cosl(ph0);
                    long double bi = ai[p] + f[j] * sinl(ph0);
                    long double pr = br + f[j] * cosl(ph0 + dph), pi = bi - f[j] * sinl(ph0 + dph);
                    long double mr = br + f[j] * cosl(ph0 - dph), mi = bi - f[j] * sinl(ph0 - dph);
                    long double Ip = pr * pr + pi * pi, Im = mr * mr + mi * mi;
                    or_nsum(&lsum, &lcomp, (Ip - Im) * (Ip + Im - 2.0L * It[p]));
                }
#pragma omp critical
                {
                    or_nsum(&sum, &comp, lsum);
                    or_nsum(&sum, &comp, lcomp);
                }
            }
            out[3 * s + c] = (double)((sum + comp) / (S * 2.0L * h));
        }
    }
    free(ar); free(ai);
    return OR_OK;
}
