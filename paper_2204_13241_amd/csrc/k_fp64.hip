// Exact FP64 form of the direct method (Sec. 3.1, Algorithm 1; Eqs. (pe_ri),
// (Iq_pq)) and of its position gradient.
//
// The operation sequence is fixed so that the result is reproducible bit for
// bit on any IEEE-754 binary64 machine with fused multiply-add:
//   phase in revolutions  t = q_rev . r,  q_rev = q * RN(1/(2 pi))   (fma chain z,y,x)
//   n = rint(t), u = t - n, m = rint(4u), v = u - m/4    (all exact)
//   x = 2 pi v with a two-term 2 pi, z = x^2
//   sin x, cos x by the Taylor series to x^15 / x^16 (Horner, fma)
//   quarter-turn rotation by m mod 4
//   amplitude sums in input order from +0.0, I = a*a + b*b (fma).
// Built with contraction off: every fused multiply-add here is explicit.
#include <hip/hip_runtime.h>

#include "xs_internal.h"

namespace xs {
namespace {

// RN(1/(2 pi)), RN(2 pi) and RN(2 pi - RN(2 pi)).
constexpr double kInvTwoPi = 0x1.45f306dc9c883p-3;
constexpr double kTwoPiHi = 0x1.921fb54442d18p+2;
constexpr double kTwoPiLo = 0x1.1a62633145c07p-52;

// sin(2 pi t), cos(2 pi t) for t in revolutions.
__device__ __forceinline__ void sincos_turns(double t, double &sn, double &cs) {
    const double n = __builtin_rint(t);
    const double u = t - n;
    const double m = __builtin_rint(4.0 * u);
    const double v = u - m * 0.25;
    const double x = __builtin_fma(kTwoPiHi, v, kTwoPiLo * v);
    const double z = x * x;
    // Taylor coefficients (-1)^k / (2k+1)!  and  (-1)^k / (2k)!, rounded once.
    double ps = __builtin_fma(z, -1.0 / 1307674368000.0, 1.0 / 6227020800.0);
    ps = __builtin_fma(z, ps, -1.0 / 39916800.0);
    ps = __builtin_fma(z, ps, 1.0 / 362880.0);
    ps = __builtin_fma(z, ps, -1.0 / 5040.0);
    ps = __builtin_fma(z, ps, 1.0 / 120.0);
    ps = __builtin_fma(z, ps, -1.0 / 6.0);
    const double s = __builtin_fma(x * z, ps, x);
    double pc = __builtin_fma(z, 1.0 / 20922789888000.0, -1.0 / 87178291200.0);
    pc = __builtin_fma(z, pc, 1.0 / 479001600.0);
    pc = __builtin_fma(z, pc, -1.0 / 3628800.0);
    pc = __builtin_fma(z, pc, 1.0 / 40320.0);
    pc = __builtin_fma(z, pc, -1.0 / 720.0);
    pc = __builtin_fma(z, pc, 1.0 / 24.0);
    pc = __builtin_fma(z, pc, -0.5);
    const double c = __builtin_fma(z, pc, 1.0);
    // Quarter turns: m = 0: (s, c); 1: (c, -s); 2: (-s, -c); 3: (-c, s).
    const int quarter = static_cast<int>(m) & 3;
    const double s_sel = (quarter & 1) ? c : s;
    const double c_sel = (quarter & 1) ? s : c;
    sn = (quarter & 2) ? -s_sel : s_sel;
    cs = ((quarter + 1) & 2) ? -c_sel : c_sel;
}

__device__ __forceinline__ double phase_turns(double qx, double qy, double qz, double x,
                                              double y, double z) {
    return __builtin_fma(qz, z, __builtin_fma(qy, y, qx * x));
}

constexpr int kBlock = 256;
constexpr int kAtomStage = 256;   // atoms staged in LDS per pass of the forward
constexpr int kPixStage = 256;    // pixels staged in LDS per pass of the gradient

// One thread per pixel; the segment's atoms are staged in LDS in chunks, in
// input order (x, y, z, f), and every thread reads them as broadcasts.  Four
// pairs per unrolled step give independent sine/cosine chains; the sums still
// take the atoms one by one in order.  grid = (pixel blocks, segments).
__global__ __launch_bounds__(kBlock) void k_forward_fp64(const Segment *__restrict__ segs,
                                                         const double *__restrict__ pos,
                                                         const double *__restrict__ f,
                                                         const double *__restrict__ q,
                                                         double *__restrict__ I,
                                                         double *__restrict__ amp) {
    __shared__ double4 s_atom[kAtomStage];
    const Segment sg = segs[blockIdx.y];
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (blockIdx.x * kBlock >= sg.n_q) return;  // whole block past this segment's pixels
    const bool active = p < sg.n_q;
    const int pc = active ? p : sg.n_q - 1;
    const double *qp = q + (sg.q + pc) * 3;
    const double qx = qp[0] * kInvTwoPi, qy = qp[1] * kInvTwoPi, qz = qp[2] * kInvTwoPi;
    const double *r = pos + sg.pos * 3;
    const double *ff = f + sg.f;
    double ac = 0.0, as = 0.0;
    for (int j0 = 0; j0 < sg.n_atoms; j0 += kAtomStage) {
        const int nj = min(kAtomStage, sg.n_atoms - j0);
        __syncthreads();  // the previous chunk has been read by every thread
        for (int t = threadIdx.x; t < nj; t += kBlock) {
            const int64_t j = j0 + t;
            s_atom[t] = make_double4(r[3 * j], r[3 * j + 1], r[3 * j + 2], ff[j]);
        }
        __syncthreads();
#pragma unroll 4
        for (int t = 0; t < nj; ++t) {
            const double4 at = s_atom[t];
            double sn, cs;
            sincos_turns(phase_turns(qx, qy, qz, at.x, at.y, at.z), sn, cs);
            ac = __builtin_fma(at.w, cs, ac);
            as = __builtin_fma(at.w, sn, as);
        }
    }
    if (!active) return;
    const double a = ac, b = -as;
    const int64_t o = sg.out + p;
    I[o] = __builtin_fma(a, a, b * b);
    if (amp) {
        amp[2 * o] = a;
        amp[2 * o + 1] = b;
    }
}

// One thread per atom; the segment's pixels are staged in LDS in chunks, in
// input order: q / (2 pi) (the phase operand, the same product the per-pair
// form would round), q, the amplitude (a, b) and the weight w.
//   h = fma(a, s, b*c), k = w*h, g += k*q (fma per component), dL/dr = (-2 f) g.
struct PixFp64 {
    double2 qr01, qr2w, q01, q2, ab;
};

__global__ __launch_bounds__(kBlock) void k_grad_fp64(const Segment *__restrict__ segs,
                                                      const double *__restrict__ pos,
                                                      const double *__restrict__ f,
                                                      const double *__restrict__ q,
                                                      const double *__restrict__ amp,
                                                      const double *__restrict__ w,
                                                      float *__restrict__ g32,
                                                      double *__restrict__ g64) {
    __shared__ PixFp64 s_pix[kPixStage];
    const Segment sg = segs[blockIdx.y];
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (blockIdx.x * kBlock >= sg.n_atoms) return;
    const bool active = j < sg.n_atoms;
    const int jc = active ? j : sg.n_atoms - 1;
    const double *rj = pos + (sg.pos + jc) * 3;
    const double x = rj[0], y = rj[1], z = rj[2];
    const double *qq = q + sg.q * 3;
    const double *aa = amp + sg.out * 2;
    const double *ww = w + sg.out;
    double gx = 0.0, gy = 0.0, gz = 0.0;
    for (int p0 = 0; p0 < sg.n_q; p0 += kPixStage) {
        const int np = min(kPixStage, sg.n_q - p0);
        __syncthreads();  // the previous chunk has been read by every thread
        for (int t = threadIdx.x; t < np; t += kBlock) {
            const int64_t p = p0 + t;
            const double q0 = qq[3 * p], q1 = qq[3 * p + 1], q2 = qq[3 * p + 2];
            PixFp64 v;
            v.qr01 = make_double2(q0 * kInvTwoPi, q1 * kInvTwoPi);
            v.qr2w = make_double2(q2 * kInvTwoPi, ww[p]);
            v.q01 = make_double2(q0, q1);
            v.q2 = make_double2(q2, 0.0);
            v.ab = make_double2(aa[2 * p], aa[2 * p + 1]);
            s_pix[t] = v;
        }
        __syncthreads();
#pragma unroll 4
        for (int t = 0; t < np; ++t) {
            const double2 qr01 = s_pix[t].qr01, qr2w = s_pix[t].qr2w, q01 = s_pix[t].q01, ab = s_pix[t].ab;
            const double q2 = s_pix[t].q2.x;
            double sn, cs;
            sincos_turns(phase_turns(qr01.x, qr01.y, qr2w.x, x, y, z), sn, cs);
            const double h = __builtin_fma(ab.x, sn, ab.y * cs);
            const double k = qr2w.y * h;
            gx = __builtin_fma(k, q01.x, gx);
            gy = __builtin_fma(k, q01.y, gy);
            gz = __builtin_fma(k, q2, gz);
        }
    }
    if (!active) return;
    const double m = -2.0 * f[sg.f + j];
    const int64_t o = (sg.pos + j) * 3;
    const double r0 = m * gx, r1 = m * gy, r2 = m * gz;
    if (g64) {
        g64[o] = r0;
        g64[o + 1] = r1;
        g64[o + 2] = r2;
    }
    if (g32) {
        g32[o] = static_cast<float>(r0);
        g32[o + 1] = static_cast<float>(r1);
        g32[o + 2] = static_cast<float>(r2);
    }
}

}  // namespace

xs_status fp64_forward(hipStream_t s, const Segment *segs_host, int n_segs, int max_q,
                       const double *pos, const double *f, const double *q, double *I,
                       double *amp) {
    if (n_segs <= 0 || max_q <= 0) return XS_OK;
    void *d_segs = nullptr;
    XS_TRY(upload(s, SLOT_SEGS, segs_host, sizeof(Segment) * n_segs, &d_segs));
    dim3 grid((max_q + kBlock - 1) / kBlock, n_segs);
    double work = 0.0;
    for (int i = 0; i < n_segs; ++i) work += static_cast<double>(segs_host[i].n_atoms) * segs_host[i].n_q;
    TimerScope tm(s, TIMER_FWD64);
    hipLaunchKernelGGL(k_forward_fp64, grid, dim3(kBlock), 0, s,
                       static_cast<const Segment *>(d_segs), pos, f, q, I, amp);
    tm.end(work);
    XS_HIP(hipGetLastError());
    return XS_OK;
}

xs_status fp64_grad(hipStream_t s, const Segment *segs_host, int n_segs, int max_atoms,
                    const double *pos, const double *f, const double *q, const double *amp,
                    const double *dL_dI, float *dL_dr, double *dL_dr64) {
    if (n_segs <= 0 || max_atoms <= 0) return XS_OK;
    void *d_segs = nullptr;
    XS_TRY(upload(s, SLOT_SEGS, segs_host, sizeof(Segment) * n_segs, &d_segs));
    dim3 grid((max_atoms + kBlock - 1) / kBlock, n_segs);
    double work = 0.0;
    for (int i = 0; i < n_segs; ++i) work += static_cast<double>(segs_host[i].n_atoms) * segs_host[i].n_q;
    TimerScope tm(s, TIMER_GRAD64);
    hipLaunchKernelGGL(k_grad_fp64, grid, dim3(kBlock), 0, s,
                       static_cast<const Segment *>(d_segs), pos, f, q, amp, dL_dI, dL_dr,
                       dL_dr64);
    tm.end(work);
    XS_HIP(hipGetLastError());
    return XS_OK;
}

}  // namespace xs
