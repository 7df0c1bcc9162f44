// FFT-based method of Sec. 3.2 (Algorithm 2): the comparison baseline of the
// direct method.  One frame per call, in FP64:
//   1. rho = 0 on an n x n x n grid over the periodic box [0, L)^3 (spacing
//      delta = L / n, grid point m at m delta);
//   2. every atom adds f_i (1 / (sqrt(2 pi) eta))^3 exp(-|x_m - r_i|^2 / (2 eta^2))
//      to the k grid points nearest to it along each axis (indices modulo n),
//      Eq. (modified_r) weighted by the atom's form factor;
//   3. P = D2Z FFT of rho (hipFFT), P[h] = sum_m rho[m] exp(-2 pi i h.m / n), so
//      that delta^3 P[h] is the transform of Eq. (pq_rq_app_alt) at q_h = 2 pi h / L;
//   4. G = the same transform of one Gaussian centred at the origin (k^3 points),
//      the discrete f^eta of the method (cached per stream while n, eta, k and L
//      stay the same);
//   5. I(q_h) = |P[h]|^2 / |G[h]|^2 (Eq. (Iq_pq_new); delta^3 cancels), and the
//      amplitude p^e = P / G when asked.
// The spreading adds with FP64 atomics, so the order of the additions into one
// grid point (and the last bits of rho) varies from run to run.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <cmath>
#include <map>
#include <mutex>

#include "xs_internal.h"

namespace xs {
namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void k_fft_zero(double *__restrict__ p, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kBlock)
        p[i] = 0.0;
}

// One thread per (atom, first-axis point, second-axis point); it walks the k points
// of the third axis.  Grid points in row-major order [m_x][m_y][m_z].
__global__ __launch_bounds__(kBlock) void k_fft_spread(const double *__restrict__ pos, const double *__restrict__ f,
                                                       int64_t n_atoms, int32_t n, double delta, double eta,
                                                       int32_t k, double *__restrict__ rho) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t kk = static_cast<int64_t>(k) * k;
    if (t >= n_atoms * kk) return;
    const int64_t i = t / kk;
    const int a = static_cast<int>((t - i * kk) / k), b = static_cast<int>(t - i * kk - static_cast<int64_t>(a) * k);
    const double rx = pos ? pos[3 * i] : 0.0, ry = pos ? pos[3 * i + 1] : 0.0, rz = pos ? pos[3 * i + 2] : 0.0;
    const double w = f ? f[i] : 1.0;
    const double inv2e2 = 1.0 / (2.0 * eta * eta);
    const double s2pe = 1.0 / (sqrt(2.0 * M_PI) * eta);
    const double norm = s2pe * s2pe * s2pe;
    // first of the k grid indices nearest to each coordinate: ceil(x / delta - k / 2)
    const int64_t mx = static_cast<int64_t>(ceil(rx / delta - 0.5 * k)) + a;
    const int64_t my = static_cast<int64_t>(ceil(ry / delta - 0.5 * k)) + b;
    const int64_t mz0 = static_cast<int64_t>(ceil(rz / delta - 0.5 * k));
    const double dx = static_cast<double>(mx) * delta - rx, dy = static_cast<double>(my) * delta - ry;
    const double gxy = w * norm * exp(-dx * dx * inv2e2) * exp(-dy * dy * inv2e2);
    const int64_t ix = ((mx % n) + n) % n, iy = ((my % n) + n) % n;
    double *row = rho + (ix * n + iy) * n;
    for (int c = 0; c < k; ++c) {
        const int64_t mz = mz0 + c;
        const double dz = static_cast<double>(mz) * delta - rz;
        atomicAdd(row + ((mz % n) + n) % n, gxy * exp(-dz * dz * inv2e2));
    }
}

// |G|^2 of the half spectrum (n x n x (n/2 + 1)), read back for the full grid by symmetry.
__global__ __launch_bounds__(kBlock) void k_fft_gauss_abs2(const double2 *__restrict__ G, int64_t n_half,
                                                           double *__restrict__ g2) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n_half) return;
    const double2 v = G[i];
    g2[i] = v.x * v.x + v.y * v.y;
}

// Full-grid intensity (and amplitude) from the half spectrum of the D2Z transform:
// index (hx, hy, hz) with hz > n/2 reads the conjugate at (-hx, -hy, -hz) mod n.
__global__ __launch_bounds__(kBlock) void k_fft_intensity(const double2 *__restrict__ P, const double2 *__restrict__ G,
                                                          const double *__restrict__ g2, int32_t n,
                                                          double *__restrict__ I, double2 *__restrict__ amp) {
    const int64_t nn = static_cast<int64_t>(n) * n * n;
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (t >= nn) return;
    const int64_t hz = t % n, hy = (t / n) % n, hx = t / (static_cast<int64_t>(n) * n);
    const int64_t nh = n / 2 + 1;
    int64_t j;
    bool conj = false;
    if (hz < nh) {
        j = (hx * n + hy) * nh + hz;
    } else {
        j = (((n - hx) % n) * n + (n - hy) % n) * nh + (n - hz);
        conj = true;
    }
    double2 p = P[j];
    const double gg = g2[j];
    I[t] = (p.x * p.x + p.y * p.y) / gg;
    if (amp) {
        double2 g = G[j];
        if (conj) {
            p.y = -p.y;
            g.y = -g.y;
        }
        // p / g = p conj(g) / |g|^2
        amp[t] = make_double2((p.x * g.x + p.y * g.y) / gg, (p.y * g.x - p.x * g.y) / gg);
    }
}

unsigned blocks_for(int64_t n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }

struct FftState {
    hipfftHandle plan = 0;
    int n = 0;
    // what the Gaussian slots hold
    int g_n = 0, g_k = 0;
    double g_eta = 0.0, g_delta = 0.0;
    const void *g_ptr = nullptr, *g2_ptr = nullptr;
};
std::mutex g_fft_mu;
std::map<std::pair<int, hipStream_t>, FftState> g_fft;

const char *fft_err(hipfftResult r) {
    switch (r) {
    case HIPFFT_ALLOC_FAILED: return "allocation failed";
    case HIPFFT_INVALID_VALUE: return "invalid value";
    case HIPFFT_EXEC_FAILED: return "execution failed";
    case HIPFFT_SETUP_FAILED: return "setup failed";
    case HIPFFT_INVALID_SIZE: return "invalid size";
    default: return "error";
    }
}

}  // namespace

xs_status fft_intensity(hipStream_t s, const double *pos, const double *f, int64_t n_atoms, double box,
                        int32_t n, double eta, int32_t k, double *I, double *amp) {
    const double delta = box / n;
    const int64_t nn = static_cast<int64_t>(n) * n * n;
    // one spreading thread per (atom, first-axis point, second-axis point) in one grid
    if (n_atoms > (static_cast<int64_t>(0x7fffffff) * kBlock) / (static_cast<int64_t>(k) * k))
        return set_error(XS_EINVAL, "%lld atoms x k^2 = %d^2 spreading threads exceed one launch",
                         static_cast<long long>(n_atoms), k);
    const int64_t nhalf = static_cast<int64_t>(n) * n * (n / 2 + 1);
    void *rho = nullptr, *spec = nullptr, *gspec = nullptr, *g2 = nullptr;
    XS_TRY(scratch(s, SLOT_FFT_RHO, sizeof(double) * nn, &rho));
    XS_TRY(scratch(s, SLOT_FFT_SPEC, sizeof(double2) * nhalf, &spec));
    XS_TRY(scratch(s, SLOT_FFT_GAUSS, sizeof(double2) * nhalf, &gspec));
    XS_TRY(scratch(s, SLOT_FFT_GAUSS2, sizeof(double) * nhalf, &g2));
    int dev = 0;
    XS_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_fft_mu);
    FftState &st = g_fft[std::make_pair(dev, s)];
    if (st.plan && st.n != n) {
        (void)hipfftDestroy(st.plan);
        st.plan = 0;
    }
    if (!st.plan) {
        const hipfftResult r = hipfftPlan3d(&st.plan, n, n, n, HIPFFT_D2Z);
        if (r != HIPFFT_SUCCESS) {
            st.plan = 0;
            return set_error(r == HIPFFT_ALLOC_FAILED ? XS_ENOMEM : XS_EDEVICE, "hipfftPlan3d(%d): %s", n, fft_err(r));
        }
        st.n = n;
    }
    if (hipfftSetStream(st.plan, s) != HIPFFT_SUCCESS) return set_error(XS_EDEVICE, "hipfftSetStream failed");
    const unsigned zb = std::min<unsigned>(blocks_for(nn), 65536u);
    // the discrete f^eta: transform of the centred Gaussian, unless the slots hold it already
    if (!(st.g_n == n && st.g_k == k && st.g_eta == eta && st.g_delta == delta && st.g_ptr == gspec &&
          st.g2_ptr == g2)) {
        hipLaunchKernelGGL(k_fft_zero, dim3(zb), dim3(kBlock), 0, s, static_cast<double *>(rho), nn);
        hipLaunchKernelGGL(k_fft_spread, dim3(blocks_for(static_cast<int64_t>(k) * k)), dim3(kBlock), 0, s,
                           static_cast<const double *>(nullptr), static_cast<const double *>(nullptr),
                           int64_t(1), n, delta, eta, k, static_cast<double *>(rho));
        XS_HIP(hipGetLastError());
        const hipfftResult r = hipfftExecD2Z(st.plan, static_cast<hipfftDoubleReal *>(rho),
                                             static_cast<hipfftDoubleComplex *>(gspec));
        if (r != HIPFFT_SUCCESS) return set_error(XS_EDEVICE, "hipfftExecD2Z (Gaussian): %s", fft_err(r));
        hipLaunchKernelGGL(k_fft_gauss_abs2, dim3(blocks_for(nhalf)), dim3(kBlock), 0, s,
                           static_cast<const double2 *>(gspec), nhalf, static_cast<double *>(g2));
        XS_HIP(hipGetLastError());
        st.g_n = n;
        st.g_k = k;
        st.g_eta = eta;
        st.g_delta = delta;
        st.g_ptr = gspec;
        st.g2_ptr = g2;
    }
    hipLaunchKernelGGL(k_fft_zero, dim3(zb), dim3(kBlock), 0, s, static_cast<double *>(rho), nn);
    if (n_atoms > 0)
        hipLaunchKernelGGL(k_fft_spread, dim3(blocks_for(n_atoms * k * k)), dim3(kBlock), 0, s, pos, f, n_atoms, n,
                           delta, eta, k, static_cast<double *>(rho));
    XS_HIP(hipGetLastError());
    const hipfftResult r = hipfftExecD2Z(st.plan, static_cast<hipfftDoubleReal *>(rho),
                                         static_cast<hipfftDoubleComplex *>(spec));
    if (r != HIPFFT_SUCCESS) return set_error(XS_EDEVICE, "hipfftExecD2Z: %s", fft_err(r));
    hipLaunchKernelGGL(k_fft_intensity, dim3(blocks_for(nn)), dim3(kBlock), 0, s, static_cast<const double2 *>(spec),
                       static_cast<const double2 *>(gspec), static_cast<const double *>(g2), n, I,
                       reinterpret_cast<double2 *>(amp));
    XS_HIP(hipGetLastError());
    return XS_OK;
}

void release_fft_plans() {
    std::lock_guard<std::mutex> lk(g_fft_mu);
    for (auto &kv : g_fft)
        if (kv.second.plan) (void)hipfftDestroy(kv.second.plan);
    g_fft.clear();
}

}  // namespace xs
