// lbm_structures.hip -- coherent-structure identification on the GPU
// (arXiv:2405.12082, Section II.C): the streamwise velocity on the circle
// r = r0, the Fourier transform of its azimuthal correlation
// R_uu(r0, dtheta) = < u_z(theta0) u_z(theta0 + dtheta) >_theta0 / u_rms^2 per
// cross-section, the plane average, and the dominant azimuthal mode.
//
// By the Wiener-Khinchin relation the transform of the circular correlation
// of one plane is |U(m)|^2 / sum_j du_j^2, U the DFT of the fluctuation du
// (about the ring mean), so a plane costs one DFT of its N ring samples.
#include <mutex>

#include "../../include/lbm.h"
#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

// One block per (pipe, plane): u_z = j_z / rho + a_z / 2 (Eq.
// (macroscopic_u), as lbm_moments reports it) at each distinct node the
// ring touches, gathered from the state like the step does, into LDS; then
// every ring point by bilinear interpolation of its four nodes (FP64).
constexpr int kRingNodes = 16384;  // 4 x the largest ring
template <typename T, int FORM, bool WALL>
__global__ __launch_bounds__(256) void k_ring(const Geom g, const RingArgs r, const T *__restrict__ state, float *ring)
{
    __shared__ float uz[kRingNodes];
    const int z = blockIdx.x % g.nz, b = blockIdx.x / g.nz;
    using R = typename RealOf<T>::type;
    const R sig = sigma_of<R>(g, *g.step_dev);
    const unsigned rowb = (unsigned)g.P * sizeof(T);
    const unsigned zo = (unsigned)z * rowb, zmo = (unsigned)wrap_m(z, g.nz) * rowb, zpo = (unsigned)wrap_p(z, g.nz) * rowb;
    __shared__ float lref[href_lds_floats<T, 256>()];
    for (int u = threadIdx.x; u < r.n_nodes; u += 256) {
        const int col = r.nodes[u];
        const Pull<T, WALL> p = make_pull<T, WALL>(state + (size_t)b * g.pipe, (size_t)g.pstride, g.nbr, g.P, col,
                                                   g.bcoef, g.href, lref + 27 * threadIdx.x, g.check);
        R v[27];
        gather<T, FORM, WALL>(p, zo, zmo, zpo, v);
        R ax, ay, az;
        const Shape<R> sh = shape_of<R>(g, b, col);
        body_force<R>(g, z, sig, sh.px, sh.py, sh.pq, ax, ay, az);
        const Moments<R> m = moments_of<R>(v);
        uz[u] = (float)(m.jz * rcp_r(R(1) + m.dr) + R(0.5) * az);
    }
    __syncthreads();
    float *out = ring + ((size_t)b * g.nz + z) * r.ntheta;
    for (int j = threadIdx.x; j < r.ntheta; j += 256) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) acc += r.w[j * 4 + q] * (double)uz[r.idx[j * 4 + q]];
        out[j] = (float)acc;
    }
}

// One block per (pipe, plane): fluctuation about the ring mean, then the
// normalised power |U(m)|^2 / sum du^2 for m = 1..mmax (m = 0 is 0), FP64,
// twiddles exp(-2 pi i q / N) from a table.
__global__ __launch_bounds__(256) void k_ring_spectrum(const float *__restrict__ ring, int n, int mmax,
                                                       const double *__restrict__ tw, double *__restrict__ spec)
{
    __shared__ double u[4096];
    __shared__ double red[256];
    const int plane = blockIdx.x;
    const float *rz = ring + (size_t)plane * n;
    double s = 0.0;
    for (int j = threadIdx.x; j < n; j += 256) {
        u[j] = (double)rz[j];
        s += u[j];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double mean = red[0] / n;
    __syncthreads();
    double e = 0.0;
    for (int j = threadIdx.x; j < n; j += 256) {
        u[j] -= mean;
        e += u[j] * u[j];
    }
    red[threadIdx.x] = e;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double energy = red[0];
    double *out = spec + (size_t)plane * (mmax + 1);
    if (threadIdx.x == 0) out[0] = 0.0;
    for (int m = 1 + threadIdx.x; m <= mmax; m += 256) {
        double re = 0.0, im = 0.0;
        int q = 0;  // (m j) mod n
        for (int j = 0; j < n; ++j) {
            re += u[j] * tw[2 * q];
            im += u[j] * tw[2 * q + 1];
            q += m;
            if (q >= n) q -= n;
        }
        out[m] = energy > 0.0 ? (re * re + im * im) / energy : 0.0;
    }
}

// One block per pipe: plane average of the spectra (a fixed-order tree over
// the planes) and the dominant mode, the highest peak among m >= 1 (first on
// ties; 0 when the spectrum vanishes).
__global__ __launch_bounds__(256) void k_spectrum_mean(const double *__restrict__ spec, int nz, int mmax,
                                                       double *__restrict__ mean, int *__restrict__ dominant)
{
    __shared__ double red[256];
    const int b = blockIdx.x;
    double *mb = mean + (size_t)b * (mmax + 1);
    for (int m = 0; m <= mmax; ++m) {
        double s = 0.0;
        for (int z = threadIdx.x; z < nz; z += 256) s += spec[((size_t)b * nz + z) * (mmax + 1) + m];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) mb[m] = red[0] / nz;
        __syncthreads();
    }
    if (threadIdx.x == 0 && dominant) {
        int best = 0;
        double top = 0.0;
        for (int m = 1; m <= mmax; ++m) {
            const double p = mb[m] * mb[m];
            if (p > top) {
                top = p;
                best = m;
            }
        }
        dominant[b] = best;
    }
}

template <typename T, int FORM, bool WALL>
static void ring_t(const Geom &g, const RingArgs &r, const void *state, float *ring, hipStream_t s)
{
    hipLaunchKernelGGL((k_ring<T, FORM, WALL>), dim3((unsigned)(g.B * g.nz)), dim3(256), 0, s, g, r, (const T *)state,
                       ring);
}
template <typename T>
static void ring_form(int form, const Geom &g, const RingArgs &r, const void *state, float *ring, hipStream_t s)
{
    if (form == FORM_N)
        ring_t<T, FORM_N, false>(g, r, state, ring, s);
    else if (form == FORM_W)
        ring_t<T, FORM_W, false>(g, r, state, ring, s);
    else if (g.bcoef)
        ring_t<T, FORM_S, true>(g, r, state, ring, s);
    else
        ring_t<T, FORM_S, false>(g, r, state, ring, s);
}

hipError_t launch_ring(int storage, int form, const Geom &g, const RingArgs &r, const void *state, float *ring,
                       hipStream_t s)
{
    if (storage == 2)
        ring_form<double>(form, g, r, state, ring, s);
    else if (storage == 1)
        ring_form<__half>(form, g, r, state, ring, s);
    else
        ring_form<float>(form, g, r, state, ring, s);
    return hipGetLastError();
}

hipError_t launch_ring_spectrum(const float *ring, int planes, int n, int mmax, const double *tw, double *spec,
                                hipStream_t s)
{
    hipLaunchKernelGGL(k_ring_spectrum, dim3(planes), dim3(256), 0, s, ring, n, mmax, tw, spec);
    return hipGetLastError();
}

hipError_t launch_spectrum_mean(const double *spec, int B, int nz, int mmax, double *mean, int *dominant,
                                hipStream_t s)
{
    hipLaunchKernelGGL(k_spectrum_mean, dim3(B), dim3(256), 0, s, spec, nz, mmax, mean, dominant);
    return hipGetLastError();
}

// ---------------------------------------------------------------- context-free spectrum
// lbm_ring_spectrum_static: the transform above without a context or
// workspace, for callers that cannot allocate device memory.  Its only
// scratch is the twiddle table, in a file-scope device array of
// kStaticRing points (64 KiB, one copy per GPU, held until the process
// ends); the host never names the array directly: hipGetSymbolAddress
// gives its address on each device once, at lbm_init or at the first call
// on that device (with that device current), and that address is what the
// kernels receive.  Every call rewrites the whole table it uses, so nothing
// has to start at zero; calls that overlap on one GPU share the table and
// race.
constexpr int kStaticRing = 4096;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[2 * kStaticRing];

// twiddles exp(-2 pi i q / n), q < n
__global__ __launch_bounds__(256) void k_twiddle(double *__restrict__ tw, int n)
{
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    double sn, cs;
    sincospi(2.0 * (double)q / (double)n, &sn, &cs);
    tw[2 * q] = cs;
    tw[2 * q + 1] = -sn;
}

static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up once per device)
hipError_t static_scratch(double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace lbm

extern "C" int lbm_ring_spectrum_static(const float *ring, int32_t batch, int32_t nz, int32_t ntheta, int32_t mmax,
                                        double *spec, double *mean, int32_t *dominant, void *stream)
{
    using namespace lbm;
    if (!ring || !spec || batch < 1 || nz < 1 || (long long)batch * nz > 0x7fffffffLL || ntheta < 4 ||
        ntheta > kStaticRing || mmax < 1 || mmax > ntheta / 2 || (dominant && !mean))
        return LBM_EINVAL;
    double *tw = nullptr;
    if (static_scratch(&tw) != hipSuccess) return LBM_EHIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_twiddle, dim3((unsigned)((ntheta + 255) / 256)), dim3(256), 0, s, tw, ntheta);
    if (hipGetLastError() != hipSuccess) return LBM_EHIP;
    if (launch_ring_spectrum(ring, batch * nz, ntheta, mmax, tw, spec, s) != hipSuccess) return LBM_EHIP;
    if (mean && launch_spectrum_mean(spec, batch, nz, mmax, mean, dominant, s) != hipSuccess) return LBM_EHIP;
    return LBM_OK;
}
