// lbm_adjoint.hip -- discrete adjoint of the fused stream-collide step.
//
// Forward step: f^{n+1} = S C(f^n, a^n).  One reverse step at cursor c:
//     mu        = S^T lambda^{c+1}                  (adjoint of the post-collision state)
//     lambda^c  = (dC/df)^T mu + dE_c/df            (E_c: streamwise energy of f^c)
//     s(x)      = (dC/da)^T mu + dE_c/da            (sensitivity to the body acceleration)
// C depends on f only through rho, j and the stress moments m_4..m_8, so the
// vector-Jacobian product is the chain rule through these 9 moments, derived
// by hand from the collision of the forward kernel (deviation form of the
// Hermite-6 equilibrium, Guo forcing, relaxation of m_4..8 with omega).
// The force sensitivities are accumulated per column in FP64 and projected
// onto the trigger-force mode shapes of Eq. (TurbForce).
#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

// mu_j(y) = lambda_j(y + c_j) if y + c_j is fluid, else lambda_opp(j)(y):
// the transpose of the pull gather with halfway bounce-back.
template <int J = 0>
__device__ __forceinline__ void gather_transpose(const float *__restrict__ lam, int pstride, int P, const int (&col)[9],
                                                 int k, int z, int zm, int zp, float (&mu)[27])
{
    constexpr int cx = CX(J), cy = CY(J), cz = CZ(J);
    constexpr int d = NSLOT(cx, cy);
    const int zs = cz == 0 ? z : (cz > 0 ? zp : zm);
    const int sc = col[d];
    if (d == 4 || sc >= 0)
        mu[J] = lam[J * pstride + zs * P + sc];
    else
        mu[J] = lam[OPP(J) * pstride + z * P + k];
    if constexpr (J + 1 < 27) gather_transpose<J + 1>(lam, pstride, P, col, k, z, zm, zp, mu);
}

__device__ __forceinline__ float hsel(int c) { return c == 0 ? -3.f : 6.f; }  // d''_c

struct PopAdj {
    float Sr, Sux, Suy, Suz, Sax, Say, Saz;
};

// population part: sum_i mu_i d/d(rho, u, a) [ (f^eq_i - w_i) + F_i/2 ]
template <int I = 0>
__device__ __forceinline__ void pop_adjoint(const CollideCtx &c, const float (&mu)[27], PopAdj &s)
{
    constexpr int cx = CX(I), cy = CY(I), cz = CZ(I);
    const float dx = dsel<cx>(c.X), dy = dsel<cy>(c.Y), dz = dsel<cz>(c.Z);
    const float qx = qsel<cx>(c.X), qy = qsel<cy>(c.Y), qz = qsel<cz>(c.Z);
    constexpr float hx = cx == 0 ? -3.f : 6.f, hy = cy == 0 ? -3.f : 6.f, hz = cz == 0 ? -3.f : 6.f;
    const float ex = 1.f + dx, ey = 1.f + dy, ez = 1.f + dz;
    const float eyz = ey * ez, exz = ex * ez, exy = ex * ey;
    const float pi = ex * eyz;
    const float px = qx * eyz, py = qy * exz, pz = qz * exy;      // d Pi / d u
    const float api = c.ax * px + c.ay * py + c.az * pz;           // F_i / (rho w)
    const float pxy = qx * qy * ez, pxz = qx * qz * ey, pyz = qy * qz * ex;
    const float dax = c.ax * hx * eyz + c.ay * pxy + c.az * pxz;   // d api / d u_x
    const float day = c.ax * pxy + c.ay * hy * exz + c.az * pyz;
    const float daz = c.ax * pxz + c.ay * pyz + c.az * hz * exy;
    const float wm = WGT(I) * mu[I];
    s.Sr += wm * (pi + 0.5f * api);
    s.Sux += wm * (px + 0.5f * dax);
    s.Suy += wm * (py + 0.5f * day);
    s.Suz += wm * (pz + 0.5f * daz);
    s.Sax += wm * px;
    s.Say += wm * py;
    s.Saz += wm * pz;
    if constexpr (I + 1 < 27) pop_adjoint<I + 1>(c, mu, s);
}

// D_k = <mu, d_k>, the columns 4..8 of the inverse moment matrix
template <int I = 0>
__device__ __forceinline__ void dual_dots(const float (&mu)[27], float (&D)[5])
{
    constexpr int cx = CX(I), cy = CY(I), cz = CZ(I);
    const float m = mu[I];
    if constexpr (SHELL(I) == 2) {
        if constexpr (cz == 0) D[0] += (cx * cy > 0 ? 0.25f : -0.25f) * m;
        if constexpr (cy == 0) D[1] += (cx * cz > 0 ? 0.25f : -0.25f) * m;
        if constexpr (cx == 0) D[2] += (cy * cz > 0 ? 0.25f : -0.25f) * m;
    }
    if constexpr (SHELL(I) == 1) {
        if constexpr (cy != 0) D[3] -= m * (1.f / 3.f);
        else D[3] += m * (1.f / 6.f);
        if constexpr (cz != 0) D[4] -= m * (1.f / 3.f);
        else D[4] += m * (1.f / 6.f);
    }
    if constexpr (I + 1 < 27) dual_dots<I + 1>(mu, D);
}

template <int J = 0>
__device__ __forceinline__ void write_lambda(float *__restrict__ lam, int pstride, int off, float Ldr, float Ljx,
                                             float Ljy, float Ljz, const float (&Dp)[5])
{
    constexpr int cx = CX(J), cy = CY(J), cz = CZ(J);
    float v = Ldr + cx * Ljx + cy * Ljy + cz * Ljz;
    v += (cx * cy) * Dp[0] + (cx * cz) * Dp[1] + (cy * cz) * Dp[2];
    v += (cx * cx - cy * cy) * Dp[3] + (cx * cx - cz * cz) * Dp[4];
    lam[J * pstride + off] = v;
    if constexpr (J + 1 < 27) write_lambda<J + 1>(lam, pstride, off, Ldr, Ljx, Ljy, Ljz, Dp);
}

template <typename T, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_adjoint(const Geom g, const Tiles t, const AdjointArgs a)
{
    const int tile = xcd_tile(blockIdx.x, gridDim.x, t.xcd);
    const int kb = tile % t.nkb, rest = tile / t.nkb, zc = rest % t.nzc, b = rest / t.nzc + t.b0;
    const int k = kb * BLOCK + threadIdx.x;
    if (k >= g.ncol) return;
    int col[9];
#pragma unroll
    for (int d = 0; d < 9; ++d) col[d] = g.nbr[d * g.P + k];
    const Pull<T> p = make_pull((const T *)a.state + (size_t)b * g.pipe, (size_t)g.pstride, g.nbr, g.P, k);
    const unsigned rowb = (unsigned)g.P * sizeof(T);
    const float *fs = g.fshape + (size_t)b * 3 * g.P;
    const float px = fs[k], py = fs[g.P + k], pq = fs[2 * g.P + k];
    const float sig = (a.cursor >= 0 && a.cursor < g.n_sigma) ? g.sigma[a.cursor] : 0.f;
    const float *lin = a.lam_in + (size_t)b * g.pipe;
    float *lout = a.lam_out + (size_t)b * g.pipe;
    const float om1 = 1.f - g.omega;
    const float we = (float)a.energy_weight;
    double G[3] = {0.0, 0.0, 0.0};
    const int z0 = zc * t.zchunk, z1 = min(z0 + t.zchunk, g.nz);
    for (int z = z0; z < z1; ++z) {
        const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z == g.nz - 1 ? 0 : z + 1;
        float v[27];
        gather<T>(p, (unsigned)z * rowb, (unsigned)zm * rowb, (unsigned)zp * rowb, v);
        const float cz = g.ztab[z], sz = g.ztab[g.nz + z];
        const float ax = sig * cz * px, ay = sig * cz * py, az = g.accel_z + sig * sz * pq;
        const Moments m = moments_of(v);
        float ux, uy, uz;
        const CollideCtx c = collide_setup(m, ax, ay, az, g.omega, ux, uy, uz);
        const float rho = c.rho;
        float mu[27];
        if (a.has_next) {
            gather_transpose(lin, g.pstride, g.P, col, k, z, zm, zp, mu);
        } else {
#pragma unroll
            for (int i = 0; i < 27; ++i) mu[i] = 0.f;
        }
        PopAdj s = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        pop_adjoint(c, mu, s);
        float D[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
        dual_dots(mu, D);
        float Dp[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) Dp[q] = om1 * D[q];
        // moment part: sum_k D'_k (-m^eq_k + R_k / 2), printed m_4..8^eq and R_4..8
        const float Qr = Dp[0] * (-ux * uy + 0.5f * (ay * ux + ax * uy)) + Dp[1] * (-ux * uz + 0.5f * (az * ux + ax * uz)) +
                         Dp[2] * (-uy * uz + 0.5f * (az * uy + ay * uz)) +
                         Dp[3] * (-(ux * ux - uy * uy) + (ax * ux - ay * uy)) +
                         Dp[4] * (-(ux * ux - uz * uz) + (ax * ux - az * uz));
        const float Qux = rho * (Dp[0] * (-uy + 0.5f * ay) + Dp[1] * (-uz + 0.5f * az) + (Dp[3] + Dp[4]) * (-2.f * ux + ax));
        const float Quy = rho * (Dp[0] * (-ux + 0.5f * ax) + Dp[2] * (-uz + 0.5f * az) + Dp[3] * (2.f * uy - ay));
        const float Quz = rho * (Dp[1] * (-ux + 0.5f * ax) + Dp[2] * (-uy + 0.5f * ay) + Dp[4] * (2.f * uz - az));
        const float Qax = rho * (0.5f * Dp[0] * uy + 0.5f * Dp[1] * uz + (Dp[3] + Dp[4]) * ux);
        const float Qay = rho * (0.5f * Dp[0] * ux + 0.5f * Dp[2] * uz - Dp[3] * uy);
        const float Qaz = rho * (0.5f * Dp[1] * ux + 0.5f * Dp[2] * uy - Dp[4] * uz);
        float Lr = s.Sr + Qr;
        float Lux = rho * s.Sux + Qux, Luy = rho * s.Suy + Quy, Luz = rho * s.Suz + Quz;
        if (a.in_window) {  // E = 1/2 rho u_z^2 with weight 1/(W N_f)
            Lr += we * 0.5f * uz * uz;
            Luz += we * rho * uz;
        }
        // chain rule through u = j/rho + a/2
        const float inv = __builtin_amdgcn_rcpf(rho);
        const float Ljx = Lux * inv, Ljy = Luy * inv, Ljz = Luz * inv;
        const float Ldr = Lr - (Lux * (ux - 0.5f * ax) + Luy * (uy - 0.5f * ay) + Luz * (uz - 0.5f * az)) * inv;
        const float sx = 0.5f * rho * s.Sax + Qax + 0.5f * Lux;
        const float sy = 0.5f * rho * s.Say + Qay + 0.5f * Luy;
        const float sz_ = 0.5f * rho * s.Saz + Qaz + 0.5f * Luz;
        write_lambda(lout, g.pstride, z * g.P + k, Ldr, Ljx, Ljy, Ljz, Dp);
        G[0] += (double)cz * (double)sx;
        G[1] += (double)cz * (double)sy;
        G[2] += (double)sz * (double)sz_;
    }
    double *gp = a.grad_part + (((size_t)b * t.nzc + zc) * g.P + k) * 3;
    gp[0] = G[0];
    gp[1] = G[1];
    gp[2] = G[2];
}

// per-column sums over z-chunks (fixed order)
__global__ __launch_bounds__(256) void k_grad_columns(const double *__restrict__ part, double *__restrict__ colsum,
                                                      int nzc, int P, int ncol, int B)
{
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (long long)B * ncol) return;
    const int b = (int)(idx / ncol), k = (int)(idx % ncol);
    double s[3] = {0.0, 0.0, 0.0};
    for (int zc = 0; zc < nzc; ++zc) {
        const double *p = part + (((size_t)b * nzc + zc) * P + k) * 3;
        s[0] += p[0];
        s[1] += p[1];
        s[2] += p[2];
    }
    double *o = colsum + ((size_t)b * P + k) * 3;
    o[0] = s[0];
    o[1] = s[1];
    o[2] = s[2];
}

// grad[b][q] += sigma * sum_k colsum[b][k] . shape_q(k), one block per (b, q)
__global__ __launch_bounds__(256) void k_project(const double *__restrict__ colsum, const double *__restrict__ modes,
                                                 int nq, int P, int ncol, double sigma, double *__restrict__ grad)
{
    __shared__ double lds[256];
    const int b = blockIdx.x / nq, q = blockIdx.x % nq;
    double acc = 0.0;
    for (int k = threadIdx.x; k < ncol; k += 256) {
        const double *cs = colsum + ((size_t)b * P + k) * 3;
        acc += cs[0] * modes[((size_t)q * 3 + 0) * P + k] + cs[1] * modes[((size_t)q * 3 + 1) * P + k] +
               cs[2] * modes[((size_t)q * 3 + 2) * P + k];
    }
    lds[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) grad[(size_t)b * nq + q] += sigma * lds[0];
}

hipError_t launch_adjoint(int storage, const Geom &g, const Tiles &t, const AdjointArgs &a, hipStream_t s)
{
    const dim3 grid((unsigned)(t.count() * t.nb));
    if (storage == 1)
        hipLaunchKernelGGL((k_adjoint<__half, 256>), grid, dim3(256), 0, s, g, t, a);
    else
        hipLaunchKernelGGL((k_adjoint<float, 256>), grid, dim3(256), 0, s, g, t, a);
    return hipGetLastError();
}

hipError_t launch_project_grad(const Geom &g, const Tiles &t, const double *grad_part, double *colsum,
                               const double *modes, int nq, double sigma, double *grad, hipStream_t s)
{
    const long long n = (long long)g.B * g.ncol;
    hipLaunchKernelGGL(k_grad_columns, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, grad_part, colsum, t.nzc, g.P,
                       g.ncol, g.B);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_project, dim3((unsigned)(g.B * nq)), dim3(256), 0, s, colsum, modes, nq, g.P, g.ncol, sigma,
                       grad);
    return hipGetLastError();
}

}  // namespace lbm
