// lbm_adjoint.hip -- discrete adjoint of the fused stream-collide step.
//
// Forward step: f^{n+1} = S C(f^n, a^n).  One reverse step at cursor c:
//     mu        = S^T lambda^{c+1}                  (adjoint of the post-collision state)
//     lambda^c  = (dC/df)^T mu + dE_c/df            (E_c: streamwise energy of f^c)
//     s(x)      = (dC/da)^T mu + dE_c/da            (sensitivity to the body acceleration)
// C depends on f only through rho, j and the stress moments m_4..m_8, so the
// vector-Jacobian product is the chain rule through these 9 moments, derived
// by hand from the collision of the forward kernel (deviation form of the
// Hermite-6 equilibrium, Guo forcing, relaxation of m_4..8 with omega).  The
// stress moments enter C linearly with constant coefficients, so dC/df
// depends on f only through rho and j: the reverse step reads them from a
// moment record of the recompute (k_step_record below) or sums them from a
// saved state.
// The force sensitivities are accumulated per column in FP64 and projected
// onto the trigger-force mode shapes of Eq. (TurbForce).
#include "lbm_device.h"
#include "lbm_internal.h"
#include "lbm_step.h"

namespace lbm {

// The adjoint state is stored as S (float or double); the vector-Jacobian
// arithmetic is FP64 (R) for either: the forward moments (recorded in the
// forward's arithmetic type, or summed from the saved state decoded as in
// the forward kernel) are promoted, the adjoint state promoted on load and
// rounded to S on store.  (With FP32 arithmetic the gradient of the 2000-step
// adjoint workload is 1.4e-4 from central differences; with FP64 arithmetic
// it is 3.6e-5 whether the state is stored in FP32 or FP64.)

// mu = S^T lambda, the transpose of the pull.  Bounce-back wall: mu_j(y) =
// lambda_j(y + c_j) if y + c_j is fluid, else lambda_opp(j)(y).  The
// interpolated wall (coefficients cf as in the forward pull) adds, for the
// post-collision value g*_j(y):
//  - y + c_j solid: it enters the wall link (y, opp(j)) with weight c = |cf|;
//  - y - c_j solid, link (y, j) in own-node mode (cf > 0): weight 1 - cf in
//    that link (X = g*_j(y));
//  - y + c_j fluid with y + 2 c_j solid, link (y + c_j, opp(j)) in far mode
//    (cf < 0): weight 1 + cf in that link (X = g*_j of the node behind it).
// Coefficient tables hold 0 for fluid slots, so the mode tests need no
// neighbour masks.
template <typename S, typename R, bool WALL, int J = 0, typename M>
__device__ __forceinline__ void gather_transpose(const Pull<S> &pl, unsigned zo, unsigned zmo, unsigned zpo,
                                                 const double *bcoef, M (&mu)[27])
{
    constexpr int cx = CX(J), cy = CY(J);
    constexpr int d = NSLOT(cx, cy);
    // lambda_J(y + c_J), or lambda_opp(J)(y) where y + c_J is solid: the
    // pull of population opp(J) with the slots swapped
    mu[J] = M(pull_one<S, OPP(J), FORM_W, false>(pl, zo, zmo, zpo));
    if constexpr (WALL && d != 4) {
        constexpr int cz = CZ(J);
        const unsigned zs = cz == 0 ? zo : (cz > 0 ? zpo : zmo);
        const bool solid = pl.wall & (1u << d);
        const unsigned sc = pl.colo[d] / sizeof(S);  // the neighbour's column (this one where solid)
        const double cf = bcoef[(size_t)d * pl.P + sc];
        if (solid) {
            mu[J] *= R(cf > 0.0 ? cf : -cf);
        } else if (cf < 0.0) {
            const unsigned off = zs + pl.colo[d];
            if (pl.ok_load(off)) mu[J] += R(1.0 + cf) * R(Codec<S>::template ld<0>(pl.base + OPP(J) * pl.pbytes, off));
        }
        const double co = bcoef[(size_t)(8 - d) * pl.P + pl.own / sizeof(S)];
        if (co > 0.0 && co != 1.0) {
            const unsigned off = zo + pl.own;
            if (pl.ok_load(off)) mu[J] += R(1.0 - co) * R(Codec<S>::template ld<0>(pl.base + J * pl.pbytes, off));
        }
    }
    if constexpr (J + 1 < 27) gather_transpose<S, R, WALL, J + 1>(pl, zo, zmo, zpo, bcoef, mu);
}

// per-axis equilibrium factors 1 + d_c(u) and their u-derivatives (see the
// forward collision): d_0 = -3u^2/2, d_+-1 = +-3u + 3u^2, their first
// derivatives d'_0 = -3u, d'_+-1 = +-3 + 6u (the second, -3 and 6, are constants)
template <typename R> struct AxisR {
    R e0, ep, em;   // 1 + d_c
    R q0, qp, qm;   // d'_c
};
template <typename R> __device__ __forceinline__ AxisR<R> axis_r(R u)
{
    const R u2 = u * u, u3 = R(3) * u;
    return AxisR<R>{R(1) - R(1.5) * u2, R(1) + u3 + R(3) * u2, R(1) - u3 + R(3) * u2, -u3, R(3) + R(6) * u,
                    R(-3) + R(6) * u};
}

template <typename R> struct PopAdj {
    R Sr, Sux, Suy, Suz, Sax, Say, Saz;
};

// population part: sum_i mu_i d/d(rho, u, a) [ (f^eq_i - w_i) + F_i/2 ]
// with f^eq_i - w_i = w_i (rho Pi_i - 1), Pi_i = e_x e_y e_z (one factor
// 1 + d_c(u) per axis) and F_i = rho w_i a . grad_u Pi_i.  The weights
// factor by axis too (w_i = w1(c_x) w1(c_y) w1(c_z), w1(0) = 2/3, w1(+-1) =
// 1/6), so every term of the sum over the 27 populations is a product of one
// factor per axis: w1 e, w1 q = w1 d'_c or w1 h = w1 d''_c of that axis.  The
// sum is contracted one axis at a time (x, then y, then z): ten sums T_fgh =
// sum_i mu_i (w1 f)(c_x) (w1 g)(c_y) (w1 h)(c_z) give every derivative.
template <typename R> struct AxisW {
    R e[3], q[3];  // w1(c) (1 + d_c(u)) and w1(c) d'_c(u) for c = 0, +1, -1
};
template <typename R> __device__ __forceinline__ AxisW<R> axis_w(const AxisR<R> &a)
{
    const R w0 = R(2) / R(3), w1 = R(1) / R(6);
    return AxisW<R>{{w0 * a.e0, w1 * a.ep, w1 * a.em}, {w0 * a.q0, w1 * a.qp, w1 * a.qm}};
}
// w1(c) d''_c: d''_0 = -3, d''_+-1 = 6
template <typename R> __device__ __forceinline__ constexpr R axis_h(int k) { return k == 0 ? R(-2) : R(1); }
__host__ __device__ constexpr int cval(int k) { return k == 0 ? 0 : (k == 1 ? 1 : -1); }

template <typename R, typename M>
__device__ __forceinline__ void pop_adjoint(const AxisR<R> &X, const AxisR<R> &Y, const AxisR<R> &Z, R ax, R ay, R az,
                                            const M (&mu)[27], PopAdj<R> &s)
{
    const AxisW<R> x = axis_w(X), y = axis_w(Y), z = axis_w(Z);
    R eee = 0, qee = 0, eqe = 0, eeq = 0, hee = 0, ehe = 0, eeh = 0, qqe = 0, qeq = 0, eqq = 0;
#pragma unroll
    for (int kz = 0; kz < 3; ++kz) {
        R Yee = 0, Yqe = 0, Yeq = 0, Yhe = 0, Yeh = 0, Yqq = 0;  // (x factor, y factor)
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
            R Xe = 0, Xq = 0, Xh = 0;
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const R m = R(mu[IDX(cval(kx), cval(ky), cval(kz))]);
                Xe += m * x.e[kx];
                Xq += m * x.q[kx];
                Xh += m * axis_h<R>(kx);
            }
            Yee += Xe * y.e[ky];
            Yqe += Xq * y.e[ky];
            Yeq += Xe * y.q[ky];
            Yhe += Xh * y.e[ky];
            Yeh += Xe * axis_h<R>(ky);
            Yqq += Xq * y.q[ky];
        }
        eee += Yee * z.e[kz];
        qee += Yqe * z.e[kz];
        eqe += Yeq * z.e[kz];
        eeq += Yee * z.q[kz];
        hee += Yhe * z.e[kz];
        ehe += Yeh * z.e[kz];
        eeh += Yee * axis_h<R>(kz);
        qqe += Yqq * z.e[kz];
        qeq += Yqe * z.q[kz];
        eqq += Yeq * z.q[kz];
    }
    const R h = R(0.5);
    s.Sr = eee + h * (ax * qee + ay * eqe + az * eeq);            // d/d rho
    s.Sux = qee + h * (ax * hee + ay * qqe + az * qeq);           // d/d u_x (then times rho)
    s.Suy = eqe + h * (ax * qqe + ay * ehe + az * eqq);
    s.Suz = eeq + h * (ax * qeq + ay * eqq + az * eeh);
    s.Sax = qee;                                                  // d/d a (then times rho/2)
    s.Say = eqe;
    s.Saz = eeq;
}

// D_k = <mu, d_k>, the columns 4..8 of the inverse moment matrix
template <typename R, int I = 0, typename M>
__device__ __forceinline__ void dual_dots(const M (&mu)[27], R (&D)[5])
{
    constexpr int cx = CX(I), cy = CY(I), cz = CZ(I);
    const R m = R(mu[I]);
    if constexpr (SHELL(I) == 2) {
        if constexpr (cz == 0) D[0] += (cx * cy > 0 ? R(0.25) : R(-0.25)) * m;
        if constexpr (cy == 0) D[1] += (cx * cz > 0 ? R(0.25) : R(-0.25)) * m;
        if constexpr (cx == 0) D[2] += (cy * cz > 0 ? R(0.25) : R(-0.25)) * m;
    }
    if constexpr (SHELL(I) == 1) {
        if constexpr (cy != 0) D[3] -= m * (R(1) / R(3));
        else D[3] += m * (R(1) / R(6));
        if constexpr (cz != 0) D[4] -= m * (R(1) / R(3));
        else D[4] += m * (R(1) / R(6));
    }
    if constexpr (I + 1 < 27) dual_dots<R, I + 1>(mu, D);
}

template <typename S, typename R, int J = 0>
__device__ __forceinline__ void write_lambda(const Pull<S> &pl, char *lam, unsigned off, R Ldr, R Ljx, R Ljy, R Ljz,
                                             const R (&Dp)[5])
{
    constexpr int cx = CX(J), cy = CY(J), cz = CZ(J);
    R v = Ldr + R(cx) * Ljx + R(cy) * Ljy + R(cz) * Ljz;
    v += R(cx * cy) * Dp[0] + R(cx * cz) * Dp[1] + R(cy * cz) * Dp[2];
    v += R(cx * cx - cy * cy) * Dp[3] + R(cx * cx - cz * cz) * Dp[4];
    if (pl.ok_store(off)) Codec<S>::template st<J>(lam + J * pl.pbytes, off, S(v));
    if constexpr (J + 1 < 27) write_lambda<S, R, J + 1>(pl, lam, off, Ldr, Ljx, Ljy, Ljz, Dp);
}

#ifndef LBM_ADJ_WAVES_PER_EU
#define LBM_ADJ_WAVES_PER_EU 0
#endif
#if LBM_ADJ_WAVES_PER_EU > 0
#define LBM_ADJ_OCCUPANCY __attribute__((amdgpu_waves_per_eu(LBM_ADJ_WAVES_PER_EU)))
#else
#define LBM_ADJ_OCCUPANCY
#endif

// REC: the forward state's moments come from a record of the recording step
// (a.rec, [b][4][population stride] of W) instead of a gather of the saved
// state (a.state): 16 B (FP64 forward: 32 B) per node instead of 108 B, and
// no forward-state gather in the kernel.
template <typename T, typename S, int BLOCK, bool WALL, bool REC>
__global__ __launch_bounds__(BLOCK) LBM_ADJ_OCCUPANCY void k_adjoint(const Geom g, const Tiles t, const AdjointArgs a)
{
    using R = double;
    using W = typename RealOf<T>::type;  // the forward step's arithmetic type
    const int tile = xcd_tile(blockIdx.x, gridDim.x, t.xcd);
    const int kb = tile % t.nkb, rest = tile / t.nkb, zc = rest % t.nzc, b = rest / t.nzc + t.b0;
    const int k = kb * BLOCK + threadIdx.x;
    if (k >= g.ncol) return;
    __shared__ float lref[REC ? 1 : href_lds_floats<T, BLOCK>()];
    Pull<T, WALL> p{};
    if constexpr (!REC)
        p = make_pull<T, WALL>((const T *)a.state + (size_t)b * g.pipe, (size_t)g.pstride, g.nbr, g.P, k, g.bcoef,
                               g.href, lref + 27 * threadIdx.x, g.check);
    const unsigned rowb = (unsigned)g.P * sizeof(T);
    const W *rec = REC ? (const W *)a.rec + (size_t)b * 4 * g.pstride + k : nullptr;
    const Shape<W> sh = shape_of<W>(g, b, k);
    const W sig = sigma_of<W>(g, a.cursor);
    // the adjoint state, addressed as the forward state (32-bit offsets within a population)
    const Pull<S> pl = make_pull<S, false>((const S *)a.lam_in + (size_t)b * g.pipe, (size_t)g.pstride, g.nbr, g.P,
                                           k, nullptr, nullptr, nullptr, g.check);
    char *lout = reinterpret_cast<char *>((S *)a.lam_out + (size_t)b * g.pipe);
    const unsigned lrow = (unsigned)g.P * sizeof(S);
    const R om1 = R(1) - R(omega_of<W>(g));
    const R we = R(a.energy_weight);
    double G[3] = {0.0, 0.0, 0.0};
    const int z0 = zc * t.zchunk, z1 = min(z0 + t.zchunk, g.nz);
    for (int z = z0; z < z1; ++z) {
        const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z == g.nz - 1 ? 0 : z + 1;
        // the forward's z factors, for the projection of the sensitivities
        double cz, sz;
        if constexpr (sizeof(W) == 8) {
            cz = g.ztab64[z];
            sz = g.ztab64[g.nz + z];
        } else {
            cz = (double)g.ztab[z];
            sz = (double)g.ztab[g.nz + z];
        }
        // the forward step's body acceleration (computed in its arithmetic type W), then promoted
        W fax, fay, faz;
        body_force<W>(g, z, sig, sh.px, sh.py, sh.pq, fax, fay, faz);
        const R ax = R(fax), ay = R(fay), az = R(faz);
        R dr = 0, jx = 0, jy = 0, jz = 0;
        if constexpr (REC) {
            // the moments the forward step computed from this state
            const size_t e = (size_t)z * g.P;
            if (check_ok(g.check, e + k < (size_t)g.pstride, CHK_LOAD)) {
                dr = R(rec[e]);
                jx = R(rec[e + g.pstride]);
                jy = R(rec[e + 2 * (size_t)g.pstride]);
                jz = R(rec[e + 3 * (size_t)g.pstride]);
            }
        } else {
            W v[27];
            pull_opaque<true>(p);
            gather<T, FORM_S, WALL>(p, (unsigned)z * rowb, (unsigned)zm * rowb, (unsigned)zp * rowb, v);
#pragma unroll
            for (int i = 0; i < 27; ++i) {
                const R vi = R(v[i]);
                dr += vi;
                jx += R(CX(i)) * vi;
                jy += R(CY(i)) * vi;
                jz += R(CZ(i)) * vi;
            }
        }
        const R rho = R(1) + dr;
        const R inv = R(1) / rho;
        const R ux = jx * inv + R(0.5) * ax, uy = jy * inv + R(0.5) * ay, uz = jz * inv + R(0.5) * az;
        const AxisR<R> X = axis_r(ux), Y = axis_r(uy), Z = axis_r(uz);
        // the gathered adjoint values: without the interpolated wall they are
        // the stored values themselves, kept in the storage type
        using M = typename std::conditional<WALL, R, S>::type;
        M mu[27];
        if (a.has_next) {
            gather_transpose<S, R, WALL>(pl, (unsigned)z * lrow, (unsigned)zm * lrow, (unsigned)zp * lrow, g.bcoef, mu);
        } else {
#pragma unroll
            for (int i = 0; i < 27; ++i) mu[i] = M(0);
        }
        PopAdj<R> s;
        pop_adjoint<R>(X, Y, Z, ax, ay, az, mu, s);
        R D[5] = {0, 0, 0, 0, 0};
        dual_dots<R>(mu, D);
        R Dp[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) Dp[q] = om1 * D[q];
        const R h = R(0.5);
        // moment part: sum_k D'_k (-m^eq_k + R_k / 2), printed m_4..8^eq and R_4..8
        const R Qr = Dp[0] * (-ux * uy + h * (ay * ux + ax * uy)) + Dp[1] * (-ux * uz + h * (az * ux + ax * uz)) +
                     Dp[2] * (-uy * uz + h * (az * uy + ay * uz)) + Dp[3] * (-(ux * ux - uy * uy) + (ax * ux - ay * uy)) +
                     Dp[4] * (-(ux * ux - uz * uz) + (ax * ux - az * uz));
        const R Qux = rho * (Dp[0] * (-uy + h * ay) + Dp[1] * (-uz + h * az) + (Dp[3] + Dp[4]) * (R(-2) * ux + ax));
        const R Quy = rho * (Dp[0] * (-ux + h * ax) + Dp[2] * (-uz + h * az) + Dp[3] * (R(2) * uy - ay));
        const R Quz = rho * (Dp[1] * (-ux + h * ax) + Dp[2] * (-uy + h * ay) + Dp[4] * (R(2) * uz - az));
        const R Qax = rho * (h * Dp[0] * uy + h * Dp[1] * uz + (Dp[3] + Dp[4]) * ux);
        const R Qay = rho * (h * Dp[0] * ux + h * Dp[2] * uz - Dp[3] * uy);
        const R Qaz = rho * (h * Dp[1] * ux + h * Dp[2] * uy - Dp[4] * uz);
        R Lr = s.Sr + Qr;
        R Lux = rho * s.Sux + Qux, Luy = rho * s.Suy + Quy, Luz = rho * s.Suz + Quz;
        if (a.in_window) {  // E = 1/2 rho u_z^2 with weight 1/(W N_f)
            Lr += we * h * uz * uz;
            Luz += we * rho * uz;
        }
        // chain rule through u = j/rho + a/2
        const R Ljx = Lux * inv, Ljy = Luy * inv, Ljz = Luz * inv;
        const R Ldr = Lr - (Lux * (ux - h * ax) + Luy * (uy - h * ay) + Luz * (uz - h * az)) * inv;
        const R sx = h * rho * s.Sax + Qax + h * Lux;
        const R sy = h * rho * s.Say + Qay + h * Luy;
        const R sz_ = h * rho * s.Saz + Qaz + h * Luz;
        write_lambda<S, R>(pl, lout, (unsigned)z * lrow + pl.own, Ldr, Ljx, Ljy, Ljz, Dp);
        G[0] += cz * (double)sx;
        G[1] += cz * (double)sy;
        G[2] += sz * (double)sz_;
    }
    // accumulated over the steps of the sweep with sigma(c), the time factor
    // of this step's trigger force (each slot belongs to one thread, and the
    // steps run in order, so the sums are deterministic)
    const double sd = (double)sig;
    if (sd != 0.0) {
        double *gp = a.grad_part + (((size_t)b * t.nzc + zc) * g.P + k) * 3;
        gp[0] += sd * G[0];
        gp[1] += sd * G[1];
        gp[2] += sd * G[2];
    }
}

// acc[b][k] = sum over the z-chunks of the column partials (each the sum
// over the sweep's steps so far of sigma(n) times the step's sensitivities):
// the force sensitivity of every column.  The partials of one (pipe,
// z-chunk) are 3 P consecutive doubles; a block takes 64 of them (one per
// lane), its 16 waves sum every 16th z-chunk each, and wave 0 adds the 16
// wave sums in a fixed order (deterministic).
constexpr int kAccWaves = 16;
__global__ __launch_bounds__(64 * kAccWaves) void k_grad_accumulate(const double *__restrict__ part,
                                                                    double *__restrict__ acc, int nzc, int P,
                                                                    int ncol, int blocks_per_pipe)
{
    __shared__ double red[kAccWaves][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int b = blockIdx.x / blocks_per_pipe;
    const int e = (blockIdx.x % blocks_per_pipe) * 64 + lane;  // 3 k + component
    const bool in = e < 3 * ncol;
    double s = 0.0;
    if (in)
        for (int zc = w; zc < nzc; zc += kAccWaves) s += part[((size_t)b * nzc + zc) * 3 * P + e];
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && in) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < kAccWaves; ++q) t += red[q][lane];
        acc[(size_t)b * 3 * P + e] = t;
    }
}

// grad[b][q] = base[b][q] + sum_k acc[b][k] . shape_q(k), one block per (b, q)
__global__ __launch_bounds__(256) void k_project(const double *__restrict__ acc, const double *__restrict__ modes,
                                                 int nq, int P, int ncol, const double *__restrict__ base,
                                                 double *__restrict__ grad)
{
    __shared__ double lds[256];
    const int b = blockIdx.x / nq, q = blockIdx.x % nq;
    double sum = 0.0;
    for (int k = threadIdx.x; k < ncol; k += 256) {
        const double *cs = acc + ((size_t)b * P + k) * 3;
        sum += cs[0] * modes[((size_t)q * 3 + 0) * P + k] + cs[1] * modes[((size_t)q * 3 + 1) * P + k] +
               cs[2] * modes[((size_t)q * 3 + 2) * P + k];
    }
    lds[threadIdx.x] = sum;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) grad[(size_t)b * nq + q] = base[(size_t)b * nq + q] + lds[0];
}

template <typename T, typename R, bool REC>
static void adjoint_wall(const Geom &g, const Tiles &t, const AdjointArgs &a, hipStream_t s)
{
    const dim3 grid((unsigned)(t.count() * t.nb));
    if (g.bcoef)
        hipLaunchKernelGGL((k_adjoint<T, R, 256, true, REC>), grid, dim3(256), 0, s, g, t, a);
    else
        hipLaunchKernelGGL((k_adjoint<T, R, 256, false, REC>), grid, dim3(256), 0, s, g, t, a);
}

template <typename T, typename R>
static void adjoint_source(const Geom &g, const Tiles &t, const AdjointArgs &a, hipStream_t s)
{
    if (a.rec)
        adjoint_wall<T, R, true>(g, t, a, s);
    else
        adjoint_wall<T, R, false>(g, t, a, s);
}

hipError_t launch_adjoint(int storage, int precision, const Geom &g, const Tiles &t, const AdjointArgs &a,
                          hipStream_t s)
{
    if (storage == 2)  // FP64 forward: FP64 adjoint
        adjoint_source<double, double>(g, t, a, s);
    else if (precision == 2)
        storage == 1 ? adjoint_source<__half, double>(g, t, a, s) : adjoint_source<float, double>(g, t, a, s);
    else
        storage == 1 ? adjoint_source<__half, float>(g, t, a, s) : adjoint_source<float, float>(g, t, a, s);
    return hipGetLastError();
}

hipError_t launch_grad_accumulate(const Geom &g, const Tiles &t, const double *grad_part, double *acc, hipStream_t s)
{
    const int per_pipe = (3 * g.ncol + 63) / 64;
    hipLaunchKernelGGL(k_grad_accumulate, dim3((unsigned)(per_pipe * g.B)), dim3(64 * kAccWaves), 0, s, grad_part, acc,
                       t.nzc, g.P, g.ncol, per_pipe);
    return hipGetLastError();
}

hipError_t launch_project_grad(const Geom &g, const double *acc, const double *modes, int nq, const double *base,
                               double *grad, hipStream_t s)
{
    hipLaunchKernelGGL(k_project, dim3((unsigned)(g.B * nq)), dim3(256), 0, s, acc, modes, nq, g.P, g.ncol, base, grad);
    return hipGetLastError();
}

// One step of the two-buffer pattern (the step kernel's gather, collision and
// store, so the state equals lbm_step's bitwise) that also records the
// moments of the state it consumes for the adjoint (see step_tile).
template <typename T, int BLOCK, bool WALL>
__global__ __launch_bounds__(BLOCK) void k_step_record(const Geom g, const Tiles t, const T *__restrict__ src,
                                                       T *__restrict__ dst, int step_off,
                                                       typename RealOf<T>::type *__restrict__ rec)
{
    __shared__ float lref[href_lds_floats<T, BLOCK>()];
    const TileCoord tc = decode_tile(t, BLOCK);
    if (tc.k >= g.ncol) return;
    step_tile<T, STEP_AB, WALL, KIND_MRT6, true>(g, t, tc, src, dst, *g.step_dev + step_off,
                                                 lref + 27 * threadIdx.x, rec);
}

template <typename T>
static hipError_t step_record_t(const Geom &g, const Tiles &t, const void *src, void *dst, int off, void *rec,
                                hipStream_t s)
{
    using W = typename RealOf<T>::type;
    // the step's tiles and tile order, 256 columns wide
    Tiles tr = t;
    tr.block = 256;
    tr.nkb = (g.ncol + 255) / 256;
    const dim3 grid((unsigned)(tr.count() * tr.nb));
    if (g.bcoef)
        hipLaunchKernelGGL((k_step_record<T, 256, true>), grid, dim3(256), 0, s, g, tr, (const T *)src, (T *)dst, off,
                           (W *)rec);
    else
        hipLaunchKernelGGL((k_step_record<T, 256, false>), grid, dim3(256), 0, s, g, tr, (const T *)src, (T *)dst,
                           off, (W *)rec);
    return hipGetLastError();
}

hipError_t launch_step_record(int storage, const Geom &g, const Tiles &t, const void *src, void *dst, int off,
                              void *rec, hipStream_t s)
{
    if (storage == 2) return step_record_t<double>(g, t, src, dst, off, rec, s);
    return storage == 1 ? step_record_t<__half>(g, t, src, dst, off, rec, s)
                        : step_record_t<float>(g, t, src, dst, off, rec, s);
}

}  // namespace lbm
