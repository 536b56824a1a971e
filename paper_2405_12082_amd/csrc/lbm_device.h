// lbm_device.h -- device-side building blocks of the D3Q27 MRT pipe stepper
// for gfx950: lattice constants, storage codecs, the pull gather with
// halfway bounce-back, and the per-node collision in deviation form.
//
// Method: arXiv:2405.12082, appendix (Eqs. (Mmatrix), (mrt), (lambda), (m*),
// (Rmrti), (BoltzmannEquilibriumDistribution), (k*f*)) and Section II
// (Eqs. (collision), (streaming), (macroscopic_rho), (macroscopic_u), (fbc1)).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// D3Q27 velocities in the appendix order (rest, faces, xy/xz/yz edges, corners).
__host__ __device__ constexpr int CX(int i)
{
    constexpr int v[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
    return v[i];
}
__host__ __device__ constexpr int CY(int i)
{
    constexpr int v[27] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, 1, -1, -1, 1, 1, -1, -1};
    return v[i];
}
__host__ __device__ constexpr int CZ(int i)
{
    constexpr int v[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1};
    return v[i];
}
// opposite direction: c_opp(i) = -c_i
__host__ __device__ constexpr int OPP(int i)
{
    constexpr int v[27] = {0, 2, 1, 4, 3, 6, 5, 10, 9, 8, 7, 14, 13, 12, 11, 18, 17, 16, 15, 26, 25, 24, 23, 22, 21, 20, 19};
    return v[i];
}
__host__ __device__ constexpr int SHELL(int i) { return CX(i) * CX(i) + CY(i) * CY(i) + CZ(i) * CZ(i); }
// weights, Eq. (omegas): w0 = 8/27, w0/4, w0/16, w0/64 by |c|^2
__host__ __device__ constexpr float WGT(int i)
{
    return SHELL(i) == 0 ? 8.0f / 27.0f : SHELL(i) == 1 ? 2.0f / 27.0f : SHELL(i) == 2 ? 1.0f / 54.0f : 1.0f / 216.0f;
}
// FP16 storage scale 2^k ~ 1/w_i (exact power of two: the scaling is lossless)
__host__ __device__ constexpr float H_SCALE(int i)
{
    return SHELL(i) == 0 ? 4.0f : SHELL(i) == 1 ? 16.0f : SHELL(i) == 2 ? 64.0f : 256.0f;
}
__host__ __device__ constexpr float H_INV_SCALE(int i)
{
    return SHELL(i) == 0 ? 0.25f : SHELL(i) == 1 ? 0.0625f : SHELL(i) == 2 ? 0.015625f : 0.00390625f;
}
// in-plane neighbour slot of offset (dx, dy): d = (dy + 1) * 3 + (dx + 1)
__host__ __device__ constexpr int NSLOT(int dx, int dy) { return (dy + 1) * 3 + (dx + 1); }

// ---------------------------------------------------------------- codecs
template <typename T> struct Codec;
template <> struct Codec<float> {
    template <int I> __device__ static __forceinline__ float load(const float *p) { return __builtin_nontemporal_load(p); }
    template <int I> __device__ static __forceinline__ void store(float *p, float v) { __builtin_nontemporal_store(v, p); }
};
template <> struct Codec<__half> {
    template <int I> __device__ static __forceinline__ float load(const __half *p)
    {
        const unsigned short raw = __builtin_nontemporal_load(reinterpret_cast<const unsigned short *>(p));
        return __half2float(__ushort_as_half(raw)) * H_INV_SCALE(I);
    }
    template <int I> __device__ static __forceinline__ void store(__half *p, float v)
    {
        const __half h = __float2half_rn(v * H_SCALE(I));
        __builtin_nontemporal_store(__half_as_ushort(h), reinterpret_cast<unsigned short *>(p));
    }
};

// ---------------------------------------------------------------- gather
// Pull streaming, Eq. (streaming): g_i(x, n) = g*_i(x - c_i, n-1) if x - c_i
// is fluid, else the halfway bounce-back g*_opp(i)(x, n-1) (the Delta = 1/2
// case of Eq. (fbc1)).  `col` holds the columns of the 9 in-plane offsets
// (dx, dy) of the node (-1: solid); z - c_z wraps periodically.
template <typename T, int I>
__device__ __forceinline__ float pull_one(const T *__restrict__ pipe, int pstride, int P, const int (&col)[9],
                                          int k, int z, int zm, int zp)
{
    constexpr int cx = CX(I), cy = CY(I), cz = CZ(I);
    constexpr int d = NSLOT(-cx, -cy);
    const int zs = cz == 0 ? z : (cz > 0 ? zm : zp);
    const int sc = col[d];
    if (d == 4 || sc >= 0) return Codec<T>::template load<I>(pipe + I * pstride + zs * P + sc);
    return Codec<T>::template load<OPP(I)>(pipe + OPP(I) * pstride + z * P + k);
}

template <typename T, int I = 0>
__device__ __forceinline__ void gather(const T *__restrict__ pipe, int pstride, int P, const int (&col)[9], int k,
                                       int z, int zm, int zp, float (&g)[27])
{
    g[I] = pull_one<T, I>(pipe, pstride, P, col, k, z, zm, zp);
    if constexpr (I + 1 < 27) gather<T, I + 1>(pipe, pstride, P, col, k, z, zm, zp, g);
}

template <typename T, int I = 0>
__device__ __forceinline__ void store_all(T *__restrict__ pipe, int pstride, int off, const float (&g)[27])
{
    Codec<T>::template store<I>(pipe + I * pstride + off, g[I]);
    if constexpr (I + 1 < 27) store_all<T, I + 1>(pipe, pstride, off, g);
}

// ---------------------------------------------------------------- moments
struct Moments {
    float dr;           // rho - 1 = sum g_i
    float jx, jy, jz;   // sum c_i g_i (the weights carry no momentum)
    float m4, m5, m6;   // sum c_x c_y g, c_x c_z g, c_y c_z g
    float m7, m8;       // sum (c_x^2 - c_y^2) g, (c_x^2 - c_z^2) g
};

template <int I = 0>
__device__ __forceinline__ void accumulate_moments(const float (&g)[27], Moments &m)
{
    constexpr int cx = CX(I), cy = CY(I), cz = CZ(I);
    const float v = g[I];
    m.dr += v;
    if constexpr (cx == 1) m.jx += v;
    if constexpr (cx == -1) m.jx -= v;
    if constexpr (cy == 1) m.jy += v;
    if constexpr (cy == -1) m.jy -= v;
    if constexpr (cz == 1) m.jz += v;
    if constexpr (cz == -1) m.jz -= v;
    if constexpr (cx * cy == 1) m.m4 += v;
    if constexpr (cx * cy == -1) m.m4 -= v;
    if constexpr (cx * cz == 1) m.m5 += v;
    if constexpr (cx * cz == -1) m.m5 -= v;
    if constexpr (cy * cz == 1) m.m6 += v;
    if constexpr (cy * cz == -1) m.m6 -= v;
    if constexpr (cx * cx - cy * cy == 1) m.m7 += v;
    if constexpr (cx * cx - cy * cy == -1) m.m7 -= v;
    if constexpr (cx * cx - cz * cz == 1) m.m8 += v;
    if constexpr (cx * cx - cz * cz == -1) m.m8 -= v;
    if constexpr (I + 1 < 27) accumulate_moments<I + 1>(g, m);
}

__device__ __forceinline__ Moments moments_of(const float (&g)[27])
{
    Moments m = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    accumulate_moments(g, m);
    return m;
}

// ---------------------------------------------------------------- collision
// Per-axis factors of the equilibrium.  On D3Q27 the sixth-order Hermite
// equilibrium is exactly f_i^eq = rho w_i prod_a (1 + d_{c_ia}(u_a)) with
// d_0(u) = -3u^2/2 and d_{+-1}(u) = +-3u + 3u^2; its u-derivative uses
// d'_0 = -3u and d'_{+-1} = +-3 + 6u.
struct Axis {
    float d0, dp, dm;   // d_0, d_+1, d_-1
    float q0, qp, qm;   // derivatives
};
__device__ __forceinline__ Axis axis_factors(float u)
{
    const float u2 = u * u, u3 = 3.f * u;
    Axis a;
    a.d0 = -1.5f * u2;
    a.dp = u3 + 3.f * u2;
    a.dm = -u3 + 3.f * u2;
    a.q0 = -u3;
    a.qp = 3.f + 6.f * u;
    a.qm = -3.f + 6.f * u;
    return a;
}
template <int C> __device__ __forceinline__ float dsel(const Axis &a) { return C == 0 ? a.d0 : (C > 0 ? a.dp : a.dm); }
template <int C> __device__ __forceinline__ float qsel(const Axis &a) { return C == 0 ? a.q0 : (C > 0 ? a.qp : a.qm); }

struct CollideCtx {
    Axis X, Y, Z;
    float dr, rho;      // rho - 1 and rho
    float ax, ay, az;   // body acceleration
    float c4, c5, c6, c7, c8;   // (1 - omega) (m_k - m_k^eq + R_k/2), k = 4..8
};

// Relaxed non-equilibrium part of the stress moments, Eq. (m*) with
// Lam_k = omega for k = 4..8: m*_k - m^eq_k - R_k/2 = (1 - omega)(m_k - m^eq_k + R_k/2),
// using the printed m_4..8^eq and R_4..8.
__device__ __forceinline__ CollideCtx collide_setup(const Moments &m, float ax, float ay, float az, float omega,
                                                    float &ux, float &uy, float &uz)
{
    CollideCtx c;
    c.dr = m.dr;
    c.rho = 1.f + m.dr;
    const float inv = 1.f / c.rho;
    // Eq. (macroscopic_u): u = j/rho + a/2
    ux = m.jx * inv + 0.5f * ax;
    uy = m.jy * inv + 0.5f * ay;
    uz = m.jz * inv + 0.5f * az;
    c.ax = ax;
    c.ay = ay;
    c.az = az;
    c.X = axis_factors(ux);
    c.Y = axis_factors(uy);
    c.Z = axis_factors(uz);
    const float r = c.rho, om1 = 1.f - omega;
    const float xx = ux * ux, yy = uy * uy, zz = uz * uz;
    c.c4 = om1 * (m.m4 - r * ux * uy + 0.5f * r * (ay * ux + ax * uy));
    c.c5 = om1 * (m.m5 - r * ux * uz + 0.5f * r * (az * ux + ax * uz));
    c.c6 = om1 * (m.m6 - r * uy * uz + 0.5f * r * (az * uy + ay * uz));
    c.c7 = om1 * (m.m7 - r * (xx - yy) + r * (ax * ux - ay * uy));
    c.c8 = om1 * (m.m8 - r * (xx - zz) + r * (ax * ux - az * uz));
    return c;
}

// Post-collision deviation of population I:
//   g*_I = (f^eq_I - w_I) + F_I/2 + sum_k c_k d_k(I)
// f^eq - w = w (rho Pi - 1) = w ((rho-1) Pi + (Pi - 1)), Pi - 1 built without
// cancellation; F_I = a . grad_u f^eq_I (Guo forcing in population form,
// whose moments are the printed R^MRT); d_k = columns 4..8 of the inverse
// moment matrix (sparse: edge links for k = 4..6, face links for 7, 8).
template <int I>
__device__ __forceinline__ float post_collision(const CollideCtx &c)
{
    constexpr int cx = CX(I), cy = CY(I), cz = CZ(I);
    constexpr float w = WGT(I);
    const float dx = dsel<cx>(c.X), dy = dsel<cy>(c.Y), dz = dsel<cz>(c.Z);
    const float qx = qsel<cx>(c.X), qy = qsel<cy>(c.Y), qz = qsel<cz>(c.Z);
    const float exy = dx + dy + dx * dy;          // (1+dx)(1+dy) - 1
    const float pim1 = exy + dz * (1.f + exy);    // Pi - 1
    const float ez = 1.f + dz;
    const float feq = w * (c.dr * (1.f + pim1) + pim1);
    const float Fi = c.rho * w * (ez * (c.ax * qx * (1.f + dy) + c.ay * qy * (1.f + dx)) + c.az * qz * (1.f + exy));
    float v = feq + 0.5f * Fi;
    if constexpr (SHELL(I) == 1) {
        if constexpr (cx != 0) v += (c.c7 + c.c8) * (1.f / 6.f);
        if constexpr (cy != 0) v += c.c8 * (1.f / 6.f) - c.c7 * (1.f / 3.f);
        if constexpr (cz != 0) v += c.c7 * (1.f / 6.f) - c.c8 * (1.f / 3.f);
    }
    if constexpr (SHELL(I) == 2) {
        if constexpr (cz == 0) v += (cx * cy > 0 ? 0.25f : -0.25f) * c.c4;
        if constexpr (cy == 0) v += (cx * cz > 0 ? 0.25f : -0.25f) * c.c5;
        if constexpr (cx == 0) v += (cy * cz > 0 ? 0.25f : -0.25f) * c.c6;
    }
    return v;
}

template <int I = 0>
__device__ __forceinline__ void post_collision_all(const CollideCtx &c, float (&g)[27])
{
    g[I] = post_collision<I>(c);
    if constexpr (I + 1 < 27) post_collision_all<I + 1>(c, g);
}

// Equilibrium deviation f^eq_I(rho = 1 + dr, u) - w_I (used by the initialiser)
template <int I>
__device__ __forceinline__ float feq_dev(float dr, const Axis &X, const Axis &Y, const Axis &Z)
{
    const float dx = dsel<CX(I)>(X), dy = dsel<CY(I)>(Y), dz = dsel<CZ(I)>(Z);
    const float exy = dx + dy + dx * dy;
    const float pim1 = exy + dz * (1.f + exy);
    return WGT(I) * (dr * (1.f + pim1) + pim1);
}

// Workgroup -> tile: consecutive tiles go to the same XCD (workgroups are
// dispatched round-robin over the 8 XCDs, each with its own L2), so the
// halo lines shared by neighbouring tiles stay in one L2.
__device__ __forceinline__ int xcd_tile(int bid, int nblocks)
{
    const int q = nblocks >> 3, r = nblocks & 7, x = bid & 7, s = bid >> 3;
    return x * q + (x < r ? x : r) + s;
}

}  // namespace lbm
