// lbm_device.h -- device-side building blocks of the D3Q27 MRT pipe stepper
// for gfx950: lattice constants, storage codecs, the pull gather with the
// halfway bounce-back or the interpolated wall and the stores of the
// two-buffer and AA patterns, the per-node collision in deviation form, the
// body force and the XCD-aware tile order.
//
// Method: arXiv:2405.12082, appendix (Eqs. (Mmatrix), (mrt), (lambda), (m*),
// (Rmrti), (BoltzmannEquilibriumDistribution), (k*f*)) and Section II
// (Eqs. (collision), (streaming), (macroscopic_rho), (macroscopic_u), (fbc1),
// (fbc2), (TurbForce)).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_internal.h"

// Checked builds (LBM_CHECKED, see lbm_internal.h): every population load
// and store of the gather and store helpers below and every neighbour-table
// entry they use is tested against its extent; a violation sets a bit of
// the device word Geom::check and the access is skipped (a load returns 0).
// Release builds compile the tests away.
namespace lbm {

enum CheckBit : unsigned { CHK_NBR = 1u, CHK_LOAD = 2u, CHK_STORE = 4u, CHK_INDEX = 8u };
// true when ok; otherwise (checked builds) records bit in *flags
__device__ __forceinline__ bool check_ok(unsigned *flags, bool ok, unsigned bit)
{
    if constexpr (LBM_CHECKED) {
        if (!ok && flags) atomicOr(flags, bit);
        return ok;
    } else {
        return true;
    }
}

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
// the same weights as exact rationals in the arithmetic type R
template <typename R> __host__ __device__ constexpr R wgt(int i)
{
    return SHELL(i) == 0 ? R(8) / R(27) : SHELL(i) == 1 ? R(2) / R(27) : SHELL(i) == 2 ? R(1) / R(54) : R(1) / R(216);
}
// The weights are 2^k / 27: in FP32 every one of them carries the same
// relative rounding error (7.45e-9), so a post-collision state built as
// w_i X_i scales the mass and momentum deviations by 1 + 7.45e-9 at every
// step, a drift that grows with the steps where the flow is smooth enough
// for the roundings not to cancel.  w_i X = hi X + lo X with hi = fp32(w_i)
// and lo = fp32(w_i - hi) carries the weights to about 2^-48.  SPLIT = false
// (FP16 storage, whose own rounding is 2^-11 relative) takes fp32(w_i) alone:
// one FMA instead of two per population, 5% of that step's VALU work.
template <typename R, bool SPLIT = true> __device__ __forceinline__ R weigh(int i, R x, R add)
{
    if constexpr (sizeof(R) == 4 && SPLIT) {
        constexpr double dw[4] = {8.0 / 27.0, 2.0 / 27.0, 1.0 / 54.0, 1.0 / 216.0};
        const double w = dw[SHELL(i)];
        const float hi = (float)w, lo = (float)(w - (double)hi);
        return fmaf(hi, x, fmaf(lo, x, add));
    } else {
        return fma(wgt<R>(i), x, add);
    }
}
// arithmetic type of a storage type: FP64 storage computes in FP64, FP32 and
// FP16 storage compute in FP32
template <typename T> struct RealOf { using type = float; };
template <> struct RealOf<double> { using type = double; };
__device__ __forceinline__ float fma_r(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_r(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float rcp_r(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_r(double x) { return 1.0 / x; }

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
// Loads take a uniform (scalar) base and a 32-bit byte offset, so that the
// compiler emits global loads with an SGPR base and one VGPR offset.  Loads
// go through the caches (neighbouring waves share the partial lines of the
// shifted pull reads); stores are non-temporal (written once, read next step).
//
// FP16 storage keeps each value relative to a per-column reference: a
// post-collision deviation g*_i produced by node y is held as
//     h = fp16_rne(s_i g*_i - E_c(y)),   g*_i = h / s_i + E_c(y) / s_i,
// wherever it is stored (two buffers, AA slots), with s_i = 2^k ~ 1/w_i and
// E_c(y) = fp32(32/27 d_c(u0(y))), c = c_z of population i, d_c the
// per-axis equilibrium factor and u0 the streamwise velocity of the
// column's initial state (log-law profile; 0 when the pipe starts at rest).
// A reader decodes with the producer's column: the column it pulls from, or
// its own for a bounce-back.  The rounding of a value thus depends only on
// the value and its producer, so every pattern and launch form stores the
// same bits.  Since s_i w_i = 32/27 for every i, E_c / s_i is the
// initial equilibrium deviation w_i d_c(u0) of that population, so the 11
// bits of the FP16 mantissa go to the departure from the mean-flow
// equilibrium rather than to the mean flow itself.  ld/st take the addend
// E_c / s_i and the reference E_c; FP32 and FP64 storage ignore them.
// raw/dec split ld into the load of the stored word and its decode, for
// paths that issue several conditional loads before decoding any.
template <typename T> struct Codec;
template <> struct Codec<float> {
    using Raw = float;
    template <int I> __device__ static __forceinline__ float ld(const char *base, unsigned off, float = 0.f)
    {
        return *reinterpret_cast<const float *>(base + off);
    }
    __device__ static __forceinline__ Raw raw(const char *base, unsigned off)
    {
        return *reinterpret_cast<const float *>(base + off);
    }
    template <int I> __device__ static __forceinline__ float dec(Raw r, float = 0.f) { return r; }
    template <int I> __device__ static __forceinline__ void st(char *base, unsigned off, float v, float = 0.f)
    {
        __builtin_nontemporal_store(v, reinterpret_cast<float *>(base + off));
    }
};
template <> struct Codec<double> {
    using Raw = double;
    template <int I> __device__ static __forceinline__ double ld(const char *base, unsigned off, double = 0.0)
    {
        return *reinterpret_cast<const double *>(base + off);
    }
    __device__ static __forceinline__ Raw raw(const char *base, unsigned off)
    {
        return *reinterpret_cast<const double *>(base + off);
    }
    template <int I> __device__ static __forceinline__ double dec(Raw r, double = 0.0) { return r; }
    template <int I> __device__ static __forceinline__ void st(char *base, unsigned off, double v, double = 0.0)
    {
        __builtin_nontemporal_store(v, reinterpret_cast<double *>(base + off));
    }
};
// FP16 encode and decode, written out so that every kernel rounds alike.
// The encode is one mixed-precision FMA that rounds s v - E once, to the
// nearest half (v_fma_mixlo_f16; left to itself the compiler forms it in
// some kernels and an FP32 FMA plus a conversion, two roundings, in others).
// The decode converts the loaded half exactly, then one FP32 FMA (folded
// into a mixed-precision FMA that reads the loaded half, the scheduler
// interleaves the loads with their uses and the two-buffer step runs 25%
// slower, measured).  The scale is a uniform operand; the stored half sits
// zero-extended in a register of its own (see Raw).
__device__ __forceinline__ unsigned short h_encode(float v, float scale, float ref)
{
    unsigned h;
    asm("v_fma_mixlo_f16 %0, %1, %2, -%3" : "=v"(h) : "v"(v), "s"(scale), "v"(ref));
    return (unsigned short)(h & 0xffffu);
}
__device__ __forceinline__ float h_decode(unsigned raw, float inv_scale, float addend)
{
    float f;
    asm("v_cvt_f32_f16 %0, %1" : "=v"(f) : "v"(raw));
    return fmaf(f, inv_scale, addend);
}
template <> struct Codec<__half> {
    // a stored half, zero-extended into a word of its own (two halves packed
    // into one register would make each load wait for the other)
    using Raw = unsigned;
    template <int I> __device__ static __forceinline__ float ld(const char *base, unsigned off, float addend = 0.f)
    {
        return h_decode(*reinterpret_cast<const unsigned short *>(base + off), H_INV_SCALE(I), addend);
    }
    __device__ static __forceinline__ Raw raw(const char *base, unsigned off)
    {
        return *reinterpret_cast<const unsigned short *>(base + off);
    }
    template <int I> __device__ static __forceinline__ float dec(Raw r, float addend = 0.f)
    {
        return h_decode(r, H_INV_SCALE(I), addend);
    }
    template <int I> __device__ static __forceinline__ void st(char *base, unsigned off, float v, float ref = 0.f)
    {
        __builtin_nontemporal_store(h_encode(v, H_SCALE(I), ref), reinterpret_cast<unsigned short *>(base + off));
    }
};
// index of the population with velocity (cx, cy, cz)
__host__ __device__ constexpr int IDX(int cx, int cy, int cz)
{
    for (int i = 0; i < 27; ++i)
        if (CX(i) == cx && CY(i) == cy && CZ(i) == cz) return i;
    return -1;
}
// index of the reference of c_z = c in a column's three (c = 0, +1, -1)
__host__ __device__ constexpr int CZI(int c) { return c == 0 ? 0 : (c > 0 ? 1 : 2); }

// ---------------------------------------------------------------- gather
// FP16 references of one thread's column (see the codecs): the decode addend
// of the value population I receives, E_c(y) / s_I with y its producer (the
// source column, c = c_z of I; for a bounce-back link this column, c = c_z
// of opp(I)), and the own column's E_0, E_+, E_-.  Empty for FP32 / FP64.
template <typename T> struct HRef {
};
template <> struct HRef<__half> {
    // 27 floats of this thread in LDS, read back at each use: the kernels
    // make the pointer opaque once per plane (pull_opaque), so that the
    // compiler neither forwards the thread's own writes nor hoists the reads
    // out of the plane loop; either would hold all 27 values in vector
    // registers, which costs the step kernel its occupancy and serialises its
    // loads
    __attribute__((address_space(3))) float *pull;
    float own[3];
};
// an LDS pointer the compiler cannot see through (an empty asm statement
// that takes and returns the address; no memory is accessed)
__device__ __forceinline__ void lds_opaque(__attribute__((address_space(3))) float *&p)
{
    unsigned a = (unsigned)(size_t)p;
    asm volatile("" : "+v"(a));
    p = (__attribute__((address_space(3))) float *)(size_t)a;
}
// LDS the FP16 references of a workgroup of BLOCK threads take: 27 floats per
// thread, at stride 27 (odd: the lanes of a wave hit distinct banks)
template <typename T, int BLOCK> constexpr int href_lds_floats() { return sizeof(T) == 2 ? 27 * BLOCK : 1; }

// Per-thread view of one pipe's population buffer for one column k:
// byte offsets of the 9 in-plane neighbour columns (own column where the
// neighbour is solid), a bit mask of the solid ones, (interpolated wall
// only) where the column's wall coefficients are, and the FP16 references.
template <typename T, bool WALL = false> struct Pull {
    const char *base;   // pipe base
    size_t pbytes;      // bytes between populations (nz * P * sizeof(T))
    unsigned colo[9];   // byte offset of the column in slot d within a plane
    unsigned wall;      // bit d set: slot d is solid
    unsigned own;       // byte offset of column k within a plane
    const double *bc;   // interpolated wall: coefficient of slot d at bc[d * P] (0 for fluid slots)
    int P;
    HRef<T> ref;
    unsigned *chk;      // checked builds: the violation flags
    using R = typename RealOf<T>::type;
    // checked builds: a byte offset within one population's region
    __device__ __forceinline__ bool ok_load(unsigned off) const { return check_ok(chk, off < pbytes, CHK_LOAD); }
    __device__ __forceinline__ bool ok_store(unsigned off) const { return check_ok(chk, off < pbytes, CHK_STORE); }
    // decode addend of the value population I receives (pull or bounce-back)
    template <int I> __device__ __forceinline__ R add_pull() const
    {
        if constexpr (sizeof(T) == 2) return ref.pull[I];
        else return R(0);
    }
    // decode addend of population I's value produced by this column
    template <int I> __device__ __forceinline__ R add_own() const
    {
        if constexpr (sizeof(T) == 2) return ref.own[CZI(CZ(I))] * H_INV_SCALE(I);
        else return R(0);
    }
    // reference of population I's value produced by this column
    template <int I> __device__ __forceinline__ R ref_own() const
    {
        if constexpr (sizeof(T) == 2) return ref.own[CZI(CZ(I))];
        else return R(0);
    }
};

// href: FP16 storage's per-column references [3][P] (c_z = 0, +1, -1);
// lds: FP16 storage, this thread's 27 floats of LDS for them (see
// href_lds_floats; each thread reads back only what it wrote, so no barrier)
template <typename T, bool WALL = false>
__device__ __forceinline__ Pull<T, WALL> make_pull(const T *pipe, size_t pstride, const int *nbr, int P, int k,
                                                   const double *bcoef = nullptr, const float *href = nullptr,
                                                   float *lds = nullptr, unsigned *chk = nullptr)
{
    Pull<T, WALL> p;
    p.base = reinterpret_cast<const char *>(pipe);
    p.pbytes = pstride * sizeof(T);
    p.own = (unsigned)k * sizeof(T);
    p.wall = 0;
    p.chk = chk;
    check_ok(chk, k >= 0 && k < P, CHK_INDEX);
    int src[9];
#pragma unroll
    for (int d = 0; d < 9; ++d) {
        int c = nbr[d * P + k];
        if (!check_ok(chk, c >= -1 && c < P, CHK_NBR)) c = k;
        src[d] = c >= 0 ? c : k;
        p.colo[d] = (unsigned)src[d] * sizeof(T);
        if (c < 0) p.wall |= 1u << d;
    }
    p.bc = WALL ? bcoef + k : nullptr;
    p.P = P;
    if constexpr (sizeof(T) == 2) {
        p.ref.pull = (__attribute__((address_space(3))) float *)lds;
#pragma unroll
        for (int c = 0; c < 3; ++c) p.ref.own[c] = href[c * P + k];
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            const int d = NSLOT(-CX(i), -CY(i));
            const bool bb = p.wall & (1u << d);  // bounce-back: g*_opp(i) of this column
            p.ref.pull[i] = href[CZI(bb ? -CZ(i) : CZ(i)) * P + src[d]] * H_INV_SCALE(i);
        }
    }
    return p;
}

// Once per plane, FP16 storage: the LDS pointer of the references (see
// HRef) and, with MASK, the solid-slot mask made opaque.  The FP16 gather
// selects, per lane, the population a load reads (the pull or its
// bounce-back); with the mask visible the compiler hoists the 27 resulting
// 64-bit addresses out of the plane loop and keeps them in vector registers
// (some 50).  Where that costs an occupancy level (the interpolated wall,
// the AA pattern's push step, the observers) recomputing them per plane is
// faster; in the plain two-buffer step it is not (measured), so that one
// keeps them.  No effect for FP32 / FP64 storage.
template <bool MASK, typename T, bool WALL>
__device__ __forceinline__ void pull_opaque(Pull<T, WALL> &p)
{
    if constexpr (sizeof(T) == 2) {
        lds_opaque(p.ref.pull);
        if constexpr (MASK) asm volatile("" : "+v"(p.wall));
    }
}

// Pull streaming, Eq. (streaming): g_i(x, n) = g*_i(x - c_i, n-1) if x - c_i
// is fluid, else the halfway bounce-back g*_opp(i)(x, n-1) (the Delta = 1/2
// case of Eq. (fbc1)).  zo/zmo/zpo: byte offsets of planes z, z-1, z+1
// (periodic in z).  FORM_N reads the own slot.
template <typename T, int I, int FORM, bool WALL>
__device__ __forceinline__ typename RealOf<T>::type pull_one(const Pull<T, WALL> &p, unsigned zo, unsigned zmo,
                                                             unsigned zpo)
{
    if constexpr (FORM == FORM_N) {
        // g_I(x) itself, produced by x - c_I (or by x, as g*_opp(I), where x - c_I is solid)
        if (!p.ok_load(zo + p.own)) return 0;
        return Codec<T>::template ld<I>(p.base + I * p.pbytes, zo + p.own, p.template add_pull<I>());
    } else {
        constexpr int cx = CX(I), cy = CY(I), cz = CZ(I);
        constexpr int d = NSLOT(-cx, -cy);
        constexpr int here = FORM == FORM_W ? OPP(I) : I;  // physical slot of g*_I
        const unsigned zs = cz == 0 ? zo : (cz > 0 ? zmo : zpo);
        if constexpr (sizeof(T) == 2 && d != 4) {
            // FP16: one load from the selected slot (the producer's addend of
            // population I is fixed per column, bounce-back or not)
            const bool bb = p.wall & (1u << d);
            const char *b = p.base + (size_t)(bb ? OPP(here) : here) * p.pbytes;
            const unsigned off = bb ? zo + p.own : zs + p.colo[d];
            if (!p.ok_load(off)) return 0;
            return Codec<T>::template ld<I>(b, off, p.template add_pull<I>());
        }
        if (!p.ok_load(zs + p.colo[d]) || !p.ok_load(zo + p.own)) return 0;
        typename RealOf<T>::type v =
            Codec<T>::template ld<I>(p.base + here * p.pbytes, zs + p.colo[d], p.template add_pull<I>());
        if constexpr (d != 4) {
            if (p.wall & (1u << d))
                v = Codec<T>::template ld<OPP(I)>(p.base + OPP(here) * p.pbytes, zo + p.own, p.template add_pull<I>());
        }
        return v;
    }
}

// Interpolated wall, Eqs. (fbc1)/(fbc2): a wall link's value becomes
// c g*_opp(i)(x) + (1 - c) X (g*_opp(i)(x) is what the pull above read),
// with the column's coefficient cf = +-c: cf > 0 (Delta >= 1/2, c =
// 1/(2 Delta)): X = g*_i(x); cf < 0 (Delta < 1/2 and x + c_i fluid, c =
// 2 Delta): X = g*_opp(i)(x + c_i); cf = 1: bounce-back (also stored for
// fluid slots, where it leaves the value unchanged).  Deviations g = f - w
// combine like f: the weights sum to 1 and w_i = w_opp(i).  The X loads of
// a node are issued in groups (one c_z each), then decoded and combined, so
// a wave with wall columns waits once per group: the stored words are
// loaded under the lane's condition and decoded outside it (a decode
// inside the condition would wait for its own load).
template <typename T, int FORM, int ZC, int I = 0>
__device__ __forceinline__ void wall_loads(const Pull<T, true> &p, const typename RealOf<T>::type (&cf)[9],
                                           unsigned zo, unsigned zmo, unsigned zpo, typename Codec<T>::Raw (&x)[27])
{
    constexpr int cx = CX(I), cy = CY(I), cz = CZ(I);
    constexpr int d = NSLOT(-cx, -cy);
    if constexpr (d != 4 && cz == ZC) {
        constexpr int here = FORM == FORM_W ? OPP(I) : I;
        // only the lanes with a cut link load (fluid slots keep the zero
        // word: they combine with c = 1, which leaves the value as it is)
        x[I] = 0;
        if (p.wall & (1u << d)) {
            const bool own_mode = cf[d] > 0;
            const unsigned zf = cz == 0 ? zo : (cz > 0 ? zpo : zmo);
            const unsigned off = own_mode ? zo + p.own : zf + p.colo[8 - d];
            // own mode: population I at this column; far mode: population
            // opp(I) at the neighbour x + c_I, the column opp(I) pulls from
            if (p.ok_load(off)) x[I] = Codec<T>::raw(p.base + (own_mode ? here : OPP(here)) * p.pbytes, off);
        }
    }
    if constexpr (I + 1 < 27) wall_loads<T, FORM, ZC, I + 1>(p, cf, zo, zmo, zpo, x);
}

template <typename T, int ZC, int I = 0>
__device__ __forceinline__ void wall_combine(const Pull<T, true> &p, const typename RealOf<T>::type (&cf)[9],
                                             const typename Codec<T>::Raw (&x)[27], typename RealOf<T>::type (&v)[27])
{
    using R = typename RealOf<T>::type;
    constexpr int d = NSLOT(-CX(I), -CY(I));
    if constexpr (d != 4 && CZ(I) == ZC) {
        // the producer of the X value: this column (own mode) or x + c_I
        const R add = cf[d] > R(0) ? p.template add_own<I>() : p.template add_pull<OPP(I)>();
        const R xi = Codec<T>::template dec<I>(x[I], add);
        const R c = cf[d] > R(0) ? cf[d] : -cf[d];
        v[I] = c * v[I] + (R(1) - c) * xi;
    }
    if constexpr (I + 1 < 27) wall_combine<T, ZC, I + 1>(p, cf, x, v);
}

// WALL: interpolated wall (coefficients at p.bc); else halfway bounce-back
template <typename T, int FORM = FORM_S, bool WALL = false, int I = 0>
__device__ __forceinline__ void gather(const Pull<T, WALL> &p, unsigned zo, unsigned zmo, unsigned zpo,
                                       typename RealOf<T>::type (&g)[27])
{
    g[I] = pull_one<T, I, FORM, WALL>(p, zo, zmo, zpo);
    if constexpr (I + 1 < 27) {
        gather<T, FORM, WALL, I + 1>(p, zo, zmo, zpo, g);
    } else if constexpr (WALL) {
        if (p.wall & 0x1efu) {  // a solid in-plane neighbour (slot 4 is the column itself)
            // coefficients (1 for fluid slots: the value stays), then the X
            // values in three groups of eight (c_z = -1, 0, +1)
            using R = typename RealOf<T>::type;
            R cf[9];
#pragma unroll
            for (int d = 0; d < 9; ++d) {
                const double c = p.bc[d * p.P];
                cf[d] = (p.wall & (1u << d)) ? R(c) : R(1);
            }
            typename Codec<T>::Raw x[27];
            wall_loads<T, FORM, -1>(p, cf, zo, zmo, zpo, x);
            wall_combine<T, -1>(p, cf, x, g);
            wall_loads<T, FORM, 0>(p, cf, zo, zmo, zpo, x);
            wall_combine<T, 0>(p, cf, x, g);
            wall_loads<T, FORM, 1>(p, cf, zo, zmo, zpo, x);
            wall_combine<T, 1>(p, cf, x, g);
        }
    }
}

// two-buffer store: g*_i(x) into slot i of node x of the other buffer (p:
// the thread's view of the source buffer, for its FP16 references)
template <typename T, bool WALL, int I = 0>
__device__ __forceinline__ void store_all(char *pipe, const Pull<T, WALL> &p, unsigned off,
                                          const typename RealOf<T>::type (&g)[27])
{
    if (p.ok_store(off)) Codec<T>::template st<I>(pipe + I * p.pbytes, off, g[I], p.template ref_own<I>());
    if constexpr (I + 1 < 27) store_all<T, WALL, I + 1>(pipe, p, off, g);
}

// AA pattern, even step: g*_i(x) into slot opp(i) of node x (in place), which
// leaves the buffer in FORM_W
template <typename T, int I = 0>
__device__ __forceinline__ void store_swapped(char *pipe, const Pull<T> &p, unsigned off,
                                              const typename RealOf<T>::type (&g)[27])
{
    if (p.ok_store(off)) Codec<T>::template st<I>(pipe + OPP(I) * p.pbytes, off, g[I], p.template ref_own<I>());
    if constexpr (I + 1 < 27) store_swapped<T, I + 1>(pipe, p, off, g);
}

// AA pattern, odd step: g*_i(x) into slot i of node x + c_i, or, where x + c_i
// is solid, into slot opp(i) of node x (the bounce-back arrives there as
// g_opp(i)(x, n+1)); leaves the buffer in FORM_N.  Each location is read and
// written by the one node that owns it, so the update is race-free in place.
template <typename T, int I = 0>
__device__ __forceinline__ void store_push(char *pipe, const Pull<T> &p, unsigned zo, unsigned zmo, unsigned zpo,
                                           const typename RealOf<T>::type (&g)[27])
{
    constexpr int cx = CX(I), cy = CY(I), cz = CZ(I);
    constexpr int d = NSLOT(cx, cy);
    const unsigned zt = cz == 0 ? zo : (cz > 0 ? zpo : zmo);
    if (d != 4 && (p.wall & (1u << d))) {
        if (p.ok_store(zo + p.own))
            Codec<T>::template st<I>(pipe + OPP(I) * p.pbytes, zo + p.own, g[I], p.template ref_own<I>());
    } else if (p.ok_store(zt + p.colo[d])) {
        Codec<T>::template st<I>(pipe + I * p.pbytes, zt + p.colo[d], g[I], p.template ref_own<I>());
    }
    if constexpr (I + 1 < 27) store_push<T, I + 1>(pipe, p, zo, zmo, zpo, g);
}

// ---------------------------------------------------------------- moments
template <typename R> struct Moments {
    R dr;           // rho - 1 = sum g_i
    R jx, jy, jz;   // sum c_i g_i (the weights carry no momentum)
    R m4, m5, m6;   // sum c_x c_y g, c_x c_z g, c_y c_z g
    R m7, m8;       // sum (c_x^2 - c_y^2) g, (c_x^2 - c_z^2) g
};

// Moments accumulated per in-plane group (c_x, c_y): with S = sum over c_z
// of g, Zs = g(+1) - g(-1) and T = g(+1) + g(-1), every needed raw moment is
// a signed sum of the group values.
template <typename R, int G = 0>
__device__ __forceinline__ void group_moments(const R (&g)[27], Moments<R> &m)
{
    constexpr int cx = G % 3 - 1, cy = G / 3 - 1;
    const R g0 = g[IDX(cx, cy, 0)], gp = g[IDX(cx, cy, 1)], gm = g[IDX(cx, cy, -1)];
    const R T = gp + gm, S = g0 + T, Zs = gp - gm;
    m.dr += S;
    m.jz += Zs;
    if constexpr (cx == 1) { m.jx += S; m.m5 += Zs; }
    if constexpr (cx == -1) { m.jx -= S; m.m5 -= Zs; }
    if constexpr (cy == 1) { m.jy += S; m.m6 += Zs; }
    if constexpr (cy == -1) { m.jy -= S; m.m6 -= Zs; }
    if constexpr (cx * cy == 1) m.m4 += S;
    if constexpr (cx * cy == -1) m.m4 -= S;
    if constexpr (cx != 0 && cy == 0) m.m7 += S;
    if constexpr (cx == 0 && cy != 0) m.m7 -= S;
    if constexpr (cx != 0) m.m8 += S;
    m.m8 -= T;
    if constexpr (G + 1 < 9) group_moments<R, G + 1>(g, m);
}

template <typename R>
__device__ __forceinline__ Moments<R> moments_of(const R (&g)[27])
{
    Moments<R> m = {R(0), R(0), R(0), R(0), R(0), R(0), R(0), R(0), R(0)};
    group_moments<R>(g, m);
    return m;
}

// ---------------------------------------------------------------- collision
// Per-axis factors of the equilibrium.  On D3Q27 the sixth-order Hermite
// equilibrium is exactly f_i^eq = rho w_i prod_a (1 + d_{c_ia}(u_a)) with
// d_0(u) = -3u^2/2 and d_{+-1}(u) = +-3u + 3u^2; its u-derivative uses
// d'_0 = -3u and d'_{+-1} = +-3 + 6u.
template <typename R> struct Axis {
    R d0, dp, dm;   // d_0, d_+1, d_-1
    R q0, qp, qm;   // derivatives
};
template <typename R> __device__ __forceinline__ Axis<R> axis_factors(R u)
{
    const R u2 = u * u, u3 = R(3) * u;
    Axis<R> a;
    a.d0 = R(-1.5) * u2;
    a.dp = u3 + R(3) * u2;
    a.dm = -u3 + R(3) * u2;
    a.q0 = -u3;
    a.qp = R(3) + R(6) * u;
    a.qm = R(-3) + R(6) * u;
    return a;
}
template <int C, typename R> __device__ __forceinline__ R dsel(const Axis<R> &a) { return C == 0 ? a.d0 : (C > 0 ? a.dp : a.dm); }
template <int C, typename R> __device__ __forceinline__ R qsel(const Axis<R> &a) { return C == 0 ? a.q0 : (C > 0 ? a.qp : a.qm); }

// Collision kinds.  KIND_MRT6 is the paper's scheme: the multiple-relaxation-
// time collision of the appendix with the sixth-order Hermite equilibrium.
// The others are the comparison schemes: the same MRT collision with the
// second-order equilibrium of the LBM-O(2) scheme (Section III, Table I), and
// the single-relaxation-time BGK operator of Eq. (srt) (every population
// relaxed at omega) with either equilibrium.  All use Guo forcing in
// population form, F_i = a . grad_u f^eq_i.
enum CollisionKind : int { KIND_MRT6 = 0, KIND_MRT2 = 1, KIND_SRT6 = 2, KIND_SRT2 = 3 };
__host__ __device__ constexpr bool kind_srt(int kind) { return kind >= KIND_SRT6; }
__host__ __device__ constexpr bool kind_eq2(int kind) { return (kind & 1) != 0; }

template <typename R> struct CollideCtx {
    Axis<R> X, Y, Z;
    R dr, rho;      // rho - 1 and rho
    R ax, ay, az;   // body acceleration
    R ux, uy, uz;   // velocity u = j/rho + a/2
    R c4, c5, c6, c7, c8;   // (1 - omega) (m_k - m_k^eq + R_k/2), k = 4..8
    R omega;
};

// Relaxed non-equilibrium part of the stress moments, Eq. (m*) with
// Lam_k = omega for k = 4..8: m*_k - m^eq_k - R_k/2 = (1 - omega)(m_k - m^eq_k + R_k/2),
// using the printed m_4..8^eq and R_4..8 (the second-order equilibrium has
// the same second-order moments, so these hold for it too).
template <typename R>
__device__ __forceinline__ CollideCtx<R> collide_setup(const Moments<R> &m, R ax, R ay, R az, R omega, R &ux, R &uy,
                                                       R &uz)
{
    CollideCtx<R> c;
    c.dr = m.dr;
    c.rho = R(1) + m.dr;
    c.omega = omega;
    const R inv = rcp_r(c.rho);
    // Eq. (macroscopic_u): u = j/rho + a/2
    ux = m.jx * inv + R(0.5) * ax;
    uy = m.jy * inv + R(0.5) * ay;
    uz = m.jz * inv + R(0.5) * az;
    c.ux = ux;
    c.uy = uy;
    c.uz = uz;
    c.ax = ax;
    c.ay = ay;
    c.az = az;
    c.X = axis_factors(ux);
    c.Y = axis_factors(uy);
    c.Z = axis_factors(uz);
    const R r = c.rho, om1 = R(1) - omega, h = R(0.5);
    const R xx = ux * ux, yy = uy * uy, zz = uz * uz;
    c.c4 = om1 * (m.m4 - r * ux * uy + h * r * (ay * ux + ax * uy));
    c.c5 = om1 * (m.m5 - r * ux * uz + h * r * (az * ux + ax * uz));
    c.c6 = om1 * (m.m6 - r * uy * uz + h * r * (az * uy + ay * uz));
    c.c7 = om1 * (m.m7 - r * (xx - yy) + r * (ax * ux - ay * uy));
    c.c8 = om1 * (m.m8 - r * (xx - zz) + r * (ax * ux - az * uz));
    return c;
}

// Post-collision deviations, population by population:
//   g*_i = (f^eq_i - w_i) + F_i/2 + sum_k c_k d_k(i)
// f^eq_i - w_i = w_i (rho Pi_i - 1) = w_i (rho (Pi_i - 1) + (rho - 1)), with
// Pi_i - 1 = prod_a (1 + d_a) - 1 built without cancellation; F_i = a . grad_u
// f^eq_i (Guo forcing in population form, whose moments are the printed
// R^MRT); d_k = columns 4..8 of the inverse moment matrix (sparse: edge links
// for k = 4..6, face links for 7, 8).  The three populations of one in-plane
// group (c_x, c_y) share the x-y factors.
// Comparison schemes (KIND != KIND_MRT6): with the second-order equilibrium,
// Pi_i - 1 = 3 c.u + 9/2 (c.u)^2 - 3/2 u.u and F_i/(2 w_i) = rho/2 (3 (c - u).a
// + 9 (c.u)(c.a)); the BGK operator stores
//   g*_i = (1 - omega) g_i + omega (f^eq_i - w_i) + (1 - omega/2) F_i
// in place of the MRT sum (the same moments, every one relaxed at omega).
template <typename R, int KIND, bool SPLIT, int G = 0>
__device__ __forceinline__ void group_post_collision(const CollideCtx<R> &c, R hr, R f7, R f8, R f9, R usq15, R ua,
                                                     R (&g)[27])
{
    constexpr int cx = G % 3 - 1, cy = G / 3 - 1;
    const R dx = dsel<cx>(c.X), dy = dsel<cy>(c.Y);
    const R qx = qsel<cx>(c.X), qy = qsel<cy>(c.Y);
    const R exy = fma_r(dx, dy, dx + dy);   // (1+dx)(1+dy) - 1
    const R e1 = R(1) + exy;
    const R A = hr * fma_r(c.ax * qx, R(1) + dy, c.ay * qy * (R(1) + dx));
    const R Bz = hr * c.az * e1;
    // second-order equilibrium: in-plane parts of c.u and c.a
    const R s = R(cx) * c.ux + R(cy) * c.uy;
    const R sa = R(cx) * c.ax + R(cy) * c.ay;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        const int czr = t == 0 ? 0 : (t == 1 ? 1 : -1);
        R feq, fh;  // (rho Pi - 1) and F / (2 w)
        if constexpr (!kind_eq2(KIND)) {
            const R dz = czr == 0 ? c.Z.d0 : (czr > 0 ? c.Z.dp : c.Z.dm);
            const R qz = czr == 0 ? c.Z.q0 : (czr > 0 ? c.Z.qp : c.Z.qm);
            const R pim1 = fma_r(dz, e1, exy);
            feq = fma_r(pim1, c.rho, c.dr);
            fh = fma_r(qz, Bz, (R(1) + dz) * A);
        } else {
            const R cu = czr == 0 ? s : (czr > 0 ? s + c.uz : s - c.uz);
            const R ca = czr == 0 ? sa : (czr > 0 ? sa + c.az : sa - c.az);
            const R pim1 = fma_r(cu, fma_r(R(4.5), cu, R(3)), usq15);
            feq = fma_r(pim1, c.rho, c.dr);
            fh = hr * fma_r(R(9) * cu, ca, R(3) * (ca - ua));
        }
        const int i = t == 0 ? IDX(cx, cy, 0) : (t == 1 ? IDX(cx, cy, 1) : IDX(cx, cy, -1));
        if constexpr (kind_srt(KIND)) {
            const R om = c.omega;
            g[i] = weigh<R, SPLIT>(i, fma_r(om, feq, (R(2) - om) * fh), (R(1) - om) * g[i]);
        } else {
            R corr = R(0);
            const int shell = cx * cx + cy * cy + czr * czr;
            if (shell == 1) corr = cx != 0 ? f7 : (cy != 0 ? f8 : f9);
            if (shell == 2) {
                if (czr == 0) corr = (cx * cy > 0 ? R(0.25) : R(-0.25)) * c.c4;
                else if (cy == 0) corr = (cx * czr > 0 ? R(0.25) : R(-0.25)) * c.c5;
                else corr = (cy * czr > 0 ? R(0.25) : R(-0.25)) * c.c6;
            }
            g[i] = weigh<R, SPLIT>(i, feq + fh, corr);
        }
    }
    if constexpr (G + 1 < 9) group_post_collision<R, KIND, SPLIT, G + 1>(c, hr, f7, f8, f9, usq15, ua, g);
}

// SPLIT: the weights as hi + lo parts (see weigh)
template <typename R, int KIND = KIND_MRT6, bool SPLIT = true>
__device__ __forceinline__ void post_collision_all(const CollideCtx<R> &c, R (&g)[27])
{
    // face-link combinations of the relaxed stress moments 7 and 8
    const R f7 = (c.c7 + c.c8) * (R(1) / R(6));                   // +-x faces
    const R f8 = c.c8 * (R(1) / R(6)) - c.c7 * (R(1) / R(3));      // +-y faces
    const R f9 = c.c7 * (R(1) / R(6)) - c.c8 * (R(1) / R(3));      // +-z faces
    // second-order equilibrium: -3/2 u.u and u.a
    const R usq15 = R(-1.5) * (c.ux * c.ux + c.uy * c.uy + c.uz * c.uz);
    const R ua = c.ux * c.ax + c.uy * c.ay + c.uz * c.az;
    group_post_collision<R, KIND, SPLIT>(c, R(0.5) * c.rho, f7, f8, f9, usq15, ua, g);
}

// Equilibrium deviation f^eq_I(rho = 1 + dr, u) - w_I (used by the initialiser)
template <int I, typename R>
__device__ __forceinline__ R feq_dev(R dr, const Axis<R> &X, const Axis<R> &Y, const Axis<R> &Z)
{
    const R dx = dsel<CX(I)>(X), dy = dsel<CY(I)>(Y), dz = dsel<CZ(I)>(Z);
    const R exy = dx + dy + dx * dy;
    const R pim1 = exy + dz * (R(1) + exy);
    return wgt<R>(I) * (dr * (R(1) + pim1) + pim1);
}
// the same for the second-order equilibrium at rho = 1 and u = (0, 0, uz)
template <int I, typename R> __device__ __forceinline__ R feq2_dev_z(R uz)
{
    const R cu = R(CZ(I)) * uz;
    return wgt<R>(I) * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * uz * uz);
}

// ---------------------------------------------------------------- forcing
// Force inputs in the arithmetic type R: FP32 tables for FP32 and FP16
// storage, the FP64 copies for FP64 storage (which computes in FP64
// throughout, omega and h included).
// time factor sigma(n) = sin(2 pi n / T) of the trigger force, 0 once it is off
template <typename R = float>
__device__ __forceinline__ R sigma_of(const Geom &g, long long n)
{
    if constexpr (sizeof(R) == 8)
        return (n >= 0 && n < g.n_sigma) ? g.sigma64[n] : 0.0;
    else
        return (n >= 0 && n < g.n_sigma) ? g.sigma[n] : 0.f;
}
// trigger shape sums (P_x, P_y, Q) of column k of pipe b
template <typename R> struct Shape {
    R px, py, pq;
};
template <typename R = float>
__device__ __forceinline__ Shape<R> shape_of(const Geom &g, int b, int k)
{
    if constexpr (sizeof(R) == 8) {
        const double *fs = g.fshape64 + (size_t)b * 3 * g.P;
        return Shape<R>{fs[k], fs[g.P + k], fs[2 * g.P + k]};
    } else {
        const float *fs = g.fshape + (size_t)b * 3 * g.P;
        return Shape<R>{fs[k], fs[g.P + k], fs[2 * g.P + k]};
    }
}
template <typename R> __device__ __forceinline__ R omega_of(const Geom &g)
{
    if constexpr (sizeof(R) == 8)
        return g.omega64;
    else
        return g.omega;
}

__device__ __forceinline__ int wrap_m(int z, int nz) { return z == 0 ? nz - 1 : z - 1; }
__device__ __forceinline__ int wrap_p(int z, int nz) { return z == nz - 1 ? 0 : z + 1; }

// body acceleration a(x, n) = h z^ + sigma(n) (C_z P_x, C_z P_y, S_z Q)
template <typename R>
__device__ __forceinline__ void body_force(const Geom &g, int z, R sig, R px, R py, R pq, R &ax, R &ay, R &az)
{
    if constexpr (sizeof(R) == 4) {
        const float cz = g.ztab[z], sz = g.ztab[g.nz + z];
        ax = sig * cz * px;
        ay = sig * cz * py;
        az = g.accel_z + sig * sz * pq;
    } else {
        const double cz = g.ztab64[z], sz = g.ztab64[g.nz + z];
        ax = sig * cz * px;
        ay = sig * cz * py;
        az = g.accel_z64 + sig * sz * pq;
    }
}

// One node's collision at a(x, n): moments, equilibrium, forcing and the
// relaxation, in place on the gathered deviations v.
template <typename T, int KIND = KIND_MRT6>
__device__ __forceinline__ void collide(const Geom &g, typename RealOf<T>::type (&v)[27],
                                        typename RealOf<T>::type sig, const Shape<typename RealOf<T>::type> &sh, int z)
{
    using R = typename RealOf<T>::type;
    R ax, ay, az;
    body_force<R>(g, z, sig, sh.px, sh.py, sh.pq, ax, ay, az);
    const Moments<R> m = moments_of<R>(v);
    R ux, uy, uz;
    const CollideCtx<R> c = collide_setup<R>(m, ax, ay, az, omega_of<R>(g), ux, uy, uz);
    post_collision_all<R, KIND, sizeof(T) != 2>(c, v);
}

// Workgroup -> tile.  Workgroups are dispatched round-robin over the 8 XCDs
// (workgroup w runs on XCD w % 8), each with its own L2.  remap == 0:
// dispatch order (neighbouring tiles on different XCDs); remap == 1: XCD x
// takes the x-th eighth of the tiles; remap = G >= 2: XCD x takes every
// eighth chunk of G consecutive tiles, so neighbouring tiles, which share
// the partial lines of the shifted pull reads, stay in one L2 while the XCDs
// still sweep the buffers together.  Tiles past the last whole round of 8
// chunks keep dispatch order.
__device__ __forceinline__ int xcd_tile(int bid, int nblocks, int remap)
{
    if (!remap) return bid;
    const int x = bid & 7, s = bid >> 3;
    if (remap == 1) {
        const int q = nblocks >> 3, r = nblocks & 7;
        return x * q + (x < r ? x : r) + s;
    }
    const int full = nblocks / (8 * remap) * (8 * remap);
    if (bid >= full) return bid;
    return ((s / remap) * 8 + x) * remap + s % remap;
}

}  // namespace lbm
