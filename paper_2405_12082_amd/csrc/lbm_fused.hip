// lbm_fused.hip -- two time steps of the D3Q27 MRT pipe stepper per launch
// (temporal blocking along the pipe axis) for gfx950.
//
// The single-step kernel moves every population through HBM once per step
// (216 B per fluid-node update in FP32).  Here a workgroup owns a 14 x 14
// tile of columns and a range of planes, and marches along z: for each
// plane it first runs step n (pull from HBM, collision; arXiv:2405.12082,
// Eqs. (collision), (streaming), (fbc1) at Delta = 1/2) on the tile and a
// ring of halo columns around it (a 16 x 16 box, one thread per box column),
// keeps those post-collision values in LDS, then runs step n+1 one plane
// behind, pulling from LDS, and stores only its result: one read and one
// write of the state per two updates.  The halo columns and the two extra
// planes of each z-range are computed twice (by the neighbouring
// workgroups); the halo reads hit the caches when neighbouring tiles run
// together.  Each step is the same arithmetic as the single-step kernel
// (FP16 storage rounds the intermediate state through its codec), so the
// result equals two single steps.
//
// LDS holds, per box column, the populations the next step pulls from other
// columns (8 per c_z group; the 3 that stay in the column live in
// registers): c_z = +1 for the last three planes, c_z = 0 for two, c_z = -1
// for one; 48 x 4 B per column, 48 KiB per workgroup.
#include <climits>

#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

namespace {

constexpr int FB = FUSED_BOX, FBX = FUSED_BX;
constexpr int ROW_P = 0;    // c_z = +1: 3 planes x 8 rows
constexpr int ROW_0 = 24;   // c_z = 0: 2 planes x 8 rows
constexpr int ROW_M = 40;   // c_z = -1: 1 plane x 8 rows
constexpr int NROWS = 48;

// row of population i within its c_z group: its in-plane slot 0..8 without
// the column's own slot 4
__host__ __device__ constexpr int QSLOT(int i)
{
    return NSLOT(CX(i), CY(i)) < 4 ? NSLOT(CX(i), CY(i)) : NSLOT(CX(i), CY(i)) - 1;
}

// FP16 storage: the value the single-step path would read back after
// storing it (Codec<__half>::st then ::ld, with the column's reference)
template <typename T, int I = 0>
__device__ __forceinline__ void storage_round(const Pull<T> &p, typename RealOf<T>::type (&v)[27])
{
    if constexpr (sizeof(T) == 2) {
        v[I] = h_decode(h_encode(v[I], H_SCALE(I), p.template ref_own<I>()), H_INV_SCALE(I), p.template add_own<I>());
        if constexpr (I + 1 < 27) storage_round<T, I + 1>(p, v);
    }
}

// post-collision values of step n at this box column into the LDS rows of
// the current plane (p_cur, z_cur: row bases of the c_z = +1 and c_z = 0
// rings for it)
template <int I = 0>
__device__ __forceinline__ void put(float *lds, int s, int p_cur, int z_cur, const float (&v)[27])
{
    if constexpr (NSLOT(CX(I), CY(I)) != 4) {
        constexpr int q = QSLOT(I);
        const int row = CZ(I) > 0 ? p_cur + q : (CZ(I) == 0 ? z_cur + q : ROW_M + q);
        lds[row * FB + s] = v[I];
    }
    if constexpr (I + 1 < 27) put<I + 1>(lds, s, p_cur, z_cur, v);
}

struct Rings {
    int p_nb;    // c_z = +1 rows of the plane two iterations back (what c_z = +1 pulls read)
    int p_bb;    // c_z = +1 rows of the previous plane (bounce-back of c_z = -1 links)
    int z_prev;  // c_z = 0 rows of the previous plane
};

// Pull of step n+1 at plane z from the step-n values in LDS: population I
// comes from box slot s - (c_x, c_y) at plane z - c_z, or, where that column
// is solid, is the halfway bounce-back g*_opp(I) of this column at plane z.
// The three populations that stay in the column come from registers (rest:
// r0, +z: r5, -z: r6); the own -z ring values of plane z were saved in bb
// before the ring moved on.
template <int I = 0>
__device__ __forceinline__ void pull_lds(const float *lds, int s, unsigned wall, const Rings &r, const float (&bb)[8],
                                         float r0, float r5, float r6, float (&w)[27])
{
    constexpr int cx = CX(I), cy = CY(I), cz = CZ(I);
    constexpr int d = NSLOT(-cx, -cy);
    if constexpr (d == 4) {
        w[I] = I == 0 ? r0 : (I == 5 ? r5 : r6);
    } else {
        constexpr int q = QSLOT(I);
        constexpr int off = -(cy * FBX + cx);
        const int row = cz > 0 ? r.p_nb + q : (cz == 0 ? r.z_prev + q : ROW_M + q);
        float v = lds[row * FB + s + off];
        if (wall & (1u << d)) {
            constexpr int qo = QSLOT(OPP(I));
            if constexpr (cz > 0)
                v = bb[qo];
            else if constexpr (cz == 0)
                v = lds[(r.z_prev + qo) * FB + s];
            else
                v = lds[(r.p_bb + qo) * FB + s];
        }
        w[I] = v;
    }
    if constexpr (I + 1 < 27) pull_lds<I + 1>(lds, s, wall, r, bb, r0, r5, r6, w);
}

}  // namespace

// Steps n and n+1 for one tile, one range of output planes [z0, z1) and one
// pipe.  Iteration j runs step n at plane z0 - 1 + j (all box columns) and,
// from j = 2 on, step n+1 at plane z0 + j - 2 (the tile's own columns).
// Two barriers per iteration: before the ring slots are overwritten (the
// previous step-(n+1) reads are done) and before they are read.
template <typename T>
__global__ __launch_bounds__(FUSED_BOX) void k_step2(const Geom g, const Tiles2 t, const T *__restrict__ src,
                                                      T *__restrict__ dst, int step_off)
{
    __shared__ float lds[NROWS * FB];
    const int s = threadIdx.x;
    const int bid = xcd_tile(blockIdx.x, gridDim.x, t.xcd);
    const int tile = bid % t.nt;
    const int rest = bid / t.nt;
    const int zc = rest % t.nzc;
    const int b = rest / t.nzc + t.b0;
    const int code = t.box[(size_t)tile * FB + s];
    const bool valid = code >= 0;
    const bool owned = valid && (code & FUSED_OWNED);
    const int k = valid ? (code & ~FUSED_OWNED) : 0;
    __shared__ float lref[href_lds_floats<T, FUSED_BOX>()];
    Pull<T> p = make_pull<T>(src + (size_t)b * g.pipe, (size_t)g.pstride, g.nbr, g.P, k, nullptr, g.href,
                                   lref + 27 * threadIdx.x, g.check);
    const Shape<float> sh = shape_of<float>(g, b, k);
    const long long n = *g.step_dev + step_off;
    const float sig1 = sigma_of<float>(g, n), sig2 = sigma_of<float>(g, n + 1);
    char *pout = reinterpret_cast<char *>(dst + (size_t)b * g.pipe);
    const unsigned rowb = (unsigned)g.P * sizeof(T);
    const int z0 = zc * t.zchunk;
    const int iters = min(z0 + t.zchunk, g.nz) - z0 + 2;
    int zs = wrap_m(z0, g.nz);
    float r0_0 = 0.f, r0_1 = 0.f, r5_0 = 0.f, r5_1 = 0.f, r5_2 = 0.f, r6_0 = 0.f;
    float bb[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) bb[q] = 0.f;
    int j3 = 0;  // j mod 3
    for (int j = 0; j < iters; ++j) {
        float v[27];
        if (valid) {
            const unsigned zo = (unsigned)zs * rowb;
            const unsigned zmo = (unsigned)wrap_m(zs, g.nz) * rowb, zpo = (unsigned)wrap_p(zs, g.nz) * rowb;
            pull_opaque<true>(p);
            gather<T, FORM_S, false>(p, zo, zmo, zpo, v);
            collide<T>(g, v, sig1, sh, zs);
            storage_round<T>(p, v);
        }
        __syncthreads();
        if (valid) {
            if (p.wall) {
#pragma unroll
                for (int q = 0; q < 8; ++q) bb[q] = lds[(ROW_M + q) * FB + s];
            }
            put(lds, s, ROW_P + 8 * j3, ROW_0 + 8 * (j & 1), v);
            r5_2 = r5_1;
            r5_1 = r5_0;
            r5_0 = v[5];
            r0_1 = r0_0;
            r0_0 = v[0];
            r6_0 = v[6];
        }
        __syncthreads();
        if (j >= 2 && owned) {
            const int zq = wrap_m(zs, g.nz);
            const Rings r{ROW_P + 8 * (j3 == 2 ? 0 : j3 + 1), ROW_P + 8 * (j3 == 0 ? 2 : j3 - 1),
                          ROW_0 + 8 * ((j + 1) & 1)};
            float w[27];
            pull_lds(lds, s, p.wall, r, bb, r0_1, r5_2, r6_0, w);
            collide<T>(g, w, sig2, sh, zq);
            store_all<T>(pout, p, (unsigned)zq * rowb + p.own, w);
        }
        zs = wrap_p(zs, g.nz);
        j3 = j3 == 2 ? 0 : j3 + 1;
    }
}

hipError_t launch_step2(int storage, const Geom &g, const Tiles2 &t, const void *src, void *dst, int step_off,
                        hipStream_t s)
{
    const long long blocks = t.count() * t.nb;
    if (blocks <= 0) return hipSuccess;
    if (blocks > INT_MAX) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)blocks), block(FUSED_BOX);
    if (storage == 0)
        hipLaunchKernelGGL(k_step2<float>, grid, block, 0, s, g, t, (const float *)src, (float *)dst, step_off);
    else if (storage == 1)
        hipLaunchKernelGGL(k_step2<__half>, grid, block, 0, s, g, t, (const __half *)src, (__half *)dst, step_off);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace lbm
