// lbm_step.h -- one tile of one time step (pull gather with the wall,
// collision at a(x, n), store of the two-buffer or AA pattern), shared by the
// step kernels of the paper's collision (lbm_kernels.hip) and of the
// comparison schemes (lbm_variants.hip).
#pragma once

#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

// ---------------------------------------------------------------- helpers
struct TileCoord {
    int b, zc, k, kb;
};
__device__ __forceinline__ TileCoord tile_coord(const Tiles &t, int tile, int block)
{
    TileCoord c;
    c.kb = tile % t.nkb;
    const int rest = tile / t.nkb;
    c.zc = rest % t.nzc;
    c.b = rest / t.nzc + t.b0;
    c.k = c.kb * block + threadIdx.x;
    return c;
}
__device__ __forceinline__ TileCoord decode_tile(const Tiles &t, int block)
{
    return tile_coord(t, xcd_tile(blockIdx.x, gridDim.x, t.xcd), block);
}

__device__ __forceinline__ void load_columns(const Geom &g, int k, int (&col)[9])
{
#pragma unroll
    for (int d = 0; d < 9; ++d) col[d] = g.nbr[d * g.P + k];
}


// ---------------------------------------------------------------- step
// LBM_WAVES_PER_EU (compile time) asks the compiler for a register budget
// allowing that many waves per SIMD.
#ifndef LBM_WAVES_PER_EU
#define LBM_WAVES_PER_EU 0
#endif
#if LBM_WAVES_PER_EU > 0
#define LBM_OCCUPANCY __attribute__((amdgpu_waves_per_eu(LBM_WAVES_PER_EU)))
#else
#define LBM_OCCUPANCY
#endif

// Step variants: the two-buffer pattern (read FORM_S from src, aligned store
// into dst) and the in-place AA pattern (even n: read own slots, store
// swapped -> FORM_W; odd n: gather FORM_W, push to the neighbours -> FORM_N).
enum StepMode : int { STEP_AB = 0, STEP_AA_EVEN = 1, STEP_AA_ODD = 2 };

// One tile of one time step (column k of the tile, its z planes): gather of
// g(n) (streaming + bounce-back), collision at a(x, n), store of g*(n).
// For the AA modes src and dst are the same buffer.
// lref: FP16 storage, this thread's 27 floats of LDS for its column references
// REC: also record the moments (rho - 1, j_x, j_y, j_z) of the gathered
// state g(n) into rec[b][q][z P + k] (q = 0..3, each q a region of one
// population stride), in the collision's arithmetic type: the discrete
// adjoint needs the forward state only through them
template <typename T, int MODE, bool WALL = false, int KIND = KIND_MRT6, bool REC = false>
__device__ __forceinline__ void step_tile(const Geom &g, const Tiles &t, const TileCoord &tc, const T *src, T *dst,
                                          long long n, float *lref = nullptr,
                                          typename RealOf<T>::type *rec = nullptr)
{
    const int k = tc.k;
    Pull<T, WALL> p =
        make_pull<T, WALL>(src + (size_t)tc.b * g.pipe, (size_t)g.pstride, g.nbr, g.P, k, g.bcoef, g.href, lref,
                           g.check);
    using R = typename RealOf<T>::type;
    const Shape<R> sh = shape_of<R>(g, tc.b, k);
    const R sig = sigma_of<R>(g, n);
    char *pout = reinterpret_cast<char *>(dst + (size_t)tc.b * g.pipe);
    const unsigned rowb = (unsigned)g.P * sizeof(T);
    const int z0 = tc.zc * t.zchunk;
    const int z1 = min(z0 + t.zchunk, g.nz);
    constexpr int FORM = MODE == STEP_AB ? FORM_S : (MODE == STEP_AA_EVEN ? FORM_N : FORM_W);
    for (int z = z0; z < z1; ++z) {
        const unsigned zo = (unsigned)z * rowb;
        const unsigned zmo = (unsigned)wrap_m(z, g.nz) * rowb, zpo = (unsigned)wrap_p(z, g.nz) * rowb;
        typename RealOf<T>::type v[27];
        pull_opaque<WALL || MODE == STEP_AA_ODD>(p);  // FP16 (see there)
        gather<T, FORM, WALL>(p, zo, zmo, zpo, v);
        if constexpr (REC) {
            const Moments<typename RealOf<T>::type> m = moments_of(v);
            if (p.ok_store(zo + p.own)) {
                const size_t e = (size_t)tc.b * 4 * g.pstride + (size_t)z * g.P + k;
                __builtin_nontemporal_store(m.dr, rec + e);
                __builtin_nontemporal_store(m.jx, rec + e + g.pstride);
                __builtin_nontemporal_store(m.jy, rec + e + 2 * (size_t)g.pstride);
                __builtin_nontemporal_store(m.jz, rec + e + 3 * (size_t)g.pstride);
            }
        }
        collide<T, KIND>(g, v, sig, sh, z);
        if constexpr (MODE == STEP_AB)
            store_all<T>(pout, p, zo + p.own, v);
        else if constexpr (MODE == STEP_AA_EVEN)
            store_swapped<T>(pout, p, zo + p.own, v);
        else
            store_push<T>(pout, p, zo, zmo, zpo, v);
    }
}

}  // namespace lbm
