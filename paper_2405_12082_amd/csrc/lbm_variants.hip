// lbm_variants.hip -- step kernels of the comparison schemes: the MRT
// collision with the second-order equilibrium of the LBM-O(2) scheme the
// paper compares with (Section III, Table I), and the single-relaxation-time
// BGK operator of Eq. (srt) with the sixth- or second-order equilibrium.
// Same gather, wall, forcing and stores as the paper's scheme (lbm_step.h);
// only the per-node collision differs (CollisionKind in lbm_device.h).  Two
// buffers, FP32 or FP64 storage, either wall.  In a translation unit of its
// own so that the build compiles it beside the main kernels.
#include "lbm_device.h"
#include "lbm_internal.h"
#include "lbm_step.h"

namespace lbm {

template <typename T, int BLOCK, bool WALL, int KIND>
__global__ __launch_bounds__(BLOCK) LBM_OCCUPANCY __attribute__((amdgpu_waves_per_eu(WALL && sizeof(T) == 4 ? 4 : 1)))
void k_step_kind(const Geom g, const Tiles t, const T *__restrict__ src, T *__restrict__ dst, int step_off)
{
    const TileCoord tc = decode_tile(t, BLOCK);
    if (tc.k >= g.ncol) return;
    step_tile<T, STEP_AB, WALL, KIND>(g, t, tc, src, dst, *g.step_dev + step_off);
}

template <typename T, bool WALL, int KIND>
static hipError_t step_kind_block(const Geom &g, const Tiles &t, const void *src, void *dst, int off, hipStream_t s)
{
    const dim3 grid((unsigned)(t.count() * t.nb));
    const T *a = (const T *)src;
    T *b = (T *)dst;
    switch (t.block) {
    case 64: hipLaunchKernelGGL((k_step_kind<T, 64, WALL, KIND>), grid, dim3(64), 0, s, g, t, a, b, off); break;
    case 128: hipLaunchKernelGGL((k_step_kind<T, 128, WALL, KIND>), grid, dim3(128), 0, s, g, t, a, b, off); break;
    case 512: hipLaunchKernelGGL((k_step_kind<T, 512, WALL, KIND>), grid, dim3(512), 0, s, g, t, a, b, off); break;
    default: hipLaunchKernelGGL((k_step_kind<T, 256, WALL, KIND>), grid, dim3(256), 0, s, g, t, a, b, off); break;
    }
    return hipGetLastError();
}

template <typename T, bool WALL>
static hipError_t step_kind_wall(const Geom &g, const Tiles &t, const void *src, void *dst, int off, hipStream_t s)
{
    switch (g.kind) {
    case KIND_MRT2: return step_kind_block<T, WALL, KIND_MRT2>(g, t, src, dst, off, s);
    case KIND_SRT6: return step_kind_block<T, WALL, KIND_SRT6>(g, t, src, dst, off, s);
    case KIND_SRT2: return step_kind_block<T, WALL, KIND_SRT2>(g, t, src, dst, off, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t step_kind_t(const Geom &g, const Tiles &t, const void *src, void *dst, int off, hipStream_t s)
{
    return g.bcoef ? step_kind_wall<T, true>(g, t, src, dst, off, s) : step_kind_wall<T, false>(g, t, src, dst, off, s);
}

hipError_t launch_step_kind(int storage, const Geom &g, const Tiles &t, const void *src, void *dst, int off,
                            hipStream_t s)
{
    if (storage == 0) return step_kind_t<float>(g, t, src, dst, off, s);
    if (storage == 2) return step_kind_t<double>(g, t, src, dst, off, s);
    return hipErrorInvalidValue;  // FP16 storage is not offered for the comparison schemes
}

}  // namespace lbm
